// Block-length autotuner: for each (precision, order bucket, length bucket)
// it times the per-iteration LSQR pass at every admissible FFT block length
// on synthetic data and keeps the fastest in the context's table, which
// make_plan consults when the options leave the length automatic.  Mixed
// precision: a class's block length is fixed before each fit's path (FP32-
// or FP64-product LSQR) is known; the table is taken from the FP64-product
// pass, the costlier of the two (on a batch of AR(2..64) series that choice
// beat the sum of both passes' times by 6%).
#include <algorithm>

#include "engine.h"

namespace {

constexpr int TUNE_LG_MAX_M = 26;  // longest synthetic series measured (2^26 rows)
constexpr int TUNE_REPS = 5;

struct TuneBufs {
  double* y;
  void* spec;
  void* u0;
  void* u1;
  void* Vhat;
  double* partial;
  double* g;
};

size_t tune_carve(int64_t m, int p, int lg, TuneBufs* t, char* base) {
  Arena a;
  a.base = base;
  const size_t es = sizeof(double);
  const int B = 1 << lg, L = B - p + 1;
  const int64_t nb = (m + L - 1) / L;
  t->y = a.take<double>(static_cast<size_t>(m + p));
  t->spec = a.take<char>(static_cast<size_t>(nb) * (B / 2) * 2 * es);
  t->u0 = a.take<char>(static_cast<size_t>(m) * es);
  t->u1 = a.take<char>(static_cast<size_t>(m) * es);
  t->Vhat = a.take<char>(static_cast<size_t>(B / 2) * 2 * es);
  t->partial = a.take<double>(static_cast<size_t>(p + 1) * nb);
  t->g = a.take<double>(static_cast<size_t>(p + 1));
  return a.need;
}

// Median device time (ms) of one FP64 pass + column sums at block length 2^lg.
tls_status time_pass(tls_ctx* ctx, int64_t m, int p, int lg, hipEvent_t e0, hipEvent_t e1,
                     double* ms) {
  const int prec = PREC_F64;
  hipStream_t s = ctx->stream;
  TuneBufs t{};
  const size_t need = tune_carve(m, p, lg, &t, nullptr);
  TLS_CHECK(ensure_ws(ctx, need + 256));
  tune_carve(m, p, lg, &t, static_cast<char*>(ctx->ws));
  const int B = 1 << lg, lgn = lg - 1, L = B - p + 1;
  const int nb = static_cast<int>((m + L - 1) / L);
  // synthetic series: uniform draws (the pass's cost does not depend on them)
  TLS_CHECK(launch_philox_uniform(t.y, m + p, 0, 0, 0x7475'6e65ull, 0, s));
  TLS_CHECK(launch_spectra(prec, lgn, t.y, m + p, L, nb, t.spec, ctx->tw, s));
  TLS_CHECK(launch_small_rfft(prec, lgn, t.y, p, p, 1, 1.0 / B, t.Vhat, ctx->tw, nullptr, s));
  TLS_CHECK(hipMemcpyAsync(t.u0, t.y, m * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<float> times;
  for (int r = 0; r < TUNE_REPS + 1; ++r) {
    TLS_CHECK(hipEventRecord(e0, s));
    // the fused LSQR pass (e = X v - a u, X^T e)
    TLS_CHECK(launch_toep(prec, lgn, MODE_FUSED, t.spec, t.Vhat, t.u0, t.u1, nullptr, t.partial,
                          ctx->consts, nullptr, ctx->tw, m, p, L, nb, s));
    TLS_CHECK(launch_colsum(t.partial, pass_groups(lgn, nb), p + 1, t.g, nullptr, s));
    TLS_CHECK(hipEventRecord(e1, s));
    TLS_CHECK(hipEventSynchronize(e1));
    float x = 0.f;
    TLS_CHECK(hipEventElapsedTime(&x, e0, e1));
    if (r > 0) times.push_back(x);  // the first run warms caches and code
  }
  std::sort(times.begin(), times.end());
  *ms = times[times.size() / 2];
  return TLS_OK;
}

}  // namespace

tls_status tls_autotune(tls_ctx* ctx, int32_t precision, int32_t p_min, int32_t p_max,
                        int64_t n_min, int64_t n_max, int32_t* entries) {
  if (entries) *entries = 0;
  if (!ctx) return TLS_EINVAL;
  if (precision != TLS_PREC_F64 && precision != TLS_PREC_MIXED) return TLS_EINVAL;
  if (p_min < 1 || p_max < p_min || p_max > P_MAX) return TLS_EINVAL;
  if (n_min < 2 * static_cast<int64_t>(p_max) + 1 || n_max < n_min) return TLS_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return TLS_EDEVICE;
  const int ti = tune_prec(precision);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TLS_CHECK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return TLS_EDEVICE;
  }
  tls_status st = TLS_OK;
  int written = 0;
  const int mb_lo = tune_mbucket(n_min - p_max), mb_hi = tune_mbucket(n_max - p_min);
  for (int pb = tune_pbucket(p_min); pb <= tune_pbucket(p_max) && st == TLS_OK; ++pb) {
    const int p = std::min(1 << pb, P_MAX);
    int8_t top = 0;  // the result of the longest measured bucket
    for (int mb = mb_lo; mb <= mb_hi && st == TLS_OK; ++mb) {
      const int64_t m = int64_t{1} << std::min(mb, TUNE_LG_MAX_M);
      if (m < 2 * static_cast<int64_t>(p)) continue;
      if (mb > TUNE_LG_MAX_M && top > 0) {
        ctx->tune[ti][pb][mb] = top;
        ++written;
        continue;
      }
      int lg_lo = 7;
      while ((1 << lg_lo) < 2 * p) ++lg_lo;
      // no longer than the series: one block already holds every row
      int lg_hi = std::min(LG_BMAX, std::max(lg_lo, ilog2(m + p)));
      double best = 0.0;
      int best_lg = 0;
      for (int lg = lg_lo; lg <= lg_hi; ++lg) {
        double ms = 0.0;
        st = time_pass(ctx, m, p, lg, e0, e1, &ms);
        if (st != TLS_OK) break;
        if (best_lg == 0 || ms < best) {
          best = ms;
          best_lg = lg;
        }
      }
      if (st != TLS_OK) break;
      ctx->tune[ti][pb][mb] = static_cast<int8_t>(best_lg);
      top = static_cast<int8_t>(best_lg);
      ++written;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (entries) *entries = written;
  return st;
}

tls_status tls_get_tuning(const tls_ctx* ctx, int8_t* table) {
  if (!ctx || !table) return TLS_EINVAL;
  std::copy(&ctx->tune[0][0][0], &ctx->tune[0][0][0] + TLS_TUNE_ENTRIES, table);
  return TLS_OK;
}

tls_status tls_set_tuning(tls_ctx* ctx, const int8_t* table) {
  if (!ctx || !table) return TLS_EINVAL;
  for (int i = 0; i < TLS_TUNE_ENTRIES; ++i)
    if (table[i] != 0 && (table[i] < 7 || table[i] > LG_BMAX)) return TLS_EINVAL;
  std::copy(table, table + TLS_TUNE_ENTRIES, &ctx->tune[0][0][0]);
  return TLS_OK;
}
