// LSAR: the partial autocorrelations of one series at lags 1..pmax from
// compressed fits whose rows are drawn by approximate leverage scores that
// are carried from lag to lag (Section 3.1: the approximate leverage scores
// definition, eqs. (FALS), (FAR), (FASD), and Algorithm 3).
//
// Lag h fits AR(h) on the series prefix of n - pmax + h samples, so every
// lag has the same R = n - pmax rows, and row i of lag h is row i of lag
// h - 1 with lag h - 1's response in front of it.  The scores of lag h are
//   l_h(i) = l_{h-1}(i) + r_{h-1}(i)^2 / ||r_{h-1}||^2,  r_{h-1} = X_{h-1} phi_{h-1} - b_{h-1},
// over all R rows, starting from l_0 = 0 and r_0 = -b_0 (b_0[i] = y[i]), which
// makes l_1 the exact one-column scores y[i]^2 / sum y[t]^2.  Each lag draws c
// rows with replacement from pi_h = l_h / h, solves the compressed problem
// (eq. (OLSc)) on the rescaled rows, and reads tau_h off the last coefficient.
//
// Every residual comes from one FFT pass over block spectra computed once for
// the series: with blocks laid out for order pmax (L = B - pmax + 1 rows per
// block), X_h phi - b_h = X_pmax v for the pmax-vector v that holds phi at
// offsets d .. d + h - 1 and -1 at d - 1, d = pmax - h (lag h's lag columns
// are X_pmax's columns d .. pmax - 1 and its response is column d - 1).
#include "engine.h"

namespace {

// v = [0 .. 0, -1, phi_0 .. phi_{hm1-1}] of length pmax (-1 at pmax - hm1 - 1);
// also clears the factor status words of the lag about to be fitted.
__global__ void lsar_vec_kernel(const double* __restrict__ phi_prev, int hm1, int pmax,
                                double* __restrict__ v, int* __restrict__ st) {
  const int d = pmax - hm1;
  if (threadIdx.x == 0) st[0] = st[1] = 0;
  for (int j = threadIdx.x; j < pmax; j += blockDim.x)
    v[j] = j < d - 1 ? 0.0 : (j == d - 1 ? -1.0 : phi_prev[j - d]);
}

// eq. (FALS): l = (first ? 0 : l) + r^2 / ||r||^2 with ||r||^2 at *nrm2.
__global__ void lsar_update_kernel(const double* __restrict__ r, const double* __restrict__ nrm2,
                                   double* __restrict__ l, int64_t R, int first) {
  const double inv = 1.0 / *nrm2;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < R;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double ri = r[i];
    l[i] = first ? ri * ri * inv : fma(ri * ri, inv, l[i]);
  }
}

// Lag h's results: its coefficients (packed at h(h-1)/2), tau_h, its sampled
// rows (at (h-1) c) and its factor status words.
__global__ void lsar_record_kernel(const double* __restrict__ phi0, int h,
                                   double* __restrict__ phi_packed, double* __restrict__ tau,
                                   const int64_t* __restrict__ idx, int c,
                                   int64_t* __restrict__ rows, const int* __restrict__ st,
                                   int* __restrict__ lag_st) {
  const size_t off = static_cast<size_t>(h) * (h - 1) / 2;
  for (int j = threadIdx.x; j < h; j += blockDim.x) phi_packed[off + j] = phi0[j];
  for (int t = threadIdx.x; t < c; t += blockDim.x)
    rows[static_cast<size_t>(h - 1) * c + t] = idx[t];
  if (threadIdx.x == 0) {
    tau[h - 1] = phi0[h - 1];
    lag_st[2 * (h - 1)] = st[0];
    lag_st[2 * (h - 1) + 1] = st[1];
  }
}

struct LsarBufs {
  void* Yhat;
  double *e, *l, *partial, *g, *Vhat, *v, *swork, *scale, *A, *G, *R1, *R2, *Rm, *M, *Mt, *phi0;
  double *phi_packed, *tau;
  int64_t *idx, *rows;
  int *st, *lag_st;
};

size_t lsar_carve(const Plan& pl, int c, LsarBufs* b, char* base) {
  Arena a;
  a.base = base;
  const int pmax = pl.p, q = pmax + 1, ldq = (q + 15) / 16 * 16, crows = (c + 15) / 16 * 16;
  const size_t N = static_cast<size_t>(pl.B / 2);
  b->Yhat = a.take<char>(static_cast<size_t>(pl.nblocks) * N * 16);
  b->e = a.take<double>(pl.m);
  b->l = a.take<double>(pl.m);
  b->partial = a.take<double>(static_cast<size_t>(pmax + 1) * pl.ngroups);
  b->g = a.take<double>(pmax + 1);
  b->Vhat = a.take<double>(2 * N);
  b->v = a.take<double>(pmax);
  b->swork = a.take<double>(sample_work_doubles(pl.m));
  b->idx = a.take<int64_t>(c);
  b->scale = a.take<double>(c);
  b->A = a.take<double>(static_cast<size_t>(crows) * ldq);
  b->G = a.take<double>(qr_scratch_doubles(crows, q, ldq));
  b->R1 = a.take<double>(static_cast<size_t>(q) * q);
  b->R2 = a.take<double>(static_cast<size_t>(q) * q);
  b->Rm = a.take<double>(static_cast<size_t>(q) * q);
  b->M = a.take<double>(static_cast<size_t>(pmax) * pmax);
  b->Mt = a.take<double>(static_cast<size_t>(pmax) * pmax);
  b->phi0 = a.take<double>(pmax);
  b->phi_packed = a.take<double>(static_cast<size_t>(pmax) * (pmax + 1) / 2);
  b->tau = a.take<double>(pmax);
  b->rows = a.take<int64_t>(static_cast<size_t>(pmax) * c);
  b->st = a.take<int>(4);
  b->lag_st = a.take<int>(2 * static_cast<size_t>(pmax));
  return a.need;
}

}  // namespace

tls_status tls_lsar_device(tls_ctx* ctx, const double* d_series, int64_t n, int32_t pmax,
                           int32_t c, const tls_options* opt, void* stream, double* pacf,
                           int32_t* order, double* phi_packed, int64_t* rows,
                           tls_status* lag_status, double* d_scores) {
  if (!ctx || !d_series || !pacf || pmax < 1) return TLS_EINVAL;
  if (n < 2 * static_cast<int64_t>(pmax) + 1) return TLS_EINVAL;
  if (c < pmax + 1 || c > n - pmax) return TLS_EINVAL;
  if (pmax > P_MAX) return TLS_EUNSUPPORTED;
  hipSetDevice(ctx->device);
  const tls_options& o = opt ? *opt : ctx->opt;
  // the block geometry of order pmax serves every lag (see the file comment)
  Plan pl{};
  const tls_status sp = make_plan(n, pmax, o, &pl, ctx);
  if (sp != TLS_OK) return sp;
  const int64_t R = pl.m;
  hipStream_t s = pick_stream(ctx, stream);
  LsarBufs b{};
  TLS_CHECK(ensure_ws(ctx, lsar_carve(pl, c, &b, nullptr) + 256));
  lsar_carve(pl, c, &b, static_cast<char*>(ctx->ws));
  const uint64_t seed = o.seed;
  const uint32_t fit = static_cast<uint32_t>(o.request_id);
  const double invB = 1.0 / pl.B;
  const int crows = (c + 15) / 16 * 16;
  const int ugrid = static_cast<int>(std::min<int64_t>((R + 255) / 256, 4096));

  TLS_CHECK(launch_spectra(PREC_F64, pl.lgn, d_series, n, pl.L, pl.nblocks, b.Yhat, ctx->tw, s));
  for (int h = 1; h <= pmax; ++h) {
    // r_{h-1} = X_{h-1} phi_{h-1} - b_{h-1} over all R rows (eq. (FAR)), then eq. (FALS)
    const double* phi_prev = b.phi_packed + static_cast<size_t>(h - 1) * (h - 2) / 2;
    hipLaunchKernelGGL(lsar_vec_kernel, dim3(1), dim3(256), 0, s, phi_prev, h - 1, pmax, b.v,
                       b.st);
    TLS_CHECK(hipGetLastError());
    TLS_CHECK(launch_small_rfft(PREC_F64, pl.lgn, b.v, pmax, pmax, 1, invB, b.Vhat, ctx->tw,
                                nullptr, s));
    TLS_CHECK(launch_toep(PREC_F64, pl.lgn, MODE_MV, b.Yhat, b.Vhat, nullptr, b.e, nullptr,
                          b.partial, ctx->consts + 2, nullptr, ctx->tw, R, pmax, pl.L,
                          pl.nblocks, s));
    TLS_CHECK(launch_colsum(b.partial + static_cast<size_t>(pmax) * pl.ngroups, pl.ngroups, 1,
                            b.g + pmax, nullptr, s));
    hipLaunchKernelGGL(lsar_update_kernel, dim3(ugrid), dim3(256), 0, s, b.e, b.g + pmax, b.l, R,
                       h == 1 ? 1 : 0);
    TLS_CHECK(hipGetLastError());
    // c rows from pi_h = l_h / h (eq. (FASD)), Philox stream 3 draws (h-1) c ..
    TLS_CHECK(launch_sample(PREC_F64, b.l, R, nullptr, c, b.idx, b.scale, b.swork, seed, fit, s,
                            static_cast<uint64_t>(h - 1) * c));
    // the compressed problem of lag h (eq. (OLSc)): QR of [S X_h | S b_h]
    const int q = h + 1, ldq = (q + 15) / 16 * 16;
    TLS_CHECK(launch_gather(d_series, R, h, 0, b.idx, b.scale, c, crows, ldq, b.A, nullptr,
                            nullptr, seed, fit, s));
    TLS_CHECK(launch_qr(b.A, crows, q, ldq, h, 3, b.Rm, b.G, b.R1, b.R2, b.st, s));
    TLS_CHECK(launch_triinv(b.Rm, q, h, b.M, b.Mt, b.phi0, b.st + 1, s));
    hipLaunchKernelGGL(lsar_record_kernel, dim3(1), dim3(256), 0, s, b.phi0, h, b.phi_packed,
                       b.tau, b.idx, c, b.rows, b.st, b.lag_st);
    TLS_CHECK(hipGetLastError());
  }
  if (d_scores)
    TLS_CHECK(hipMemcpyAsync(d_scores, b.l, R * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<int> hst(2 * static_cast<size_t>(pmax));
  std::vector<double> hphi;
  TLS_CHECK(hipMemcpyAsync(pacf, b.tau, pmax * sizeof(double), hipMemcpyDeviceToHost, s));
  TLS_CHECK(hipMemcpyAsync(hst.data(), b.lag_st, hst.size() * sizeof(int), hipMemcpyDeviceToHost,
                           s));
  if (phi_packed)
    TLS_CHECK(hipMemcpyAsync(phi_packed, b.phi_packed,
                             static_cast<size_t>(pmax) * (pmax + 1) / 2 * sizeof(double),
                             hipMemcpyDeviceToHost, s));
  if (rows)
    TLS_CHECK(hipMemcpyAsync(rows, b.rows, static_cast<size_t>(pmax) * c * sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
  TLS_CHECK(hipStreamSynchronize(s));
  tls_status first = TLS_OK;
  int32_t best = 0;
  for (int h = 1; h <= pmax; ++h) {
    // rank deficiency of the compressed problem (a later CholeskyQR sweep
    // broke down, or a tiny pivot), or a non-finite estimate
    const int sq = hst[2 * (h - 1)], si = hst[2 * (h - 1) + 1];
    tls_status sh = (sq & 6) || (si & 4) || !isfinite(pacf[h - 1]) ? TLS_ERANK : TLS_OK;
    if (lag_status) lag_status[h - 1] = sh;
    if (sh != TLS_OK && first == TLS_OK) first = sh;
    if (sh == TLS_OK && fabs(pacf[h - 1]) >= 1.96 / sqrt(static_cast<double>(c))) best = h;
  }
  if (order) *order = best;
  return first;
}
