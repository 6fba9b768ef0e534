// Shared host-side pieces of the Toeplitz least-squares engine: the context,
// the device workspace arena, the per-fit plan and buffer carving, and the
// small set-up kernels used by the single-fit and the batched drivers.
#pragma once

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "../../include/tls.h"

using namespace tls;

// Streams on which a batched call runs its launch classes concurrently.
constexpr int BATCH_STREAMS = 4;

struct tls_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  tls_options opt{};
  void* tw64 = nullptr;
  void* tw32 = nullptr;
  Twiddles tw;
  double* consts = nullptr;  // {-1, 1, 1, 0}
  void* ws = nullptr;        // workspace
  size_t ws_bytes = 0;
  void* scratch = nullptr;   // this device's fixed scratch array (tls_op_toeplitz_noalloc)
  void* pinned = nullptr;    // host staging
  size_t pinned_bytes = 0;
  std::vector<hipEvent_t> events;  // profile = 1: pairs around each Toeplitz pass
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // ends of the LSQR chunks in flight
  // batched calls: one stream per concurrent launch class, its end event,
  // the event the class streams wait on, and profile = 1 event pools
  hipStream_t bstream[BATCH_STREAMS] = {};
  hipEvent_t bdone[BATCH_STREAMS] = {};
  hipEvent_t bready = nullptr;
  std::vector<hipEvent_t> bevents[BATCH_STREAMS];
  // autotuned log2 block lengths, [precision][order bucket][length bucket]; 0 = not tuned
  int8_t tune[TLS_TUNE_PRECS][TLS_TUNE_PBUCKETS][TLS_TUNE_MBUCKETS] = {};
};

struct Plan {
  int prec, B, lgn, L, nblocks, ngroups, p, q, ldq, c, crows, k, all_rows;
  int64_t n, m;
};

// Device buffers of one fit, carved from the workspace.
struct FitBufs {
  double* y;        // series copy (host input) or nullptr
  void* Yhat;       // spectra in compute precision
  void* Yhat64;     // FP64 spectra (mixed: residual passes)
  void* u;          // m-vector (also sketch scores)
  double* partial;  // (p+1) x ngroups (Toeplitz pass partials per block group)
  double* g;        // p+1
  double* A;        // crows x ldq
  double* G;        // ldq^2 + 2 q^2
  double *R1, *R2, *R;
  double *M, *Mt;
  double *Pi, *Om;
  void* Omhat;
  void* Vhat;
  double *v, *w, *z, *phi0, *phi;
  double* q;        // p: M v of the wide LSQR step
  double* phib;     // mixed: best refinement iterate
  int64_t* idx;
  double* scale;
  double* swork;
  LsqrState* st;
  int* status;      // [0] QR bits, [1] triinv bits
  double* dminmax;  // scratch
  double* rr;       // residual norm^2
  double* rpart;    // direct residual partials
  void* Vhat32;     // mixed: FP32 spectrum of the CG direction
  RefineState* rst; // mixed: refinement state
  double *cw, *cres, *cd;  // mixed: CG vectors
};

namespace {


constexpr int P_MAX = 1024;
constexpr int CHUNK_ITERS = 8;

#define TLS_CHECK(call)                          \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_status(e_); \
  } while (0)

tls_status hip_status(hipError_t e) {
  if (e == hipErrorOutOfMemory) return TLS_ENOMEM;
  if (e == hipErrorInvalidValue) return TLS_EUNSUPPORTED;
  return TLS_EDEVICE;
}

int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t{1} << l) < x) ++l;
  return l;
}

// Twiddle table: for L = 2, 4, ..., BMAX the factors exp(-2 pi i e / L),
// e < L/2, at indices L/2 - 1 + e (BMAX - 1 entries; the last word unused).
hipError_t build_twiddles(tls_ctx* c) {
  std::vector<cx<double>> t64(BMAX, cx<double>{0.0, 0.0});
  std::vector<cx<float>> t32(BMAX, cx<float>{0.f, 0.f});
  for (int lg = 1; lg <= LG_BMAX; ++lg) {
    const int half = 1 << (lg - 1);
    for (int e = 0; e < half; ++e) {
      const long double k = static_cast<long double>(e) * (BMAX >> lg);
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * k / BMAX;
      t64[half - 1 + e] = {static_cast<double>(cosl(a)), static_cast<double>(sinl(a))};
      t32[half - 1 + e] = {static_cast<float>(cosl(a)), static_cast<float>(sinl(a))};
    }
  }
  hipError_t e = hipMalloc(&c->tw64, BMAX * sizeof(cx<double>));
  if (e != hipSuccess) return e;
  e = hipMalloc(&c->tw32, BMAX * sizeof(cx<float>));
  if (e != hipSuccess) return e;
  e = hipMemcpy(c->tw64, t64.data(), BMAX * sizeof(cx<double>), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemcpy(c->tw32, t32.data(), BMAX * sizeof(cx<float>), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  c->tw.d64 = c->tw64;
  c->tw.d32 = c->tw32;
  const double k4[4] = {-1.0, 1.0, 1.0, 0.0};
  e = hipMalloc(&c->consts, sizeof(k4));
  if (e != hipSuccess) return e;
  return hipMemcpy(c->consts, k4, sizeof(k4), hipMemcpyHostToDevice);
}

// Bump allocator over the context workspace (256-byte aligned slices).
struct Arena {
  size_t need = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    const size_t off = (need + 255) & ~size_t{255};
    need = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

hipError_t ensure_ws(tls_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return hipSuccess;
  if (c->ws) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  const size_t grow = bytes + bytes / 8;
  hipError_t e = hipMalloc(&c->ws, grow);
  if (e != hipSuccess) return e;
  c->ws_bytes = grow;
  return hipSuccess;
}

hipError_t ensure_pinned(tls_ctx* c, size_t bytes) {
  if (bytes <= c->pinned_bytes) return hipSuccess;
  if (c->pinned) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
  }
  hipError_t e = hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  c->pinned_bytes = bytes;
  return hipSuccess;
}

// Event pair `i` (created on first use; kept for the context's lifetime).
// Event pair i of a pool (created on first use, kept for later calls).
hipError_t pool_events(std::vector<hipEvent_t>& pool, size_t i, hipEvent_t* a, hipEvent_t* b) {
  while (pool.size() < 2 * (i + 1)) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pool.push_back(e);
  }
  *a = pool[2 * i];
  *b = pool[2 * i + 1];
  return hipSuccess;
}

hipError_t pass_events(tls_ctx* c, size_t i, hipEvent_t* a, hipEvent_t* b) {
  return pool_events(c->events, i, a, b);
}

// The batched call's class streams and events (created on first use).
hipError_t ensure_batch_streams(tls_ctx* c) {
  if (c->bready) return hipSuccess;
  for (int w = 0; w < BATCH_STREAMS; ++w) {
    hipError_t e = hipStreamCreate(&c->bstream[w]);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->bdone[w], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  return hipEventCreateWithFlags(&c->bready, hipEventDisableTiming);
}

hipStream_t pick_stream(tls_ctx* c, void* s) {
  return s ? static_cast<hipStream_t>(s) : c->stream;
}

// ---------------------------------------------------------------------------

int auto_block(int p, int64_t m) {
  // Smallest power of two >= 8 p (>= 2p always), between 256 and 16384, and
  // no longer than the data needs: shorter blocks cost fewer FFT flops per
  // sample, longer ones re-read fewer overlapping samples.
  int lg = ilog2(8 * static_cast<int64_t>(p));
  if (lg < 8) lg = 8;
  const int lgdata = ilog2(m + p);
  if (lg > lgdata) lg = lgdata < 8 ? 8 : lgdata;
  if (lg > LG_BMAX) lg = LG_BMAX;
  while ((1 << lg) < 2 * p) ++lg;
  return lg;
}

// Repeated halving: the number of halvings of the m rows until a level holds
// no more than c rows (at least 1: one level is the plain leverage sketch).
int rh_levels(int64_t m, int c) {
  int l = 1;
  while ((m >> l) > c) ++l;
  return l;
}

// Buckets of the autotuner's table: order bucket ceil(log2 p), length bucket
// ceil(log2 m) (clamped to the table).
int tune_pbucket(int p) { return ilog2(p); }
int tune_mbucket(int64_t m) {
  const int b = ilog2(m);
  return b < TLS_TUNE_MBUCKETS ? b : TLS_TUNE_MBUCKETS - 1;
}
int tune_prec(int precision) { return precision == TLS_PREC_MIXED ? 1 : 0; }

// ctx: NULL, or the context whose autotuned table supplies the block length
// when the options leave it automatic.
tls_status make_plan(int64_t n, int p, const tls_options& o, Plan* pl,
                     const tls_ctx* ctx = nullptr) {
  pl->n = n;
  pl->p = p;
  pl->m = n - p;
  pl->prec = o.precision;
  int lg = o.block_lg;
  if (lg <= 0 && ctx) {
    lg = ctx->tune[tune_prec(o.precision)][tune_pbucket(p)][tune_mbucket(pl->m)];
    if (lg > 0 && (1 << lg) < 2 * p) lg = 0;
  }
  if (lg <= 0) lg = auto_block(p, pl->m);
  if (lg < 7 || lg > LG_BMAX) return TLS_EUNSUPPORTED;
  pl->B = 1 << lg;
  if (pl->B < 2 * p) return TLS_EUNSUPPORTED;
  pl->lgn = lg - 1;
  pl->L = pl->B - p + 1;
  pl->nblocks = static_cast<int>((pl->m + pl->L - 1) / pl->L);
  pl->ngroups = pass_groups(pl->lgn, pl->nblocks);
  pl->q = p + 1;
  pl->ldq = (pl->q + 15) / 16 * 16;
  const int64_t c = static_cast<int64_t>(o.gamma > 0 ? o.gamma : 8) * p;
  pl->all_rows = c >= pl->m ? 1 : 0;
  pl->c = static_cast<int>(pl->all_rows ? pl->m : c);
  pl->crows = (pl->c + 15) / 16 * 16;
  pl->k = o.jl_k > 0 ? o.jl_k : 8;
  return TLS_OK;
}

tls_status validate(int64_t n, int p, double tol, const tls_options& o) {
  if (p < 1 || n < 2 * static_cast<int64_t>(p) + 1) return TLS_EINVAL;
  if (!(tol > 0.0 && tol < 1.0)) return TLS_EINVAL;
  if (o.precision != TLS_PREC_F64 && o.precision != TLS_PREC_MIXED) return TLS_EINVAL;
  if (o.sketch != TLS_SKETCH_LEVERAGE && o.sketch != TLS_SKETCH_UNIFORM &&
      o.sketch != TLS_SKETCH_RH)
    return TLS_EINVAL;
  if (o.jl_kind != TLS_JL_SRHT && o.jl_kind != TLS_JL_GAUSS) return TLS_EINVAL;
  if (o.estimator != TLS_EST_OLS && o.estimator != TLS_EST_SKETCH) return TLS_EINVAL;
  if (p > P_MAX) return TLS_EUNSUPPORTED;
  if (n > (int64_t{1} << 40)) return TLS_EUNSUPPORTED;
  return TLS_OK;
}


size_t carve(const Plan& pl, bool copy_y, FitBufs* b, char* base) {
  Arena a;
  a.base = base;
  const size_t es = pl.prec == TLS_PREC_F64 ? sizeof(double) : sizeof(float);
  const size_t N = static_cast<size_t>(pl.B / 2);
  b->y = copy_y ? a.take<double>(pl.n) : nullptr;
  b->Yhat = a.take<char>(static_cast<size_t>(pl.nblocks) * N * 2 * es);
  b->Yhat64 = pl.prec == TLS_PREC_MIXED ? a.take<char>(static_cast<size_t>(pl.nblocks) * N * 16)
                                        : b->Yhat;
  b->u = a.take<char>(static_cast<size_t>(pl.m) * (pl.prec == TLS_PREC_F64 ? 8 : 8));
  b->partial = a.take<double>(static_cast<size_t>(pl.p + 1) * pl.ngroups);
  b->g = a.take<double>(pl.p + 1);
  b->A = a.take<double>(static_cast<size_t>(pl.crows) * pl.ldq);
  b->G = a.take<double>(qr_scratch_doubles(pl.crows, pl.q, pl.ldq));
  b->R1 = a.take<double>(static_cast<size_t>(pl.q) * pl.q);
  b->R2 = a.take<double>(static_cast<size_t>(pl.q) * pl.q);
  b->R = a.take<double>(static_cast<size_t>(pl.q) * pl.q);
  b->M = a.take<double>(static_cast<size_t>(pl.p) * pl.p);
  b->Mt = a.take<double>(static_cast<size_t>(pl.p) * pl.p);
  b->Pi = a.take<double>(static_cast<size_t>(pl.k) * pl.p);
  b->Om = a.take<double>(static_cast<size_t>(pl.k) * pl.p);
  b->Omhat = a.take<char>(static_cast<size_t>(pl.k) * N * 16);  // FP64 in every precision
  b->Vhat = a.take<char>(N * 16);
  b->v = a.take<double>(pl.p);
  b->w = a.take<double>(pl.p);
  b->z = a.take<double>(pl.p);
  b->phi0 = a.take<double>(pl.p);
  b->phi = a.take<double>(pl.p);
  b->q = a.take<double>(pl.p);
  b->phib = a.take<double>(pl.p);
  b->idx = a.take<int64_t>(pl.c);
  b->scale = a.take<double>(pl.c);
  b->swork = a.take<double>(sample_work_doubles(pl.m));
  b->st = a.take<LsqrState>(1);
  b->status = a.take<int>(4);
  b->dminmax = a.take<double>(4);
  b->rr = a.take<double>(4);
  b->rpart = a.take<double>(resid_direct_blocks(pl.m));
  b->Vhat32 = a.take<char>(N * 8);
  b->rst = a.take<RefineState>(1);
  b->cw = a.take<double>(pl.p);
  b->cres = a.take<double>(pl.p);
  b->cd = a.take<double>(pl.p);
  return a.need + 256;
}

__global__ void fill_state_kernel(LsqrState* st, double tol, int max_iter, int* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    LsqrState s{};
    s.tol = tol;
    s.max_iter = max_iter;
    s.coef[0] = -1.0;
    s.coef[1] = 1.0;
    *st = s;
    status[0] = status[1] = status[2] = status[3] = 0;
  }
}

__global__ void fill_refine_kernel(RefineState* st, double tol, int max_refine, int inner_max,
                                   double inner_tol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    RefineState s{};
    s.tol = tol;
    s.max_refine = max_refine;
    s.inner_max = inner_max;
    s.inner_tol = inner_tol;
    *st = s;
  }
}

// The results of a fit in one buffer of pinned host memory, written by this
// kernel (no copy launch): phi (p), ||r||^2, max and min |R_ii|, the four
// status words.
__global__ void pack_results_kernel(const double* __restrict__ phi, int p,
                                    const double* __restrict__ rr,
                                    const double* __restrict__ dminmax,
                                    const int* __restrict__ status, double* __restrict__ out) {
  for (int i = threadIdx.x; i < p; i += blockDim.x) out[i] = phi[i];
  if (threadIdx.x == 0) {
    out[p] = rr[0];
    out[p + 1] = dminmax[0];
    out[p + 2] = dminmax[1];
    for (int k = 0; k < 4; ++k) out[p + 3 + k] = static_cast<double>(status[k]);
  }
}

__global__ void copy_vec_kernel(const double* a, int n, double* b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void zero_kernel(double* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// dst[i] = float(src[i]), i < n (the response b in FP32 for FP32-product LSQR)
__global__ void to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = static_cast<float>(src[i]);
}

__global__ void set_tol_kernel(LsqrState* st, double tol) {
  if (threadIdx.x == 0) st->tol = tol;
}

// Mixed precision: the products' precision is chosen per fit from
// kappa_F = ||R||_F ||R^{-1}||_F of the sketch factor (R = R[:p,:p]; kappa_F >=
// kappa_2(R), about kappa(X), and at most p times it).  LSQR with FP32
// products and FP64 recurrences, run to max(tol, MIXED_TOL_F32) (the FP32
// products' resolution), leaves a coefficient error of at most about
// 0.5 kappa eps_32 (eps_32 = 6e-8; measured 0.01..0.5 kappa eps_32) against
// the FP64 solution: with kappa_F <= MIXED_KAPPA_F32 that is below 1e-5, a
// tenth of the mixed path's 1e-4.  Above it the fit runs FP64 LSQR (FP64
// refinement around FP32 inner solves instead, when max_refine > 0 and
// kappa_F <= MIXED_KAPPA_REFINE, where that refinement contracts).
constexpr double MIXED_KAPPA_F32 = 300.0;
constexpr double MIXED_KAPPA_REFINE = 1e8;
constexpr double MIXED_TOL_F32 = 1e-7;
enum MixedPath : int { MP_NONE = 0, MP_F32 = 1, MP_REFINE = 2, MP_F64 = 3 };

__host__ __device__ inline int mixed_path_of(double kappa_f, int max_refine) {
  if (kappa_f <= MIXED_KAPPA_F32) return MP_F32;
  if (max_refine > 0 && kappa_f <= MIXED_KAPPA_REFINE) return MP_REFINE;
  return MP_F64;
}

// ||R[:p,:p]||_F * ||M||_F for the upper-triangular R (q x q, row-major) and
// M = R[:p,:p]^{-1} (p x p, row-major): one workgroup of NT threads, sums in a
// fixed order (block_sum), the same in single and batched fits.
template <int NT>
__device__ __forceinline__ double kappa_f_body(const double* __restrict__ R, int q,
                                               const double* __restrict__ M, int p,
                                               double* red) {
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < p * p; k += NT) {
    const int i = k / p, j = k - i * p;
    if (j >= i) {
      const double r = R[static_cast<size_t>(i) * q + j];
      const double m = M[static_cast<size_t>(i) * p + j];
      a = fma(r, r, a);
      b = fma(m, m, b);
    }
  }
  a = block_sum<NT>(a, red);
  b = block_sum<NT>(b, red);
  return sqrt(a) * sqrt(b);
}

__global__ __launch_bounds__(256) void kappa_f_kernel(const double* __restrict__ R, int q,
                                                      const double* __restrict__ M, int p,
                                                      double* __restrict__ out) {
  __shared__ double red[4];
  const double k = kappa_f_body<256>(R, q, M, p, red);
  if (threadIdx.x == 0) *out = k;
}

// Mixed precision: each fit's path from kappa_F of its sketch factor (as the
// single-fit driver).  FP32-product LSQR: tolerance max(tol, tol32), no
// refinement.  The others skip the FP32 LSQR (marked done and counted in
// counts[0]); refinement fits are counted in counts[1]; FP64-LSQR fits skip
// the refinement and are set up for the FP64 finish from phi0.
// phases = 0 (no refinement): only the products' precision and the FP32
// tolerance are set, the FP32-product fits are counted in counts[3], and
// both LSQR variants then run over the same lists.
__global__ __launch_bounds__(256) void mixed_dispatch_b_kernel(const Item* fits, const FitDesc* D,
                                                               int max_refine, double tol32,
                                                               int* counts, int phases) {
  __shared__ double red[4];
  const FitDesc& d = D[fits[blockIdx.x].fit];
  const double kf = kappa_f_body<256>(d.R, d.q, d.M, d.p, red);
  const int path = mixed_path_of(kf == kf ? kf : INFINITY, max_refine);
  if (phases && path == MP_F64)
    for (int i = threadIdx.x; i < d.p; i += blockDim.x) d.phib[i] = d.phi0[i];
  if (threadIdx.x == 0) {
    d.rst->path = path;
    d.st->f32 = path == MP_F32 ? 1 : 0;
    if (!phases) {
      if (path == MP_F32) {
        d.st->tol = fmax(d.st->tol, tol32);
        atomicAdd(counts + 3, 1);
      }
    } else if (path == MP_F32) {
      d.st->tol = fmax(d.st->tol, tol32);
      d.rst->done = d.rst->inner_done = 1;
      d.rst->stop = 0;
    } else {
      d.st->done = 1;
      atomicAdd(counts, 1);
      if (path == MP_REFINE) atomicAdd(counts + 1, 1);
      if (path == MP_F64) {
        d.rst->done = d.rst->inner_done = 1;
        d.rst->stop = 5;
      }
    }
  }
}

// u = float(b) (b = y[p:]) for the fits about to run FP32-product LSQR, one
// workgroup per (fit, FFT block) item: rows [idx L, (idx + 1) L).
__global__ __launch_bounds__(256) void to_f32_b_kernel(const Item* blocks, const FitDesc* D) {
  const Item it = blocks[blockIdx.x];
  const FitDesc& d = D[it.fit];
  if (d.st->done || !d.st->f32) return;
  float* u = static_cast<float*>(d.u);
  const int64_t r0 = static_cast<int64_t>(it.idx) * d.L;
  const int64_t r1 = r0 + d.L < d.m ? r0 + d.L : d.m;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) u[i] = static_cast<float>(d.y[d.p + i]);
}


struct HostOut {
  LsqrState st;
  LsqrState ring[2];  // state snapshots at the ends of the chunks in flight
  RefineState rs;
  double dminmax[4];
  double rr[4];
  int status[4];
};
}  // namespace

// The fit of one series (device series d_y, or host series host_y copied in)
// on stream s; coef host, p doubles.
tls_status run_fit(tls_ctx* ctx, const Plan& pl, const tls_options& o, const double* d_y_in,
                   const double* host_y, double tol, hipStream_t s, double* coef, tls_result* res);

// ---- batched execution core (batch.hip), shared by the batched driver and
// the server -------------------------------------------------------------------

// A range of a device work-item table.
struct List {
  int off = 0, n = 0;
};

// The compile-time choices the single-fit path makes for a fit: FFT
// half-length, Cholesky register tiles (q = p + 1; 0 = global kernels),
// inverse register tiles (p; 0 = global kernel), LDS staging of M in the
// LSQR step.  Fits with equal keys share every launch of a batched run.
struct ClassKey {
  int lgn, qt, pt, mlds;
  bool operator<(const ClassKey& o) const {
    if (lgn != o.lgn) return lgn < o.lgn;
    if (qt != o.qt) return qt < o.qt;
    if (pt != o.pt) return pt < o.pt;
    return mlds < o.mlds;
  }
};
ClassKey class_key(const Plan& pl);
// The batched sketch kernels stage 16-row panels of width ldq in LDS (the
// tile TRSM's limit, orders up to 623); fits of larger order run one at a
// time in batched calls and are not served.
constexpr int BATCH_LDQ_MAX = TRSM_TILE_LDQ_MAX;

// Work-item lists of one class (offsets into one device item table).
// jl: one item per (fit, JL column); jlg: one per (fit, group of
// jl_cols(pmax) columns solved by one wavefront), pmax over the lists' fits.
struct ClassLists {
  List blocks, groups, blocks1, rows1, rows2, tiles1, tiles2, rowtiles2, trmm2, fits, fits1, jl, jlg,
      chunks, draws, cols, rblocks;
};
// Appends the lists of the fits with descriptor indices desc[i] and plans
// plans[i] to `items`.
ClassLists build_lists(std::vector<Item>& items, const std::vector<int>& desc,
                       const std::vector<const Plan*>& plans, bool leverage);

// Per-fit result record written on the device by collect_b.
struct FitRec {
  double rr, dmax, dmin, rnorm, arnorm;
  int status[4];
  int iters, istop, refine, path;
};

void fill_desc(const Plan& pl, const FitBufs& b, const double* y, uint32_t fit, double tol,
               FitDesc* d);
// LSQR and refinement state, status words (one item per fit).
hipError_t batch_init(const Item* fits, int nfits, FitDesc* D, int max_iter, int max_refine,
                      int inner_max, double inner_tol, hipStream_t s);
hipError_t batch_zero_ints(int* x, int n, hipStream_t s);

// Event pairs around launches of the dominant pass (profile = 1).
struct PassTimer {
  std::vector<hipEvent_t>* pool = nullptr;
  size_t n = 0;
  hipError_t begin(hipStream_t s);
  hipError_t end(hipStream_t s);
  hipError_t total_ms(double* ms) const;
};

// Spectra, two-stage sketch, final QR, inverse and warm start for the fits
// of one class.
tls_status setup_class(tls_ctx* ctx, const ClassKey& k, int pmax, int ldqmax, const Item* I,
                       const ClassLists& l, FitDesc* D, const tls_options& o, hipStream_t s);
// One LSQR step for the listed fits: the fused pass (first: from b and
// phi0, after the spectrum of phi0), the column sums and the p-side step.
// precs bit 0: FP64 products, bit 1: FP32 products (each launch skips the
// fits of the other precision).  groups32 / fits32 (optional): the FP32
// launches' own lists, the FP64 ones then taking groups / fits alone.
tls_status lsqr_step_class(tls_ctx* ctx, int lgn, int pmax, bool mlds, bool first,
                           int precs, const Item* groups, int ngroups, const Item* cols, int ncols,
                           const Item* fits, int nfits, FitDesc* D, int* counts, int* done_list,
                           PassTimer* tm, hipStream_t s, const Item* groups32 = nullptr,
                           int ngroups32 = 0, const Item* fits32 = nullptr, int nfits32 = 0);
// FP64 residual of phi (row-wise) for the listed fits.
tls_status residual_class(const Item* rblocks, int nrblocks, const Item* fits, int nfits, int pmax,
                          FitDesc* D, hipStream_t s);
// Coefficients (packed at item.idx) and result records (rec[k] for the k-th item).
// flags[k] = 1 when the k-th listed fit has finished (which 0: LSQR, 1: refinement).
hipError_t launch_done_flags_b(const Item* fits, int nfits, const FitDesc* D, int which,
                               int* flags, hipStream_t s);
// The compressed estimator for the listed fits: phi = phi0, marked finished.
hipError_t launch_compressed_b(const Item* fits, int nfits, const FitDesc* D, int* counts,
                               int* done_list, hipStream_t s);
hipError_t collect_b(const Item* fits, int nfits, const FitDesc* D, int mixed, double* coef,
                     FitRec* rec, hipStream_t s);
// Per-fit status from a record and the returned coefficients.
tls_status record_status(const FitRec& r, const double* coef, int p);
void record_result(const FitRec& r, const Plan& pl, double ms, tls_result* out);

// Batched driver: fits of `count` series (host series when host_series is
// non-null, else device series) grouped into launch classes; per-fit
// coefficients, results and statuses.
tls_status run_batch(tls_ctx* ctx, int count, const double* const* host_series,
                     const double* const* dev_series, const int64_t* n, const int32_t* p,
                     double tol, const tls_options& o, hipStream_t s, double* coef_packed,
                     const int64_t* coef_offset, tls_result* res, tls_status* fit_status);
