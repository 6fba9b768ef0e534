// p-side step of R-preconditioned LSQR (Paige and Saunders, ACM TOMS 8(1),
// 1982) on A = X M, M = R^{-1}: one workgroup per fit, or for a single fit
// of order above 128 with M in global memory the wide step (its products
// over many workgroups, four launches, the same bits).
//
// The m-side work of step i (u~ = X (M v) - (alpha/beta) u~_prev, its norm,
// and X^T u~) is done by the fused Toeplitz pass; the column sums arrive in
// g[0..p) (X^T u~) and g[p] (||u~||^2).  This kernel finishes the step:
//   beta = ||u~||,  v~ = M^T (X^T u~ / beta) - beta v,  alpha = ||v~||,
//   plane rotation (rho, c, s, theta, phi, phibar), z += (phi/rho) w,
//   w = v - (theta/rho) w, stopping tests, then either the packed spectrum
//   of M v (scaled by 1/B) for the next pass, or phi = phi0 + M z when done.
// The first call (phase 0) starts the bidiagonalisation from the residual of
// the warm start phi0: beta1 u1 = b - X phi0, alpha1 v1 = A^T u1, w1 = v1.
//
// Stopping (atol = btol = tol): ||A^T r|| <= tol ||A|| ||r|| (istop 2) or
// ||r|| <= tol ||r0|| + tol ||A|| ||z|| (istop 1); alpha or beta = 0 (istop 3,
// exact); a non-finite alpha or beta (istop 4, the last finite iterate is
// kept); no halving of the ||A^T r|| / (||A|| ||r||) estimate in
// LSQR_STALL consecutive iterations (istop 5: with A = X R^{-1} well
// conditioned each iteration gains a constant factor in exact arithmetic,
// so a stall means the rounding of the products has been reached);
// iteration limit (istop 7).
#include <math.h>

#include "fft.h"
#include "kernels.h"

namespace tls {

constexpr int LSQR_STALL = 30;

// The step kernel stages M in LDS when p <= 128 and it fits beside the
// 2^LGN-point transform buffer.
bool lsqr_step_lds(int lgn, int p) {
  const size_t with_m = (2 * static_cast<size_t>(p) + static_cast<size_t>(p) * (p | 1)) * sizeof(double);
  const size_t lds_static = static_cast<size_t>(1 << lgn) * 16 + 64;
  return p <= 128 && with_m + lds_static <= 160 * 1024;
}

// Dynamic LDS of the refinement kernels: three p-vectors, plus M (rows of
// odd length p | 1) when it is staged.
size_t refine_shm(int pmax, bool mlds) {
  return (3 * static_cast<size_t>(pmax) + (mlds ? static_cast<size_t>(pmax) * (pmax | 1) : 0)) *
         sizeof(double);
}

// The refinement kernels stage M in LDS when p <= 128 and it fits beside
// their static 2^LGN-point FP64 transform buffer and reduction words.
bool refine_lds(int lgn, int pmax) {
  const size_t lds_static = static_cast<size_t>(1 << lgn) * 16 + 64;
  return pmax <= 128 && lds_static + refine_shm(pmax, true) <= 160 * 1024;
}

namespace {

// Stages the p x p (p <= 128) row-major upper triangular matrix M into LDS
// rows of odd length ldm: wavefront w takes rows w, w + NW, ..., lanes the
// columns; every load of a thread is issued before its first store (one
// memory round trip).  Entries below the diagonal are not read.
template <int NT>
__device__ __forceinline__ void stage_m(const double* __restrict__ M, int p, int ldm,
                                        double* __restrict__ sM) {
  constexpr int NW = NT / 64;
  constexpr int RW = (128 + NW - 1) / NW;  // rows per wavefront at p = 128
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[RW][2];
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    const int r = wid + NW * u;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      v[u][h] = (r < p && c < p && c >= r) ? M[static_cast<size_t>(r) * p + c] : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    const int r = wid + NW * u;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      if (r < p && c < p) sM[r * ldm + c] = v[u][h];
    }
  }
}

// out[r] = sum_{c in [lo(r), hi(r))} Mrow[r][c] x(c) for the rows r of an
// upper (lo(r) = r, hi = p) or lower (lo = 0, hi(r) = r + 1) triangular p x p
// row-major matrix.  Wavefront w0 of wstride takes the row groups
// r0 = RU (w0 + wstride t), lanes the columns c = c0 + 64 k + lane, RU rows x
// CU column chunks of loads in flight.  Each lane sums its columns in
// increasing order and the lanes are combined by wave_sum, so a row's value
// does not depend on which wavefront or workgroup computes it, nor on RU and
// CU.  Results go to out[r] (lane 0 of the owning wave) via the callback.
template <bool UPPER, int RU, int CU, typename X, typename F>
__device__ __forceinline__ void tri_gemv_rows_at(const double* __restrict__ Mrow, int p, X&& xat,
                                                 F&& emit, int w0, int wstride) {
  const int lane = threadIdx.x & 63;
  for (int r0 = w0 * RU; r0 < p; r0 += wstride * RU) {
    double acc[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) acc[u] = 0.0;
    for (int c0 = 0; c0 < p; c0 += 64 * CU) {
      double mv[RU][CU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = r0 + u;
        const int lo = UPPER ? r : 0, hi = UPPER ? p : r + 1;
#pragma unroll
        for (int k = 0; k < CU; ++k) {
          const int c = c0 + 64 * k + lane;
          mv[u][k] = (r < p && c >= lo && c < hi) ? Mrow[static_cast<size_t>(r) * p + c] : 0.0;
        }
      }
#pragma unroll
      for (int k = 0; k < CU; ++k) {
        const int c = c0 + 64 * k + lane;
        const double xc = c < p ? xat(c) : 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) acc[u] += mv[u][k] * xc;
      }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) acc[u] = wave_sum(acc[u]);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < RU; ++u)
        if (r0 + u < p) emit(r0 + u, acc[u]);
    }
  }
}

// The same over the NT / 64 wavefronts of one workgroup, GEMV_RU rows x GEMV_CU
// column chunks in flight, x an array.
constexpr int GEMV_RU = 8, GEMV_CU = 2;
template <int NT, bool UPPER, typename F>
__device__ __forceinline__ void tri_gemv_rows(const double* __restrict__ Mrow, int p,
                                              const double* __restrict__ x, F&& emit) {
  tri_gemv_rows_at<UPPER, GEMV_RU, GEMV_CU>(Mrow, p, [&](int c) { return x[c]; }, emit,
                                      threadIdx.x >> 6, NT / 64);
}

// MLDS: M (p <= 128) is staged once into LDS (rows padded to an odd length)
// and every product with M or M^T reads it there, PARTS = NT / 128 threads
// per output (partial sums over every PARTS-th term, combined by a fixed
// butterfly: every thread of the group ends with the same value).
template <int PARTS>
__device__ __forceinline__ double parts_sum_t(double x) {
#pragma unroll
  for (int off = 1; off < PARTS; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Scalars of one LSQR step, as stored back into LsqrState.
struct StepOut {
  double alpha, beta, rhobar, phibar, anorm2, bnorm, rnorm, arnorm, znorm, best_ratio;
  int iter, istop, best_iter;
  bool done;
};

// The recurrences of one step once alpha, beta and the normalised v~ (sv,
// p values) are known: the plane rotation, z += (phi/rho) w and
// w = v - (theta/rho) w (written to w and z), ||z|| and the stopping tests.
// All NT threads of the workgroup take part (block sums).
template <int NT>
__device__ __forceinline__ StepOut lsqr_recur(int p, const LsqrState* __restrict__ st,
                                              double alpha, double beta, bool init,
                                              const double* __restrict__ sv,
                                              double* __restrict__ w, double* __restrict__ z,
                                              double* __restrict__ red) {
  const int tid = threadIdx.x;
  const double tol = st->tol;
  const double alpha_prev = st->alpha;
  StepOut o;
  o.alpha = alpha;
  o.beta = beta;
  o.rhobar = st->rhobar;
  o.phibar = st->phibar;
  o.anorm2 = st->anorm2;
  o.bnorm = st->bnorm;
  o.znorm = st->znorm;
  o.iter = st->iter;
  o.istop = 0;
  o.best_ratio = st->best_ratio;
  o.best_iter = st->best_iter;
  o.done = false;
  if (init) {
    o.bnorm = beta;
    o.phibar = beta;
    o.rhobar = alpha;
    o.anorm2 = 0.0;
    for (int j = tid; j < p; j += NT) {
      w[j] = sv[j];
      z[j] = 0.0;
    }
    o.rnorm = beta;
    o.arnorm = alpha * beta;
    o.znorm = 0.0;
    o.best_ratio = INFINITY;
    o.best_iter = 0;
    if (o.arnorm == 0.0) {
      o.done = true;
      o.istop = 0;
    }
  } else if (!isfinite(alpha) || !isfinite(beta)) {
    // numerical breakdown: keep the last finite iterate
    o.done = true;
    o.istop = 4;
    o.iter += 1;
    o.rnorm = st->rnorm;
    o.arnorm = st->arnorm;
  } else {
    o.anorm2 += alpha_prev * alpha_prev + beta * beta;
    const double rho = hypot(o.rhobar, beta);
    const double c = o.rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    o.rhobar = -c * alpha;
    const double phik = c * o.phibar;
    o.phibar = sn * o.phibar;
    const double t1 = phik / rho, t2 = -theta / rho;
    double zsq = 0.0;
    for (int j = tid; j < p; j += NT) {
      const double wj = w[j];
      const double zj = z[j] + t1 * wj;
      z[j] = zj;
      w[j] = sv[j] + t2 * wj;
      zsq += zj * zj;
    }
    o.znorm = sqrt(block_sum<NT>(zsq, red));
    o.rnorm = o.phibar;
    o.arnorm = o.phibar * alpha * fabs(c);
    const double anorm = sqrt(o.anorm2);
    o.iter += 1;
    const double ratio = o.arnorm / (anorm * o.rnorm);
    if (ratio < 0.5 * o.best_ratio) {
      o.best_ratio = ratio;
      o.best_iter = o.iter;
    }
    if (o.arnorm <= tol * anorm * o.rnorm) {
      o.done = true;
      o.istop = 2;
    } else if (o.rnorm <= tol * o.bnorm + tol * anorm * o.znorm) {
      o.done = true;
      o.istop = 1;
    } else if (alpha == 0.0 || beta == 0.0) {
      o.done = true;
      o.istop = 3;
    } else if (o.iter - o.best_iter >= LSQR_STALL) {
      o.done = true;
      o.istop = 5;
    } else if (o.iter >= st->max_iter) {
      o.done = true;
      o.istop = 7;
    }
  }
  return o;
}

__device__ __forceinline__ void lsqr_store(LsqrState* __restrict__ st, const StepOut& o) {
  if (threadIdx.x == 0) {
    st->alpha = o.alpha;
    st->beta = o.beta;
    st->rhobar = o.rhobar;
    st->phibar = o.phibar;
    st->anorm2 = o.anorm2;
    st->bnorm = o.bnorm;
    st->rnorm = o.rnorm;
    st->arnorm = o.arnorm;
    st->znorm = o.znorm;
    st->best_ratio = o.best_ratio;
    st->best_iter = o.best_iter;
    st->iter = o.iter;
    st->istop = o.istop;
    st->phase = 1;
    st->coef[0] = 1.0;
    st->coef[1] = o.beta > 0.0 ? -o.alpha / o.beta : 0.0;
    if (o.done) st->done = 1;
  }
}

// Packed spectrum (scaled 1/B) of the real p-vector q into Vhat (TS words).
template <int LGN, int NT, typename TS>
__device__ void spectrum_of(const double* __restrict__ q, int p, cx<double>* s,
                            cx<TS>* __restrict__ Vhat, const cx<double>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  for (int t = threadIdx.x; t < N; t += NT) {
    const int i0 = 2 * t;
    s[swz<double>(t)] = {i0 < p ? q[i0] : 0.0, i0 + 1 < p ? q[i0 + 1] : 0.0};
  }
  __syncthreads();
  fft_dif<double, false, LGN, NT>(s, tab);
  const double invB = 1.0 / static_cast<double>(2 * N);
  for (int k = threadIdx.x; k <= N / 2; k += NT) {
    const cx<double> wk = twiddle<double, false>(tab, k, LGN + 1);
    cx<double> Xk, Xnk;
    rfft_post(s[swz<double>(bitrev(k, LGN))], s[swz<double>(bitrev((N - k) & (N - 1), LGN))], wk,
              Xk, Xnk);
    Xk = cscale(Xk, invB);
    Xnk = cscale(Xnk, invB);
    if (k == 0) {
      Vhat[0] = {static_cast<TS>(Xk.x), static_cast<TS>(Xnk.x)};
    } else {
      Vhat[k] = {static_cast<TS>(Xk.x), static_cast<TS>(Xk.y)};
      if (2 * k != N) Vhat[N - k] = {static_cast<TS>(Xnk.x), static_cast<TS>(Xnk.y)};
    }
  }
}

template <int LGN, int NT, typename TS, bool MLDS>
__device__ __forceinline__ void lsqr_step_body(int p, LsqrState* __restrict__ st,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ M,
                                                       const double* __restrict__ Mt,
                                                       double* __restrict__ v,
                                                       double* __restrict__ w,
                                                       double* __restrict__ z,
                                                       const double* __restrict__ phi0,
                                                       double* __restrict__ phi,
                                                       cx<TS>* __restrict__ Vhat,
                                                       const cx<double>* __restrict__ tab,
                                                       LsqrState* __restrict__ snap = nullptr) {
  constexpr int N = 1 << LGN;
  constexpr int PARTS = NT / 128 > 0 ? NT / 128 : 1;
  static_assert(!MLDS || PARTS * 128 == NT, "M in LDS: NT / 128 threads per output");
  auto parts_sum = [](double x) { return parts_sum_t<PARTS>(x); };
  __shared__ cx<double> s[N];
  extern __shared__ double smem[];
  double* sg = smem;
  double* sv = sg + p;
  double* sM = sv + p;  // MLDS: p x ldm
  const int ldm = p | 1;
  __shared__ double red[NT / 64];
  // the state, g and M are requested together (one memory round trip)
  const int done_in = st->done;
  const double gp = g[p];
  const int tid = threadIdx.x;
  const double gt = tid < p ? g[tid] : 0.0;
  if constexpr (MLDS) {
    stage_m<NT>(M, p, ldm, sM);
  }
  if (done_in) {
    if (snap && tid == 0) *snap = *st;
    return;
  }
  const bool init = st->phase == 0;

  const double beta = sqrt(gp);
  const double invbeta = beta > 0.0 ? 1.0 / beta : 0.0;
  if (tid < p) sg[tid] = gt * invbeta;
  for (int i = tid + NT; i < p; i += NT) sg[i] = g[i] * invbeta;
  __syncthreads();

  // v~ = M^T (X^T u) - beta v: row j of M^T (= column j of M) is Mt[j][0..j]
  double hsq = 0.0;
  if constexpr (MLDS) {
    // PARTS consecutive threads per output j, each over every PARTS-th i
    const int j = tid / PARTS, part = tid % PARTS;
    double acc = 0.0;
    if (j < p)
      for (int i = part; i <= j; i += PARTS) acc += sM[i * ldm + j] * sg[i];
    acc = parts_sum(acc);
    if (j < p && part == 0) {
      const double h = init ? acc : acc - beta * v[j];
      sv[j] = h;
      hsq += h * h;
    }
  } else {
    // ||v~||^2: lane 0 of each wavefront over its rows in order (the wide
    // step's recurrence kernel repeats this order)
    tri_gemv_rows<NT, false>(Mt, p, sg, [&](int j, double acc) {
      const double h = init ? acc : acc - beta * v[j];
      sv[j] = h;
      hsq += h * h;
    });
  }
  const double alpha = sqrt(block_sum<NT>(hsq, red));
  const double invalpha = alpha > 0.0 ? 1.0 / alpha : 0.0;
  for (int j = tid; j < p; j += NT) {
    sv[j] *= invalpha;
    v[j] = sv[j];
  }

  const StepOut o = lsqr_recur<NT>(p, st, alpha, beta, init, sv, w, z, red);
  __syncthreads();

  if (!o.done) {
    // q = M v_new into sg, then its packed spectrum scaled by 1/B.
    if constexpr (MLDS) {
      const int i = tid / PARTS, part = tid % PARTS;
      double acc = 0.0;
      if (i < p)
        for (int j = i + part; j < p; j += PARTS) acc += sM[i * ldm + j] * sv[j];
      acc = parts_sum(acc);
      if (i < p && part == 0) sg[i] = acc;
    } else {
      tri_gemv_rows<NT, true>(M, p, sv, [&](int i, double acc) { sg[i] = acc; });
    }
    __syncthreads();
    spectrum_of<LGN, NT, TS>(sg, p, s, Vhat, tab);
  } else {
    // phi = phi0 + M z
    __syncthreads();
    if constexpr (MLDS) {
      for (int i = tid; i < p; i += NT) {
        double acc = 0.0;
        for (int j = i; j < p; ++j) acc += sM[i * ldm + j] * z[j];
        phi[i] = phi0[i] + acc;
      }
    } else {
      tri_gemv_rows<NT, true>(M, p, z, [&](int i, double acc) { phi[i] = phi0[i] + acc; });
    }
  }
  lsqr_store(st, o);
  if (snap && tid == 0) *snap = *st;
}

template <int LGN, int NT, typename TS, bool MLDS>
__global__ __launch_bounds__(NT) void lsqr_step_kernel(int p, LsqrState* __restrict__ st,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ M,
                                                       const double* __restrict__ Mt,
                                                       double* __restrict__ v,
                                                       double* __restrict__ w,
                                                       double* __restrict__ z,
                                                       const double* __restrict__ phi0,
                                                       double* __restrict__ phi,
                                                       cx<TS>* __restrict__ Vhat,
                                                       const cx<double>* __restrict__ tab,
                                                       LsqrState* __restrict__ snap) {
  lsqr_step_body<LGN, NT, TS, MLDS>(p, st, g, M, Mt, v, w, z, phi0, phi, Vhat, tab, snap);
}

// ---- wide step: M from global memory and p > WIDE_P_MIN -------------------
// The two triangular products of a step spread over ceil(p / 8) workgroups
// of 256 threads (a wavefront per group of 2 rows, 8 column chunks of its
// loads in flight: at p = 500 each CU streams 32 KB of M), the recurrences
// and the spectrum on one workgroup of 1024 threads each:
// four launches in place of the one workgroup's chain of dependent memory
// round trips (16 at p = 500).  They reproduce the one-workgroup step with M
// in global memory bit for bit: each row of a product is summed by one
// wavefront in the same lane order (tri_gemv_rows_at), and the recurrences
// and the spectrum run the same code with the same thread count.
constexpr int WIDE_NT = 1024, WIDE_GEMV_NT = 256, WIDE_RU = 2, WIDE_CU = 8, WIDE_P_MIN = 128;

int wide_groups(int p) {
  constexpr int rows = WIDE_RU * (WIDE_GEMV_NT / 64);
  return (p + rows - 1) / rows;
}

// v <- v~ = M^T (g / beta) - beta v (phase 0: without the v term), in place.
__global__ __launch_bounds__(WIDE_GEMV_NT) void wide_h_kernel(int p, const LsqrState* __restrict__ st,
                                                         const double* __restrict__ g,
                                                         const double* __restrict__ Mt,
                                                         double* __restrict__ v) {
  if (st->done) return;
  const bool init = st->phase == 0;
  const double beta = sqrt(g[p]);
  const double invbeta = beta > 0.0 ? 1.0 / beta : 0.0;
  constexpr int NW = WIDE_GEMV_NT / 64;
  tri_gemv_rows_at<false, WIDE_RU, WIDE_CU>(
      Mt, p, [&](int c) { return g[c] * invbeta; },
      [&](int j, double acc) { v[j] = init ? acc : acc - beta * v[j]; },
      static_cast<int>(blockIdx.x) * NW + static_cast<int>(threadIdx.x >> 6),
      static_cast<int>(gridDim.x) * NW);
}

// alpha = ||v~||, v = v~ / alpha, the recurrences and the stopping tests;
// phi = phi0 + M z when the step ends the iteration.  One workgroup.
__global__ __launch_bounds__(WIDE_NT) void wide_recur_kernel(int p, LsqrState* __restrict__ st,
                                                             const double* __restrict__ g,
                                                             const double* __restrict__ M,
                                                             double* __restrict__ v,
                                                             double* __restrict__ w,
                                                             double* __restrict__ z,
                                                             const double* __restrict__ phi0,
                                                             double* __restrict__ phi,
                                                             LsqrState* __restrict__ snap) {
  constexpr int NT = WIDE_NT;
  extern __shared__ double sv[];
  __shared__ double red[NT / 64];
  if (st->done) {
    if (snap && threadIdx.x == 0) *snap = *st;
    return;
  }
  const bool init = st->phase == 0;
  const double beta = sqrt(g[p]);
  const int tid = threadIdx.x;
  for (int j = tid; j < p; j += NT) sv[j] = v[j];
  __syncthreads();
  // ||v~||^2 in the one-workgroup step's order: lane 0 of wavefront w adds
  // the squares of the rows it would have computed there (groups of GEMV_RU
  // rows from GEMV_RU w, every NT / 64 groups), then the block sum
  double hsq = 0.0;
  if ((tid & 63) == 0) {
    for (int r0 = (tid >> 6) * GEMV_RU; r0 < p; r0 += GEMV_RU * (NT / 64))
      for (int u = 0; u < GEMV_RU; ++u)
        if (r0 + u < p) hsq += sv[r0 + u] * sv[r0 + u];
  }
  const double alpha = sqrt(block_sum<NT>(hsq, red));
  const double invalpha = alpha > 0.0 ? 1.0 / alpha : 0.0;
  for (int j = tid; j < p; j += NT) {
    sv[j] *= invalpha;
    v[j] = sv[j];
  }
  const StepOut o = lsqr_recur<NT>(p, st, alpha, beta, init, sv, w, z, red);
  __syncthreads();
  if (o.done)
    tri_gemv_rows<NT, true>(M, p, z, [&](int i, double acc) { phi[i] = phi0[i] + acc; });
  lsqr_store(st, o);
  if (snap && tid == 0) *snap = *st;
}

// q = M v for the next pass.
__global__ __launch_bounds__(WIDE_GEMV_NT) void wide_q_kernel(int p, const LsqrState* __restrict__ st,
                                                         const double* __restrict__ M,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ q) {
  if (st->done) return;
  constexpr int NW = WIDE_GEMV_NT / 64;
  tri_gemv_rows_at<true, WIDE_RU, WIDE_CU>(
      M, p, [&](int c) { return v[c]; }, [&](int i, double acc) { q[i] = acc; },
      static_cast<int>(blockIdx.x) * NW + static_cast<int>(threadIdx.x >> 6),
      static_cast<int>(gridDim.x) * NW);
}

// The packed spectrum of q, scaled by 1/B, into Vhat.
template <int LGN, typename TS>
__global__ __launch_bounds__(WIDE_NT) void wide_spec_kernel(int p, const LsqrState* __restrict__ st,
                                                            const double* __restrict__ q,
                                                            cx<TS>* __restrict__ Vhat,
                                                            const cx<double>* __restrict__ tab) {
  __shared__ cx<double> s[1 << LGN];
  if (st->done) return;
  spectrum_of<LGN, WIDE_NT, TS>(q, p, s, Vhat, tab);
}

template <int LGN, typename TS>
hipError_t step_one(int p, LsqrState* st, const double* g, const double* M, const double* Mt,
                    double* v, double* w, double* z, const double* phi0, double* phi, void* Vhat,
                    double* q, LsqrState* snap, const Twiddles& tw, hipStream_t stream) {
  constexpr int NT = 512;  // M in LDS: 8 wavefronts
  const size_t small = 2 * static_cast<size_t>(p) * sizeof(double);
  const size_t with_m = small + static_cast<size_t>(p) * (p | 1) * sizeof(double);
  const cx<double>* tab = static_cast<const cx<double>*>(tw.d64);
  if (lsqr_step_lds(LGN, p)) {
    hipLaunchKernelGGL((lsqr_step_kernel<LGN, NT, TS, true>), dim3(1), dim3(NT), with_m, stream, p,
                       st, g, M, Mt, v, w, z, phi0, phi, static_cast<cx<TS>*>(Vhat), tab, snap);
  } else if (p > WIDE_P_MIN && q) {
    const int groups = wide_groups(p);
    hipLaunchKernelGGL(wide_h_kernel, dim3(groups), dim3(WIDE_GEMV_NT), 0, stream, p, st, g, Mt, v);
    hipLaunchKernelGGL(wide_recur_kernel, dim3(1), dim3(WIDE_NT), p * sizeof(double), stream, p,
                       st, g, M, v, w, z, phi0, phi, snap);
    hipLaunchKernelGGL(wide_q_kernel, dim3(groups), dim3(WIDE_GEMV_NT), 0, stream, p, st, M, v, q);
    hipLaunchKernelGGL((wide_spec_kernel<LGN, TS>), dim3(1), dim3(WIDE_NT), 0, stream, p, st, q,
                       static_cast<cx<TS>*>(Vhat), tab);
  } else {
    // M read from global memory: 16 wavefronts keep more of its rows in flight
    constexpr int NTG = 1024;
    hipLaunchKernelGGL((lsqr_step_kernel<LGN, NTG, TS, false>), dim3(1), dim3(NTG), small, stream, p,
                       st, g, M, Mt, v, w, z, phi0, phi, static_cast<cx<TS>*>(Vhat), tab, snap);
  }
  return hipGetLastError();
}

// ---- mixed-precision refinement p-side kernels ---------------------------
// Both stage M into LDS when p <= 128 (padded rows), else read it from global.

// out = M^T x (M upper; out[j] = sum_{i <= j} M[i][j] x[i]) or M x.
template <int NT, bool TRANS>
__device__ void gemv_m(const double* __restrict__ M, const double* __restrict__ Mt, const double* sM,
                       int ldm, bool lds, int p, const double* x, double* out) {
  if (lds) {
    for (int r = threadIdx.x; r < p; r += NT) {
      double a0 = 0.0, a1 = 0.0;
      if (TRANS) {
        int i = 0;
        for (; i + 1 <= r; i += 2) {
          a0 += sM[i * ldm + r] * x[i];
          a1 += sM[(i + 1) * ldm + r] * x[i + 1];
        }
        if (i <= r) a0 += sM[i * ldm + r] * x[i];
      } else {
        int j = r;
        for (; j + 1 < p; j += 2) {
          a0 += sM[r * ldm + j] * x[j];
          a1 += sM[r * ldm + j + 1] * x[j + 1];
        }
        if (j < p) a0 += sM[r * ldm + j] * x[j];
      }
      out[r] = a0 + a1;
    }
  } else if (TRANS) {
    tri_gemv_rows<NT, false>(Mt, p, x, [&](int j, double acc) { out[j] = acc; });
  } else {
    tri_gemv_rows<NT, true>(M, p, x, [&](int i, double acc) { out[i] = acc; });
  }
  __syncthreads();
}

template <int NT>
__device__ double dot_block(const double* a, const double* b, int p, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < p; i += NT) acc += a[i] * b[i];
  return block_sum<NT>(acc, red);
}

template <int LGN, int NT>
__device__ __forceinline__ void refine_outer_body(int p, RefineState* __restrict__ st,
                                                          const double* __restrict__ g64,
                                                          const double* __restrict__ M,
                                                          const double* __restrict__ Mt,
                                                          const double* __restrict__ phi,
                                                          double* __restrict__ phib,
                                                          double* __restrict__ w,
                                                          double* __restrict__ res,
                                                          double* __restrict__ d,
                                                          cx<float>* __restrict__ Vhat32,
                                                          const cx<double>* __restrict__ tab,
                                                          bool mlds) {
  constexpr int N = 1 << LGN;
  __shared__ cx<double> s[N];
  __shared__ double red[NT / 64];
  extern __shared__ double smem[];
  double* sx = smem;      // p
  double* sh = sx + p;    // p
  double* sq = sh + p;    // p
  double* sM = sq + p;    // p x ldm when lds
  const int ldm = p | 1;
  const bool lds = mlds && p <= 128;
  if (st->done) return;
  // every thread reads the state it decides on before thread 0 rewrites it
  // (the barrier ahead of the state update below)
  const int outer = st->outer;
  const double hbest = st->hbest, hprev = st->hprev, tol = st->tol;
  const int max_refine = st->max_refine;
  if (lds)
    stage_m<NT>(M, p, ldm, sM);
  for (int i = threadIdx.x; i < p; i += NT) sx[i] = g64[i];
  __syncthreads();
  gemv_m<NT, true>(M, Mt, sM, ldm, lds, p, sx, sh);  // h = M^T X^T r
  const double hh = dot_block<NT>(sh, sh, p, red);
  const double hn = sqrt(hh), rn = sqrt(g64[p]);
  // keep the best iterate: the FP32 products may stop contracting, or expand,
  // beyond their resolution
  const bool best = outer == 0 || hn < hbest;
  if (best)
    for (int i = threadIdx.x; i < p; i += NT) phib[i] = phi[i];
  bool done = false;
  int stop = 0;
  if (hn <= tol * rn) {
    done = true;
    stop = 1;
  } else if (outer >= max_refine) {
    done = true;
    stop = 7;
  } else if (outer > 0 && !(hn < 0.5 * hprev)) {
    done = true;  // no further contraction (FP32 products at their resolution)
    stop = 5;
  }
  if (!done) {
    for (int i = threadIdx.x; i < p; i += NT) {
      w[i] = 0.0;
      res[i] = sh[i];
      d[i] = sh[i];
    }
    gemv_m<NT, false>(M, Mt, sM, ldm, lds, p, sh, sq);  // M d
    spectrum_of<LGN, NT, float>(sq, p, s, Vhat32, tab);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->rnorm = rn;
    st->hprev = st->hnorm > 0.0 ? fmin(st->hnorm, hn) : hn;
    if (best) st->hbest = hn;
    st->hnorm = hn;
    st->rho = hh;
    st->rho0 = hh;
    st->inner = 0;
    st->inner_done = done ? 1 : 0;
    st->outer = outer + 1;
    st->stop = stop;
    if (done) st->done = 1;
  }
}

template <int LGN, int NT>
__global__ __launch_bounds__(NT) void refine_outer_kernel(int p, RefineState* __restrict__ st,
                                                          const double* __restrict__ g64,
                                                          const double* __restrict__ M,
                                                          const double* __restrict__ Mt,
                                                          const double* __restrict__ phi,
                                                          double* __restrict__ phib,
                                                          double* __restrict__ w,
                                                          double* __restrict__ res,
                                                          double* __restrict__ d,
                                                          cx<float>* __restrict__ Vhat32,
                                                          const cx<double>* __restrict__ tab,
                                                          bool mlds) {
  refine_outer_body<LGN, NT>(p, st, g64, M, Mt, phi, phib, w, res, d, Vhat32, tab, mlds);
}

template <int LGN, int NT>
__device__ __forceinline__ void refine_cg_body(int p, RefineState* __restrict__ st,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ M,
                                                       const double* __restrict__ Mt,
                                                       double* __restrict__ w,
                                                       double* __restrict__ res,
                                                       double* __restrict__ d,
                                                       double* __restrict__ phi,
                                                       cx<float>* __restrict__ Vhat32,
                                                       const cx<double>* __restrict__ tab,
                                                       bool mlds) {
  constexpr int N = 1 << LGN;
  __shared__ cx<double> s[N];
  __shared__ double red[NT / 64];
  extern __shared__ double smem[];
  double* sx = smem;    // p
  double* st_ = sx + p; // p: t = M^T g
  double* sq = st_ + p; // p
  double* sM = sq + p;
  const int ldm = p | 1;
  const bool lds = mlds && p <= 128;
  if (st->inner_done) return;
  if (lds)
    stage_m<NT>(M, p, ldm, sM);
  for (int i = threadIdx.x; i < p; i += NT) sx[i] = g[i];
  __syncthreads();
  gemv_m<NT, true>(M, Mt, sM, ldm, lds, p, sx, st_);  // t = A^T A d
  const double dt = dot_block<NT>(d, st_, p, red);
  const double rho = st->rho;
  const double alpha = dt > 0.0 ? rho / dt : 0.0;
  double rr = 0.0;
  for (int i = threadIdx.x; i < p; i += NT) {
    w[i] += alpha * d[i];
    const double ri = res[i] - alpha * st_[i];
    res[i] = ri;
    rr += ri * ri;
  }
  const double rho_new = block_sum<NT>(rr, red);
  const int inner = st->inner + 1;
  const bool finish = !(dt > 0.0) || !isfinite(rho_new) || rho_new <= st->inner_tol * st->inner_tol * st->rho0 ||
                      inner >= st->inner_max;
  if (!finish) {
    const double beta = rho_new / rho;
    for (int i = threadIdx.x; i < p; i += NT) d[i] = res[i] + beta * d[i];
    __syncthreads();
    gemv_m<NT, false>(M, Mt, sM, ldm, lds, p, d, sq);
    spectrum_of<LGN, NT, float>(sq, p, s, Vhat32, tab);
  } else {
    __syncthreads();
    gemv_m<NT, false>(M, Mt, sM, ldm, lds, p, w, sq);  // phi += M w
    for (int i = threadIdx.x; i < p; i += NT) phi[i] += sq[i];
  }
  if (threadIdx.x == 0) {
    st->rho = rho_new;
    st->inner = inner;
    st->total_inner += 1;
    if (finish) st->inner_done = 1;
  }
}

template <int LGN, int NT>
__global__ __launch_bounds__(NT) void refine_cg_kernel(int p, RefineState* __restrict__ st,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ M,
                                                       const double* __restrict__ Mt,
                                                       double* __restrict__ w,
                                                       double* __restrict__ res,
                                                       double* __restrict__ d,
                                                       double* __restrict__ phi,
                                                       cx<float>* __restrict__ Vhat32,
                                                       const cx<double>* __restrict__ tab,
                                                       bool mlds) {
  refine_cg_body<LGN, NT>(p, st, g, M, Mt, w, res, d, phi, Vhat32, tab, mlds);
}

template <int LGN>
hipError_t refine_outer_one(int p, RefineState* st, const double* g64, const double* M,
                            const double* Mt, const double* phi, double* phib, double* w,
                            double* res, double* d, void* Vhat32, const Twiddles& tw,
                            hipStream_t s) {
  const bool mlds = refine_lds(LGN, p);
  hipLaunchKernelGGL((refine_outer_kernel<LGN, 256>), dim3(1), dim3(256), refine_shm(p, mlds), s, p,
                     st, g64, M, Mt, phi, phib, w, res, d, static_cast<cx<float>*>(Vhat32),
                     static_cast<const cx<double>*>(tw.d64), mlds);
  return hipGetLastError();
}

template <int LGN>
hipError_t refine_cg_one(int p, RefineState* st, const double* g, const double* M, const double* Mt,
                         double* w, double* res, double* d, double* phi, void* Vhat32,
                         const Twiddles& tw, hipStream_t s) {
  const bool mlds = refine_lds(LGN, p);
  hipLaunchKernelGGL((refine_cg_kernel<LGN, 256>), dim3(1), dim3(256), refine_shm(p, mlds), s, p, st,
                     g, M, Mt, w, res, d, phi, static_cast<cx<float>*>(Vhat32),
                     static_cast<const cx<double>*>(tw.d64), mlds);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void gemv_upper_kernel(const double* __restrict__ Mt,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ y0, int p,
                                                         double* __restrict__ out) {
  for (int i = threadIdx.x; i < p; i += 256) {
    double acc = 0.0;
    for (int j = i; j < p; ++j) acc += Mt[static_cast<size_t>(j) * p + i] * x[j];
    out[i] = (y0 ? y0[i] : 0.0) + acc;
  }
}

}  // namespace

hipError_t launch_lsqr_step(int prec, int lgn, int p, LsqrState* st, const double* g,
                            const double* M, const double* Mt, double* v, double* w, double* z,
                            const double* phi0, double* phi, void* Vhat, double* q,
                            LsqrState* snap, const Twiddles& tw, hipStream_t stream) {
  const size_t shm = (2 * static_cast<size_t>(1 << lgn) + 2 * p) * sizeof(double);
  if (shm > 160 * 1024) return hipErrorInvalidValue;
#define TLS_STEP_CASE(LG)                                                                       \
  case LG:                                                                                      \
    return prec == PREC_F64                                                                     \
               ? step_one<LG, double>(p, st, g, M, Mt, v, w, z, phi0, phi, Vhat, q, snap, tw, stream)   \
               : step_one<LG, float>(p, st, g, M, Mt, v, w, z, phi0, phi, Vhat, q, snap, tw, stream);
  switch (lgn) {
    TLS_STEP_CASE(6)
    TLS_STEP_CASE(7)
    TLS_STEP_CASE(8)
    TLS_STEP_CASE(9)
    TLS_STEP_CASE(10)
    TLS_STEP_CASE(11)
    TLS_STEP_CASE(12)
    TLS_STEP_CASE(13)
    default:
      return hipErrorInvalidValue;
  }
#undef TLS_STEP_CASE
}

#define TLS_LG_SWITCH(CALL)                   \
  switch (lgn) {                              \
    case 6: return CALL(6);                   \
    case 7: return CALL(7);                   \
    case 8: return CALL(8);                   \
    case 9: return CALL(9);                   \
    case 10: return CALL(10);                 \
    case 11: return CALL(11);                 \
    case 12: return CALL(12);                 \
    case 13: return CALL(13);                 \
    default: return hipErrorInvalidValue;     \
  }

hipError_t launch_refine_outer(int lgn, int p, RefineState* st, const double* g64, const double* M,
                               const double* Mt, const double* phi, double* phib, double* w,
                               double* res, double* d, void* Vhat32, const Twiddles& tw,
                               hipStream_t s) {
#define TLS_OUTER(LG) refine_outer_one<LG>(p, st, g64, M, Mt, phi, phib, w, res, d, Vhat32, tw, s)
  TLS_LG_SWITCH(TLS_OUTER)
#undef TLS_OUTER
}

hipError_t launch_refine_cg(int lgn, int p, RefineState* st, const double* g, const double* M,
                            const double* Mt, double* w, double* res, double* d, double* phi,
                            void* Vhat32, const Twiddles& tw, hipStream_t s) {
#define TLS_CG(LG) refine_cg_one<LG>(p, st, g, M, Mt, w, res, d, phi, Vhat32, tw, s)
  TLS_LG_SWITCH(TLS_CG)
#undef TLS_CG
}

// out = y0 + M x for upper-triangular M given as Mt = M^T (row-major).
hipError_t launch_vec_axpy_small(const double* Mt, const double* x, const double* y0, int p,
                                 double* out, hipStream_t st) {
  hipLaunchKernelGGL(gemv_upper_kernel, dim3(1), dim3(256), 0, st, Mt, x, y0, p, out);
  return hipGetLastError();
}

// ---- batched launches: one workgroup per fit (items[blockIdx.x].fit) ---------
namespace {

// counts[0]: fits whose LSQR (or refinement) has finished; counts[1]: fits
// whose inner CG solve of the current refinement step has finished, or,
// during LSQR, the finished fits with FP32 products.  When done_list is
// given, every fit that finishes in this launch appends its descriptor index
// there (length in counts[2]).
template <int LGN, int NT, typename TS, bool MLDS>
__global__ __launch_bounds__(NT) void lsqr_step_b_kernel(const Item* __restrict__ fits,
                                                         const FitDesc* __restrict__ D,
                                                         int* __restrict__ counts,
                                                         int* __restrict__ done_list,
                                                         const cx<double>* __restrict__ tab) {
  const int f = fits[blockIdx.x].fit;
  const FitDesc& d = D[f];
  if (d.st->done || (sizeof(TS) == 4) != (d.st->f32 != 0)) return;
  lsqr_step_body<LGN, NT, TS, MLDS>(d.p, d.st, d.g, d.M, d.Mt, d.v, d.w, d.z, d.phi0, d.phi,
                                    static_cast<cx<TS>*>(d.Vhat), tab);
  if (threadIdx.x == 0 && d.st->done) {
    atomicAdd(counts, 1);
    if (sizeof(TS) == 4) atomicAdd(counts + 1, 1);
    if (done_list) done_list[atomicAdd(counts + 2, 1)] = f;
  }
}

template <int LGN, int NT>
__global__ __launch_bounds__(NT) void refine_outer_b_kernel(const Item* __restrict__ fits,
                                                            const FitDesc* __restrict__ D,
                                                            int* __restrict__ counts,
                                                            const cx<double>* __restrict__ tab,
                                                            bool mlds) {
  const FitDesc& d = D[fits[blockIdx.x].fit];
  if (!d.rst->done)
    refine_outer_body<LGN, NT>(d.p, d.rst, d.g, d.M, d.Mt, d.phi, d.phib, d.cw, d.cres, d.cd,
                               static_cast<cx<float>*>(d.Vhat32), tab, mlds);
  if (threadIdx.x == 0) {
    if (d.rst->done) atomicAdd(counts, 1);
    if (d.rst->inner_done) atomicAdd(counts + 1, 1);
  }
}

template <int LGN, int NT>
__global__ __launch_bounds__(NT) void refine_cg_b_kernel(const Item* __restrict__ fits,
                                                         const FitDesc* __restrict__ D,
                                                         int* __restrict__ counts,
                                                         const cx<double>* __restrict__ tab,
                                                         bool mlds) {
  const FitDesc& d = D[fits[blockIdx.x].fit];
  if (d.rst->inner_done) return;
  refine_cg_body<LGN, NT>(d.p, d.rst, d.g, d.M, d.Mt, d.cw, d.cres, d.cd, d.phi,
                          static_cast<cx<float>*>(d.Vhat32), tab, mlds);
  if (threadIdx.x == 0 && d.rst->inner_done) atomicAdd(counts + 1, 1);
}

template <int LGN, typename TS>
hipError_t step_b(const Item* fits, int nfits, int pmax, bool mlds, const FitDesc* D, int* counts,
                  int* done_list, const Twiddles& tw, hipStream_t s) {
  constexpr int NT = 512;  // as the single-fit step
  const size_t small = 2 * static_cast<size_t>(pmax) * sizeof(double);
  const size_t with_m = small + static_cast<size_t>(pmax) * (pmax | 1) * sizeof(double);
  const cx<double>* tab = static_cast<const cx<double>*>(tw.d64);
  if (mlds)
    hipLaunchKernelGGL((lsqr_step_b_kernel<LGN, NT, TS, true>), dim3(nfits), dim3(NT), with_m, s,
                       fits, D, counts, done_list, tab);
  else
    hipLaunchKernelGGL((lsqr_step_b_kernel<LGN, 1024, TS, false>), dim3(nfits), dim3(1024), small,
                       s, fits, D, counts, done_list, tab);
  return hipGetLastError();
}

template <int LGN>
hipError_t outer_b(const Item* fits, int nfits, int pmax, const FitDesc* D, int* counts,
                   const Twiddles& tw, hipStream_t s) {
  const bool mlds = refine_lds(LGN, pmax);
  hipLaunchKernelGGL((refine_outer_b_kernel<LGN, 256>), dim3(nfits), dim3(256),
                     refine_shm(pmax, mlds), s, fits, D, counts,
                     static_cast<const cx<double>*>(tw.d64), mlds);
  return hipGetLastError();
}

template <int LGN>
hipError_t cg_b(const Item* fits, int nfits, int pmax, const FitDesc* D, int* counts,
                const Twiddles& tw, hipStream_t s) {
  const bool mlds = refine_lds(LGN, pmax);
  hipLaunchKernelGGL((refine_cg_b_kernel<LGN, 256>), dim3(nfits), dim3(256), refine_shm(pmax, mlds),
                     s, fits, D, counts, static_cast<const cx<double>*>(tw.d64), mlds);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lsqr_step_b(int prec, int lgn, const Item* fits, int nfits, int pmax, bool mlds,
                              const FitDesc* D, int* counts, int* done_list, const Twiddles& tw,
                              hipStream_t s) {
  if (nfits < 1) return hipSuccess;
#define TLS_STEP_B(LG)                                                                         \
  (prec == PREC_F64 ? step_b<LG, double>(fits, nfits, pmax, mlds, D, counts, done_list, tw, s) \
                    : step_b<LG, float>(fits, nfits, pmax, mlds, D, counts, done_list, tw, s))
  TLS_LG_SWITCH(TLS_STEP_B)
#undef TLS_STEP_B
}

hipError_t launch_refine_outer_b(int lgn, const Item* fits, int nfits, int pmax, const FitDesc* D,
                                 int* counts, const Twiddles& tw, hipStream_t s) {
  if (nfits < 1) return hipSuccess;
#define TLS_OUTER_B(LG) outer_b<LG>(fits, nfits, pmax, D, counts, tw, s)
  TLS_LG_SWITCH(TLS_OUTER_B)
#undef TLS_OUTER_B
}

hipError_t launch_refine_cg_b(int lgn, const Item* fits, int nfits, int pmax, const FitDesc* D,
                              int* counts, const Twiddles& tw, hipStream_t s) {
  if (nfits < 1) return hipSuccess;
#define TLS_CG_B(LG) cg_b<LG>(fits, nfits, pmax, D, counts, tw, s)
  TLS_LG_SWITCH(TLS_CG_B)
#undef TLS_CG_B
}

}  // namespace tls
