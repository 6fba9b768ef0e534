// p-side step of R-preconditioned LSQR (Paige and Saunders, ACM TOMS 8(1),
// 1982) on A = X M, M = R^{-1}, one workgroup per fit.
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
// kept); iteration limit (istop 7).
#include <math.h>

#include "fft.h"
#include "kernels.h"

namespace tls {

namespace {

// out[r] = sum_{c in [lo(r), p)} Mrow[r][c] x[c] for the rows r of an upper
// (lo(r) = r) or lower (lo = 0, hi(r) = r + 1) triangular p x p row-major
// matrix; one wavefront per row, four rows in flight, lanes over columns.
// Results go to out[r] (lane 0 of the owning wave) via the callback.
template <int NT, bool UPPER, typename F>
__device__ __forceinline__ void tri_gemv_rows(const double* __restrict__ Mrow, int p,
                                              const double* __restrict__ x, F&& emit) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  for (int r0 = wid * 4; r0 < p; r0 += NW * 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u;
      if (r < p) {
        const double* row = Mrow + static_cast<size_t>(r) * p;
        const int lo = UPPER ? r : 0, hi = UPPER ? p : r + 1;
        for (int c = lo + lane; c < hi; c += 64) acc[u] += row[c] * x[c];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = wave_sum(acc[u]);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (r0 + u < p) emit(r0 + u, acc[u]);
    }
  }
}

// MLDS: M (p <= 128) is staged once into LDS (rows padded to an odd length)
// and every product with M or M^T reads it there.
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
                                                       const cx<double>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  __shared__ cx<double> s[N];
  extern __shared__ double smem[];
  double* sg = smem;
  double* sv = sg + p;
  double* sM = sv + p;  // MLDS: p x ldm
  const int ldm = p | 1;
  __shared__ double red[NT / 64];
  if (st->done) return;
  const int tid = threadIdx.x;
  const bool init = st->phase == 0;
  const double tol = st->tol;
  if constexpr (MLDS) {
    for (int e = tid; e < p * p; e += NT) sM[(e / p) * ldm + e % p] = M[e];
  }

  const double beta = sqrt(g[p]);
  const double invbeta = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = tid; i < p; i += NT) sg[i] = g[i] * invbeta;
  __syncthreads();

  // v~ = M^T (X^T u) - beta v: row j of M^T (= column j of M) is Mt[j][0..j]
  double hsq = 0.0;
  if constexpr (MLDS) {
    for (int j = tid; j < p; j += NT) {
      double a0 = 0.0, a1 = 0.0;
      int i = 0;
      for (; i + 1 <= j; i += 2) {
        a0 += sM[i * ldm + j] * sg[i];
        a1 += sM[(i + 1) * ldm + j] * sg[i + 1];
      }
      if (i <= j) a0 += sM[i * ldm + j] * sg[i];
      const double acc = a0 + a1;
      const double h = init ? acc : acc - beta * v[j];
      sv[j] = h;
      hsq += h * h;
    }
  } else {
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

  double alpha_prev = st->alpha;
  double rhobar = st->rhobar, phibar = st->phibar, anorm2 = st->anorm2, bnorm = st->bnorm;
  double rnorm, arnorm, znorm = st->znorm;
  int iter = st->iter, istop = 0;
  bool done = false;
  if (init) {
    bnorm = beta;
    phibar = beta;
    rhobar = alpha;
    anorm2 = 0.0;
    for (int j = tid; j < p; j += NT) {
      w[j] = sv[j];
      z[j] = 0.0;
    }
    rnorm = beta;
    arnorm = alpha * beta;
    znorm = 0.0;
    if (arnorm == 0.0) {
      done = true;
      istop = 0;
    }
  } else if (!isfinite(alpha) || !isfinite(beta)) {
    // numerical breakdown: keep the last finite iterate
    done = true;
    istop = 4;
    iter += 1;
    rnorm = st->rnorm;
    arnorm = st->arnorm;
  } else {
    anorm2 += alpha_prev * alpha_prev + beta * beta;
    const double rho = hypot(rhobar, beta);
    const double c = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    rhobar = -c * alpha;
    const double phik = c * phibar;
    phibar = sn * phibar;
    const double t1 = phik / rho, t2 = -theta / rho;
    double zsq = 0.0;
    for (int j = tid; j < p; j += NT) {
      const double wj = w[j];
      const double zj = z[j] + t1 * wj;
      z[j] = zj;
      w[j] = sv[j] + t2 * wj;
      zsq += zj * zj;
    }
    znorm = sqrt(block_sum<NT>(zsq, red));
    rnorm = phibar;
    arnorm = phibar * alpha * fabs(c);
    const double anorm = sqrt(anorm2);
    iter += 1;
    if (arnorm <= tol * anorm * rnorm) {
      done = true;
      istop = 2;
    } else if (rnorm <= tol * bnorm + tol * anorm * znorm) {
      done = true;
      istop = 1;
    } else if (alpha == 0.0 || beta == 0.0) {
      done = true;
      istop = 3;
    } else if (iter >= st->max_iter) {
      done = true;
      istop = 7;
    }
  }
  __syncthreads();

  if (!done) {
    // q = M v_new into sg, then its packed spectrum scaled by 1/B.
    if constexpr (MLDS) {
      for (int i = tid; i < p; i += NT) {
        double a0 = 0.0, a1 = 0.0;
        int j = i;
        for (; j + 1 < p; j += 2) {
          a0 += sM[i * ldm + j] * sv[j];
          a1 += sM[i * ldm + j + 1] * sv[j + 1];
        }
        if (j < p) a0 += sM[i * ldm + j] * sv[j];
        sg[i] = a0 + a1;
      }
    } else {
      tri_gemv_rows<NT, true>(M, p, sv, [&](int i, double acc) { sg[i] = acc; });
    }
    __syncthreads();
    for (int t = tid; t < N; t += NT) {
      const int i0 = 2 * t;
      s[swz<double>(t)] = {i0 < p ? sg[i0] : 0.0, i0 + 1 < p ? sg[i0 + 1] : 0.0};
    }
    __syncthreads();
    fft_dif<double, false, LGN, NT>(s, tab);
    const double invB = 1.0 / static_cast<double>(2 * N);
    for (int k = tid; k <= N / 2; k += NT) {
      const cx<double> wk = twiddle<double, false>(tab, k, LGN + 1);
      cx<double> Xk, Xnk;
      rfft_post(s[swz<double>(bitrev(k, LGN))], s[swz<double>(bitrev((N - k) & (N - 1), LGN))], wk, Xk, Xnk);
      Xk = cscale(Xk, invB);
      Xnk = cscale(Xnk, invB);
      if (k == 0) {
        Vhat[0] = {static_cast<TS>(Xk.x), static_cast<TS>(Xnk.x)};
      } else {
        Vhat[k] = {static_cast<TS>(Xk.x), static_cast<TS>(Xk.y)};
        if (2 * k != N) Vhat[N - k] = {static_cast<TS>(Xnk.x), static_cast<TS>(Xnk.y)};
      }
    }
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
  if (tid == 0) {
    st->alpha = alpha;
    st->beta = beta;
    st->rhobar = rhobar;
    st->phibar = phibar;
    st->anorm2 = anorm2;
    st->bnorm = bnorm;
    st->rnorm = rnorm;
    st->arnorm = arnorm;
    st->znorm = znorm;
    st->iter = iter;
    st->istop = istop;
    st->phase = 1;
    st->coef[0] = 1.0;
    st->coef[1] = beta > 0.0 ? -alpha / beta : 0.0;
    if (done) st->done = 1;
  }
}

template <int LGN, typename TS>
hipError_t step_one(int p, LsqrState* st, const double* g, const double* M, const double* Mt,
                    double* v, double* w, double* z, const double* phi0, double* phi, void* Vhat,
                    const Twiddles& tw, hipStream_t stream) {
  constexpr int NT = 256;
  const size_t small = 2 * static_cast<size_t>(p) * sizeof(double);
  const size_t with_m = small + static_cast<size_t>(p) * (p | 1) * sizeof(double);
  const size_t lds_static = static_cast<size_t>(1 << LGN) * 16 + 64;
  if (p <= 128 && with_m + lds_static <= 160 * 1024) {
    hipLaunchKernelGGL((lsqr_step_kernel<LGN, NT, TS, true>), dim3(1), dim3(NT), with_m, stream, p,
                       st, g, M, Mt, v, w, z, phi0, phi, static_cast<cx<TS>*>(Vhat),
                       static_cast<const cx<double>*>(tw.d64));
  } else {
    hipLaunchKernelGGL((lsqr_step_kernel<LGN, NT, TS, false>), dim3(1), dim3(NT), small, stream, p,
                       st, g, M, Mt, v, w, z, phi0, phi, static_cast<cx<TS>*>(Vhat),
                       static_cast<const cx<double>*>(tw.d64));
  }
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
                            const double* phi0, double* phi, void* Vhat, const Twiddles& tw,
                            hipStream_t stream) {
  const size_t shm = (2 * static_cast<size_t>(1 << lgn) + 2 * p) * sizeof(double);
  if (shm > 160 * 1024) return hipErrorInvalidValue;
#define TLS_STEP_CASE(LG)                                                                       \
  case LG:                                                                                      \
    return prec == PREC_F64                                                                     \
               ? step_one<LG, double>(p, st, g, M, Mt, v, w, z, phi0, phi, Vhat, tw, stream)   \
               : step_one<LG, float>(p, st, g, M, Mt, v, w, z, phi0, phi, Vhat, tw, stream);
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

// out = y0 + M x for upper-triangular M given as Mt = M^T (row-major).
hipError_t launch_vec_axpy_small(const double* Mt, const double* x, const double* y0, int p,
                                 double* out, hipStream_t st) {
  hipLaunchKernelGGL(gemv_upper_kernel, dim3(1), dim3(256), 0, st, Mt, x, y0, p, out);
  return hipGetLastError();
}

}  // namespace tls
