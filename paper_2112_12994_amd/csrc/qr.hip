// QR factorisation of the sketch [S X | S b] (Section 2.1: the compressed
// problem is solved through a QR factorisation of SA) by shifted Cholesky QR
// in three sweeps (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J.
// Sci. Comput. 2020): G = A^T A + s I -> R1, A <- A R1^{-1}; G = A^T A -> R2,
// A <- A R2^{-1}; G = A^T A -> R3; R = R3 R2 R1.  The shift
// s = 11 (c q + q (q + 1)) u trace(A^T A) keeps the first Cholesky factorable
// up to condition numbers near 1/u; the later sweeps restore orthogonality.
// Near that limit the first sweep can leave kappa(A R1^{-1}) ~ 1e8, where the
// unshifted Gram matrix is on the edge of breakdown; a later sweep whose
// Cholesky breaks down is therefore redone with the shift.  After the second
// sweep, A R1^{-1} R2^{-1} is orthonormal to O(u kappa(A R1^{-1})^2); the
// third sweep runs only when the second Cholesky needed the shift or its
// pivots spanned more than 1e4 (status bit 8), otherwise R = R2 R1.
// Every Gram matrix is a dense contraction over the c rows, computed on the
// FP64 matrix cores (V_MFMA_F64_16X16X4_F64).
//
// Layout: A row-major, crows x ldq (crows a multiple of 4, ldq a multiple of
// 16; padding rows and columns are zero).  R, R1, R2: q x q row-major upper
// triangular.  status bits: 1 = first Cholesky broke down, 2 = a later
// Cholesky broke down, 4 = min|R_ii| <= q u max|R_ii|; 2 or 4 mean [S X | S b]
// is numerically rank deficient.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace tls {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// One 16x16 tile (ti <= tj) of G = A^T A per workgroup of 4 wavefronts; the
// waves take interleaved 4-row steps and their tiles are summed in a fixed order.
__device__ __forceinline__ void gram_body(const double* __restrict__ A, int crows, int ldq,
                                                   double* __restrict__ G, int tile) {
  const int nt = ldq / 16;
  const int ti = tile / nt, tj = tile % nt;
  if (ti > tj) return;
  __shared__ double part[4][16][17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ci = ti * 16 + (lane & 15);
  const int cj = tj * 16 + (lane & 15);
  const int kr = lane >> 4;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = wv * 4; r0 < crows; r0 += 16) {
    const double* row = A + static_cast<size_t>(r0 + kr) * ldq;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(row[ci], row[cj], acc, 0, 0, 0);
  }
  // output register v of lane l holds D[i][j] with i = 4 v + l / 16, j = l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wv][4 * v + (lane >> 4)][lane & 15] = acc[v];
  __syncthreads();
  const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
  const double s = ((part[0][i][j] + part[1][i][j]) + part[2][i][j]) + part[3][i][j];
  const int gi = ti * 16 + i, gj = tj * 16 + j;
  G[static_cast<size_t>(gi) * ldq + gj] = s;
  G[static_cast<size_t>(gj) * ldq + gi] = s;
}

__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ A, int crows, int ldq,
                                                   double* __restrict__ G) {
  gram_body(A, crows, ldq, G, blockIdx.x);
}

// Right-looking Cholesky of G[:q,:q] (+ shift on the diagonal) into the upper
// factor R (row-major q x q, zero below the diagonal).  One workgroup; the
// working copy lives in R.
// After a refining sweep, A R^{-1} is orthonormal to about u kappa^2, kappa
// the condition number of that sweep's input.  Its pivots (R_jj^2) give only
// a lower bound on kappa^2 (by about 1e6 on ill-conditioned lag sketches), so
// the next sweep is enabled (status bit 8) as soon as they span more than 1e4:
// well-conditioned inputs (R near the identity) skip it.
__device__ __forceinline__ bool needs_third_sweep(double dmin, double dmax) {
  return !(dmax <= 1e4 * dmin);
}

template <int NT>
__device__ __forceinline__ void chol_body(const double* __restrict__ G, int ldq, int q,
                                                  int crows, int shift, double* __restrict__ R,
                                                  int* __restrict__ status, int fail_bit,
                                                  int rank_cols) {
  __shared__ double red[NT / 64];
  __shared__ double s_shift, s_floor;
  double tr = 0.0;
  for (int i = threadIdx.x; i < q; i += NT) tr += G[static_cast<size_t>(i) * ldq + i];
  tr = block_sum<NT>(tr, red);
  if (threadIdx.x == 0) {
    s_shift = 11.0 * (static_cast<double>(crows) * q + static_cast<double>(q) * (q + 1)) * 0x1p-53 * tr;
    s_floor = tr > 0.0 ? tr * 0x1p-104 : 1e-300;
  }
  bool failed = false;
  double dmin = INFINITY, dmax = 0.0;
  for (int attempt = (shift == 1 ? 1 : 0); attempt < 2; ++attempt) {
  failed = false;
  dmin = INFINITY;
  dmax = 0.0;
  for (int e = threadIdx.x; e < q * q; e += NT) {
    const int i = e / q, k = e % q;
    R[e] = (k >= i) ? G[static_cast<size_t>(i) * ldq + k] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0 && attempt)
    for (int i = 0; i < q; ++i) R[static_cast<size_t>(i) * q + i] += s_shift;
  __syncthreads();
  for (int j = 0; j < q; ++j) {
    double d = R[static_cast<size_t>(j) * q + j];
    if (!(d > s_floor)) {
      if (j < rank_cols) failed = true;  // later columns may be exactly dependent (b in range)
      d = s_floor;
    }
    if (j < rank_cols) {
      dmin = fmin(dmin, d);
      dmax = fmax(dmax, d);
    }
    const double rjj = sqrt(d);
    const double inv = 1.0 / rjj;
    __syncthreads();
    for (int k = j + 1 + threadIdx.x; k < q; k += NT) R[static_cast<size_t>(j) * q + k] *= inv;
    if (threadIdx.x == 0) R[static_cast<size_t>(j) * q + j] = rjj;
    __syncthreads();
    const int w = q - j - 1;
    const double* rj = R + static_cast<size_t>(j) * q;
    for (int e = threadIdx.x; e < w * w; e += NT) {
      const int ii = j + 1 + e / w, kk = j + 1 + e % w;
      if (kk >= ii) R[static_cast<size_t>(ii) * q + kk] -= rj[ii] * rj[kk];
    }
    __syncthreads();
  }
  if (!failed || shift != 2 || attempt == 1) {
    if (shift == 2 && threadIdx.x == 0 && (attempt == 1 || needs_third_sweep(dmin, dmax)))
      atomicOr(status, 8);
    break;
  }
  __syncthreads();
  }
  if (failed && threadIdx.x == 0) atomicOr(status, fail_bit);
}

template <int NT>
__global__ __launch_bounds__(NT) void chol_kernel(const double* __restrict__ G, int ldq, int q,
                                                  int crows, int shift, double* __restrict__ R,
                                                  int* __restrict__ status, int fail_bit,
                                                  int rank_cols, const int* __restrict__ gate) {
  if (gate && !(*gate & 8)) return;
  chol_body<NT>(G, ldq, q, crows, shift, R, status, fail_bit, rank_cols);
}

// A <- A R^{-1} on the first q columns (each thread owns one row).
template <int ROWS, int QMAX>
__global__ __launch_bounds__(ROWS) void trsm_kernel(double* __restrict__ A, int crows, int ldq,
                                                    int q, const double* __restrict__ R) {
  __shared__ double ra[QMAX * ROWS];
  const int t = blockIdx.x * ROWS + threadIdx.x;
  const bool live = t < crows;
  double* row = A + static_cast<size_t>(t) * ldq;
  for (int k = 0; k < q; ++k) ra[k * ROWS + threadIdx.x] = live ? row[k] : 0.0;
  for (int j = 0; j < q; ++j) {
    const double* rj = R + static_cast<size_t>(j) * q;
    const double x = ra[j * ROWS + threadIdx.x] / rj[j];
    ra[j * ROWS + threadIdx.x] = x;
    for (int k = j + 1; k < q; ++k) ra[k * ROWS + threadIdx.x] -= x * rj[k];
  }
  if (live)
    for (int k = 0; k < q; ++k) row[k] = ra[k * ROWS + threadIdx.x];
}

// Same, rows kept in place in global memory (large q).
__device__ __forceinline__ void trsm_global_body(double* __restrict__ A, int crows, int ldq,
                                                         int q, const double* __restrict__ R, int blk) {
  const int t = blk * 64 + threadIdx.x;
  if (t >= crows) return;
  double* row = A + static_cast<size_t>(t) * ldq;
  for (int j = 0; j < q; ++j) {
    const double* rj = R + static_cast<size_t>(j) * q;
    const double x = row[j] / rj[j];
    row[j] = x;
    for (int k = j + 1; k < q; ++k) row[k] -= x * rj[k];
  }
}

__global__ __launch_bounds__(64) void trsm_global_kernel(double* __restrict__ A, int crows, int ldq,
                                                         int q, const double* __restrict__ R) {
  trsm_global_body(A, crows, ldq, q, R, blockIdx.x);
}

// C = Ra Rb for upper-triangular q x q (row-major); one workgroup per row.
template <int NT>
__device__ __forceinline__ void trmm_body(const double* __restrict__ Ra,
                                                  const double* __restrict__ Rb, int q,
                                                  double* __restrict__ C, int i) {
  const double* ra = Ra + static_cast<size_t>(i) * q;
  for (int j = threadIdx.x; j < q; j += NT) {
    double acc = 0.0;
    for (int k = i; k <= j; ++k) acc += ra[k] * Rb[static_cast<size_t>(k) * q + j];
    C[static_cast<size_t>(i) * q + j] = acc;
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void trmm_kernel(const double* __restrict__ Ra,
                                                  const double* __restrict__ Rb, int q,
                                                  double* __restrict__ C) {
  trmm_body<NT>(Ra, Rb, q, C, blockIdx.x);
}

// M = R[:p,:p]^{-1} (row-major, upper), Mt = M^T, phi0 = M R[:p, p] (the
// compressed problem's solution), and the rank test min|R_ii| <= p u max|R_ii|.
template <int NT>
__device__ __forceinline__ void triinv_body(const double* __restrict__ R, int q, int p,
                                                    double* __restrict__ M, double* __restrict__ Mt,
                                                    double* __restrict__ phi0,
                                                    int* __restrict__ status) {
  __shared__ double red[NT / 64];
  for (int e = threadIdx.x; e < p * p; e += NT) M[e] = 0.0;
  __syncthreads();
  for (int i = p - 1; i >= 0; --i) {
    const double* ri = R + static_cast<size_t>(i) * q;
    const double inv = 1.0 / ri[i];
    for (int j = i + threadIdx.x; j < p; j += NT) {
      double acc = (j == i) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) acc -= ri[k] * M[static_cast<size_t>(k) * p + j];
      M[static_cast<size_t>(i) * p + j] = acc * inv;
    }
    __syncthreads();
  }
  {
    // Mt = M^T: one wavefront per row of M, lanes over its columns
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < p; i += NT / 64)
      for (int j = lane; j < p; j += 64) Mt[static_cast<size_t>(j) * p + i] = M[static_cast<size_t>(i) * p + j];
  }
  if (phi0 && q > p) {
    for (int i = threadIdx.x; i < p; i += NT) {
      double acc = 0.0;
      for (int j = i; j < p; ++j) acc += M[static_cast<size_t>(i) * p + j] * R[static_cast<size_t>(j) * q + p];
      phi0[i] = acc;
    }
  }
  double dmax = 0.0, dmin = INFINITY;
  for (int i = threadIdx.x; i < p; i += NT) {
    const double d = fabs(R[static_cast<size_t>(i) * q + i]);
    dmax = fmax(dmax, d);
    dmin = fmin(dmin, d);
  }
  // block max / min via two sums of one-hot contributions would lose order; use LDS.
  __shared__ double smax[NT], smin[NT];
  smax[threadIdx.x] = dmax;
  smin[threadIdx.x] = dmin;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = INFINITY;
    for (int t = 0; t < NT; ++t) {
      a = fmax(a, smax[t]);
      b = fmin(b, smin[t]);
    }
    if (!(b > static_cast<double>(p) * 0x1p-53 * a)) atomicOr(status, 4);
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void triinv_kernel(const double* __restrict__ R, int q, int p,
                                                    double* __restrict__ M, double* __restrict__ Mt,
                                                    double* __restrict__ phi0,
                                                    int* __restrict__ status) {
  triinv_body<NT>(R, q, p, M, Mt, phi0, status);
}

// ---- LDS-resident variants for q <= 128 (the whole q x q matrix in LDS) ----

// ---- register-tiled variants for q <= 16 QT (QT <= 8) ---------------------
// Thread (tx, ty) of 256 owns the elements (ty + 16 a, tx + 16 b) of the q x q
// matrix in registers; the row a step needs is published through a
// double-buffered LDS row, so a step costs one barrier and register FMAs.

// Cholesky G[:q,:q] (+ shift) = R^T R.  shift_mode 1: always shifted; 2: unshifted, redone
// with the shift on breakdown.
template <int QT, int TD = 16>
__device__ __forceinline__ void chol_reg_body(const double* __restrict__ G, int ldq, int q,
                                                       int crows, int shift_mode,
                                                       double* __restrict__ R,
                                                       int* __restrict__ status, int fail_bit,
                                                       int rank_cols) {
  constexpr int NT = TD * TD;
  __shared__ double pub[2][TD * QT];
  __shared__ double red[NT / 64];
  __shared__ int s_fail;
  const int tx = threadIdx.x % TD, ty = threadIdx.x / TD;
  double tr = 0.0;
  for (int i = threadIdx.x; i < q; i += NT) tr += G[static_cast<size_t>(i) * ldq + i];
  tr = block_sum<NT>(tr, red);
  const double shift_amount =
      11.0 * (static_cast<double>(crows) * q + static_cast<double>(q) * (q + 1)) * 0x1p-53 * tr;
  const double floor_ = tr > 0.0 ? tr * 0x1p-104 : 1e-300;
  double reg[QT][QT];
  for (int attempt = (shift_mode == 1 ? 1 : 0); attempt < 2; ++attempt) {
    const double sh = attempt ? shift_amount : 0.0;
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int b = 0; b < QT; ++b) {
        const int i = ty + TD * a, k = tx + TD * b;
        reg[a][b] = (i < q && k < q) ? G[static_cast<size_t>(i) * ldq + k] + (i == k ? sh : 0.0) : 0.0;
      }
    if (threadIdx.x == 0) s_fail = 0;
    __syncthreads();
    double dmin = INFINITY, dmax = 0.0;
    // column j = TD a0 + jj: tiles left of / above tile a0 are final (row j's
    // multipliers vanish there), so the register tile indices are static
#pragma unroll
    for (int a0 = 0; a0 < QT; ++a0) {
      for (int jj = 0; jj < TD; ++jj) {
        const int j = TD * a0 + jj;
        if (j >= q) break;
        double* pj = pub[j & 1];
        if (ty == jj) {
#pragma unroll
          for (int b = a0; b < QT; ++b) pj[tx + TD * b] = reg[a0][b];
        }
        __syncthreads();
        double d = pj[j];
        if (!(d > floor_)) {
          if (j < rank_cols && threadIdx.x == 0) s_fail = 1;
          d = floor_;
        }
        if (j < rank_cols) {
          dmin = fmin(dmin, d);
          dmax = fmax(dmax, d);
        }
        // independent operations (shortest dependent chain per column)
        const double invd = 1.0 / d;
        const double isd = 1.0 / sqrt(d);
        const double sd = sqrt(d);
        // row j of R stays in the registers of its owner (not updated again);
        // R is written once after the last column
        if (ty == jj) {
#pragma unroll
          for (int b = a0; b < QT; ++b) {
            const int k = tx + TD * b;
            reg[a0][b] = k < j ? 0.0 : (k == j ? sd : reg[a0][b] * isd);
          }
        }
        // rank-one update of the trailing rows and columns (index > j); pub
        // entries beyond q are zero
        double fi[QT], fk[QT];
#pragma unroll
        for (int a = a0; a < QT; ++a) {
          const double v = pj[ty + TD * a] * invd;
          fi[a] = (a > a0 || ty > jj) ? v : 0.0;
        }
#pragma unroll
        for (int b = a0; b < QT; ++b) {
          const double v = pj[tx + TD * b];
          fk[b] = (b > a0 || tx > jj) ? v : 0.0;
        }
#pragma unroll
        for (int a = a0; a < QT; ++a)
#pragma unroll
          for (int b = a0; b < QT; ++b) reg[a][b] -= fi[a] * fk[b];
      }
    }
    __syncthreads();
    const int failed = s_fail;
    // R (q x q, row-major, zero below the diagonal) from the register tiles
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int b = 0; b < QT; ++b) {
        const int i = ty + TD * a, k = tx + TD * b;
        if (i < q && k < q) R[static_cast<size_t>(i) * q + k] = k < i ? 0.0 : reg[a][b];
      }
    if (!failed || shift_mode != 2 || attempt == 1) {
      if (failed && threadIdx.x == 0) atomicOr(status, fail_bit);
      if (shift_mode == 2 && threadIdx.x == 0 && (attempt == 1 || needs_third_sweep(dmin, dmax)))
        atomicOr(status, 8);
      break;
    }
    __syncthreads();
  }
}

template <int QT>
__global__ __launch_bounds__(256) void chol_reg_kernel(const double* __restrict__ G, int ldq, int q,
                                                       int crows, int shift_mode,
                                                       double* __restrict__ R,
                                                       int* __restrict__ status, int fail_bit,
                                                       int rank_cols, const int* __restrict__ gate) {
  if (gate && !(*gate & 8)) return;
  chol_reg_body<QT>(G, ldq, q, crows, shift_mode, R, status, fail_bit, rank_cols);
}

// 128 < q <= 224: a 32 x 32 thread grid, QT = ceil(q / 32) register tiles.
template <int QT>
__global__ __launch_bounds__(1024) void chol_reg32_kernel(const double* __restrict__ G, int ldq,
                                                          int q, int crows, int shift_mode,
                                                          double* __restrict__ R,
                                                          int* __restrict__ status, int fail_bit,
                                                          int rank_cols,
                                                          const int* __restrict__ gate) {
  if (gate && !(*gate & 8)) return;
  chol_reg_body<QT, 32>(G, ldq, q, crows, shift_mode, R, status, fail_bit, rank_cols);
}

// M = R[:n,:n]^{-1} (upper; row-major, leading dimension ldm, zero elsewhere
// in the ldm x ldm block): M = I, then for i = n-1 .. 0, row i of M is
// divided by R_ii and R[r][i] times it is subtracted from every row r < i.
template <int QT>
__device__ __forceinline__ void triinv_reg_body(const double* __restrict__ R, int ldr, int n,
                                                         double* __restrict__ M, int ldm) {
  extern __shared__ double Rs[];  // n x (n + 1)
  __shared__ double pub[2][16 * QT];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int ld = n + 1;
  {
    // one wavefront per 8 rows, lanes over columns, 8 loads in flight
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int r0 = wid * 8; r0 < n; r0 += 32)
      for (int c = lane; c < n; c += 64) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = r0 + u < n ? R[static_cast<size_t>(r0 + u) * ldr + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (r0 + u < n) Rs[(r0 + u) * ld + c] = v[u];
      }
  }
  double reg[QT][QT];
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b) reg[a][b] = (ty + 16 * a == tx + 16 * b && ty + 16 * a < n) ? 1.0 : 0.0;
  __syncthreads();
  // row i = 16 a0 + ii, from the last: row i of M (nonzero from column i on)
  // is final once divided by R_ii, then subtracted from the rows above it;
  // the register tile indices are static
#pragma unroll
  for (int a0 = QT - 1; a0 >= 0; --a0) {
    for (int ii = 15; ii >= 0; --ii) {
      const int i = 16 * a0 + ii;
      if (i >= n) continue;
      double* pi = pub[i & 1];
      const double inv = 1.0 / Rs[i * ld + i];
      if (ty == ii) {
#pragma unroll
        for (int b = a0; b < QT; ++b) {
          reg[a0][b] *= inv;
          pi[tx + 16 * b] = reg[a0][b];
        }
      }
      __syncthreads();
      double ri[QT], mc[QT];
#pragma unroll
      for (int a = 0; a <= a0; ++a) {
        const int r = ty + 16 * a;
        ri[a] = (a < a0 || ty < ii) ? Rs[r * ld + i] : 0.0;
      }
#pragma unroll
      for (int b = a0; b < QT; ++b) {
        const int c = tx + 16 * b;
        mc[b] = c < n ? pi[c] : 0.0;
      }
#pragma unroll
      for (int a = 0; a <= a0; ++a)
#pragma unroll
        for (int b = a0; b < QT; ++b) reg[a][b] -= ri[a] * mc[b];
    }
  }
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b) {
      const int r = ty + 16 * a, c = tx + 16 * b;
      if (r < ldm && c < ldm) M[static_cast<size_t>(r) * ldm + c] = (r < n && c < n) ? reg[a][b] : 0.0;
    }
  // rows / columns of the ldm block beyond 16 QT (only when ldm > 16 QT)
  if (ldm > 16 * QT)
    for (int e = threadIdx.x; e < ldm * ldm; e += 256) {
      const int r = e / ldm, c = e % ldm;
      if (r >= 16 * QT || c >= 16 * QT) M[e] = 0.0;
    }
}

template <int QT>
__global__ __launch_bounds__(256) void triinv_reg_kernel(const double* __restrict__ R, int ldr, int n,
                                                         double* __restrict__ M, int ldm) {
  triinv_reg_body<QT>(R, ldr, n, M, ldm);
}

// A <- A R^{-1} on the first q columns, 16 rows per wavefront (rows are
// independent).  Blocked by 16 columns as in LAPACK's triangular solve: the
// 16 x 16 diagonal block by forward substitution (one lane per row), then the
// trailing columns A[:, K] -= X[:, J] R[J, K] on the FP64 matrix cores.
// Backward stable, unlike a product with an explicitly inverted R.
__device__ __forceinline__ void trsm_tile_body(double* __restrict__ A, int ldq, int q,
                                                       const double* __restrict__ R, int rt) {
  extern __shared__ double T[];  // 16 x (ldq + 1) rows of A, then 16 x ldq rows of R
  const int ld = ldq + 1;
  double* Rp = T + 16 * ld;
  const int lane = threadIdx.x;
  const size_t r0 = static_cast<size_t>(rt) * 16;
  // the 16 rows of A: lanes over columns, 16 rows' loads in flight
  for (int c = lane; c < ldq; c += 64) {
    double v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = A[(r0 + r) * ldq + c];
#pragma unroll
    for (int r = 0; r < 16; ++r) T[r * ld + c] = v[r];
  }
  const int nt = (q + 15) / 16;
  for (int J = 0; J < nt; ++J) {
    const int j0 = J * 16;
    // rows j0 .. j0+15 of R from column j0 on (zero outside q x q; R is
    // upper triangular, so nothing left of j0 is read)
    for (int cc = j0 + lane; cc < ldq; cc += 64) {
      double v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r)
        v[r] = (j0 + r < q && cc < q) ? R[static_cast<size_t>(j0 + r) * q + cc] : 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) Rp[r * ldq + cc] = v[r];
    }
    __syncthreads();
    if (lane < 16) {
      double* row = T + lane * ld;
      for (int jj = 0; jj < 16 && j0 + jj < q; ++jj) {
        const double* rj = Rp + jj * ldq;
        const double x = row[j0 + jj] / rj[j0 + jj];
        row[j0 + jj] = x;
        for (int kk = jj + 1; kk < 16 && j0 + kk < q; ++kk) row[j0 + kk] -= x * rj[j0 + kk];
      }
    }
    __syncthreads();
    for (int K = J + 1; K < nt; ++K) {
      const int k0 = K * 16;
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = T[(4 * v + (lane >> 4)) * ld + k0 + (lane & 15)];
#pragma unroll
      for (int k4 = 0; k4 < 16; k4 += 4) {
        const double xa = -T[(lane & 15) * ld + j0 + k4 + (lane >> 4)];
        const double rb = Rp[(k4 + (lane >> 4)) * ldq + k0 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, rb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) T[(4 * v + (lane >> 4)) * ld + k0 + (lane & 15)] = acc[v];
    }
    __syncthreads();
  }
  for (int c = lane; c < ldq; c += 64) {
#pragma unroll
    for (int r = 0; r < 16; ++r) A[(r0 + r) * ldq + c] = T[r * ld + c];
  }
}

__global__ __launch_bounds__(64) void trsm_tile_kernel(double* __restrict__ A, int ldq, int q,
                                                       const double* __restrict__ R) {
  trsm_tile_body(A, ldq, q, R, blockIdx.x);
}

// status |= 4 when min|R_ii| <= k u max|R_ii| over the first k = rank_cols
// diagonal entries (numerical rank of the leading columns below k).
__device__ __forceinline__ void rank_test_body(const double* __restrict__ R, int q,
                                                       int rank_cols, int* __restrict__ status) {
  double a = 0.0, b = INFINITY;
  for (int i = threadIdx.x; i < rank_cols; i += 64) {
    const double d = fabs(R[static_cast<size_t>(i) * q + i]);
    a = fmax(a, d);
    b = fmin(b, d);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, 64));
    b = fmin(b, __shfl_xor(b, off, 64));
  }
  if (threadIdx.x == 0 && !(b > static_cast<double>(rank_cols) * 0x1p-53 * a)) atomicOr(status, 4);
}

__global__ __launch_bounds__(64) void rank_test_kernel(const double* __restrict__ R, int q,
                                                       int rank_cols, int* __restrict__ status) {
  rank_test_body(R, q, rank_cols, status);
}

// Tail of the preconditioner set-up once M = R[:p,:p]^{-1} exists: Mt = M^T,
// phi0 = M R[:p, p], rank test on R[:p,:p] (status |= 4).
// M = R[:n,:n]^{-1} for 128 < n <= 224 on a 32 x 32 thread grid with QT =
// ceil(n / 32) register tiles; the algorithm of triinv_reg_body, with the
// columns of R staged in LDS 32 at a time (n x 33 doubles) instead of all of R.
template <int QT>
__device__ __forceinline__ void triinv_reg32_body(const double* __restrict__ R, int ldr, int n,
                                                  double* __restrict__ M, int ldm) {
  constexpr int TD = 32;
  extern __shared__ double Rc[];  // rows x 33: columns 32 a0 .. 32 a0 + 31 of R
  __shared__ double pub[2][TD * QT];
  const int tx = threadIdx.x % TD, ty = threadIdx.x / TD;
  double reg[QT][QT];
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b) reg[a][b] = (ty + TD * a == tx + TD * b && ty + TD * a < n) ? 1.0 : 0.0;
#pragma unroll
  for (int a0 = QT - 1; a0 >= 0; --a0) {
    const int rows = min(n, TD * a0 + TD);
    __syncthreads();  // the previous chunk is no longer read
    for (int r = ty; r < rows; r += TD) {
      const int c = TD * a0 + tx;
      Rc[r * (TD + 1) + tx] = c < n ? R[static_cast<size_t>(r) * ldr + c] : 0.0;
    }
    __syncthreads();
    for (int ii = TD - 1; ii >= 0; --ii) {
      const int i = TD * a0 + ii;
      if (i >= n) continue;
      double* pi = pub[i & 1];
      const double inv = 1.0 / Rc[i * (TD + 1) + ii];
      if (ty == ii) {
#pragma unroll
        for (int b = a0; b < QT; ++b) {
          reg[a0][b] *= inv;
          pi[tx + TD * b] = reg[a0][b];
        }
      }
      __syncthreads();
      double ri[QT], mc[QT];
#pragma unroll
      for (int a = 0; a <= a0; ++a) {
        const int r = ty + TD * a;
        ri[a] = ((a < a0 || ty < ii) && r < n) ? Rc[r * (TD + 1) + ii] : 0.0;
      }
#pragma unroll
      for (int b = a0; b < QT; ++b) {
        const int c = tx + TD * b;
        mc[b] = c < n ? pi[c] : 0.0;
      }
#pragma unroll
      for (int a = 0; a <= a0; ++a)
#pragma unroll
        for (int b = a0; b < QT; ++b) reg[a][b] -= ri[a] * mc[b];
    }
  }
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b) {
      const int r = ty + TD * a, c = tx + TD * b;
      if (r < ldm && c < ldm) M[static_cast<size_t>(r) * ldm + c] = (r < n && c < n) ? reg[a][b] : 0.0;
    }
}

template <int QT>
__global__ __launch_bounds__(1024) void triinv_reg32_kernel(const double* __restrict__ R, int ldr,
                                                            int n, double* __restrict__ M, int ldm) {
  triinv_reg32_body<QT>(R, ldr, n, M, ldm);
}

template <int NT>
__device__ __forceinline__ void triinv_finish_body(const double* __restrict__ R, int q,
                                                           int p, const double* __restrict__ M,
                                                           double* __restrict__ Mt,
                                                           double* __restrict__ phi0,
                                                           int* __restrict__ status) {
  {
    // Mt = M^T: one wavefront per row of M, lanes over its columns
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < p; i += NT / 64)
      for (int j = lane; j < p; j += 64) Mt[static_cast<size_t>(j) * p + i] = M[static_cast<size_t>(i) * p + j];
  }
  if (phi0 && q > p) {
    for (int i = threadIdx.x; i < p; i += NT) {
      double acc = 0.0;
      for (int j = i; j < p; ++j)
        acc += M[static_cast<size_t>(i) * p + j] * R[static_cast<size_t>(j) * q + p];
      phi0[i] = acc;
    }
  }
  if (threadIdx.x < 64) {
    double a = 0.0, b = INFINITY;
    for (int i = threadIdx.x; i < p; i += 64) {
      const double d = fabs(R[static_cast<size_t>(i) * q + i]);
      a = fmax(a, d);
      b = fmin(b, d);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a = fmax(a, __shfl_xor(a, off, 64));
      b = fmin(b, __shfl_xor(b, off, 64));
    }
    if (threadIdx.x == 0 && status && !(b > static_cast<double>(p) * 0x1p-53 * a))
      atomicOr(status, 4);
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void triinv_finish_kernel(const double* __restrict__ R, int q,
                                                           int p, const double* __restrict__ M,
                                                           double* __restrict__ Mt,
                                                           double* __restrict__ phi0,
                                                           int* __restrict__ status) {
  triinv_finish_body<NT>(R, q, p, M, Mt, phi0, status);
}

}  // namespace

// Scratch: G must hold ldq*ldq + 2*q*q doubles (Gram matrix, then R3 and
// R3 R2); for q <= 128 also ldq*ldq (inverse) + crows*ldq (second copy of A)
// beyond that, i.e. qr_scratch_doubles(crows, q, ldq) in total.
size_t qr_scratch_doubles(int crows, int q, int ldq) {
  return static_cast<size_t>(ldq) * ldq * 2 + 2 * static_cast<size_t>(q) * q +
         static_cast<size_t>(crows) * ldq;
}

namespace {

template <int QT>
void chol_reg_launch(const double* G, int ldq, int q, int crows, int shift_mode, double* R,
                     int* status, int fail_bit, int rank_cols, const int* gate, hipStream_t st) {
  hipLaunchKernelGGL((chol_reg_kernel<QT>), dim3(1), dim3(256), 0, st, G, ldq, q, crows, shift_mode,
                     R, status, fail_bit, rank_cols, gate);
}

// gate: NULL, or run only when bit 8 of *gate is set (the third sweep).
void chol_launch(const double* G, int ldq, int q, int crows, int shift_mode, double* R, int* status,
                 int fail_bit, int rank_cols, const int* gate, hipStream_t st) {
  const int qt = reg_tiles(q);
  switch (qt) {
#define TLS_CHOL_QT(K) \
    case K: chol_reg_launch<K>(G, ldq, q, crows, shift_mode, R, status, fail_bit, rank_cols, gate, st); return;
    TLS_CHOL_QT(1) TLS_CHOL_QT(2) TLS_CHOL_QT(3) TLS_CHOL_QT(4)
    TLS_CHOL_QT(5) TLS_CHOL_QT(6) TLS_CHOL_QT(7) TLS_CHOL_QT(8)
#undef TLS_CHOL_QT
#define TLS_CHOL_QT32(K)                                                                        \
  case 100 + K:                                                                                 \
    hipLaunchKernelGGL((chol_reg32_kernel<K>), dim3(1), dim3(1024), 0, st, G, ldq, q, crows,     \
                       shift_mode, R, status, fail_bit, rank_cols, gate);                        \
    return;
    TLS_CHOL_QT32(5) TLS_CHOL_QT32(6) TLS_CHOL_QT32(7)
#undef TLS_CHOL_QT32
    default:
      hipLaunchKernelGGL((chol_kernel<256>), dim3(1), dim3(256), 0, st, G, ldq, q, crows, shift_mode,
                         R, status, fail_bit, rank_cols, gate);
  }
}

template <int QT>
void triinv_reg_launch(const double* R, int ldr, int n, double* M, int ldm, hipStream_t st) {
  hipLaunchKernelGGL((triinv_reg_kernel<QT>), dim3(1), dim3(256),
                     static_cast<size_t>(n) * (n + 1) * sizeof(double), st, R, ldr, n, M, ldm);
}

}  // namespace

// Triangular inverse of R[:n,:n] into M (n <= 224: register tiles on 16 x 16
// or 32 x 32 thread grids; else the
// global-memory kernel) with leading dimension ldm >= n, zero-padded.
hipError_t tri_inverse(const double* R, int ldr, int n, double* M, int ldm, hipStream_t st) {
  const size_t shm32 = static_cast<size_t>(n) * 33 * sizeof(double);
  switch (reg_tiles(n)) {
#define TLS_TRI32(K)                                                                          \
  case 100 + K:                                                                               \
    hipLaunchKernelGGL((triinv_reg32_kernel<K>), dim3(1), dim3(1024), shm32, st, R, ldr, n, M, \
                       ldm);                                                                  \
    break;
    TLS_TRI32(5) TLS_TRI32(6) TLS_TRI32(7)
#undef TLS_TRI32
    case 1: triinv_reg_launch<1>(R, ldr, n, M, ldm, st); break;
    case 2: triinv_reg_launch<2>(R, ldr, n, M, ldm, st); break;
    case 3: triinv_reg_launch<3>(R, ldr, n, M, ldm, st); break;
    case 4: triinv_reg_launch<4>(R, ldr, n, M, ldm, st); break;
    case 5: triinv_reg_launch<5>(R, ldr, n, M, ldm, st); break;
    case 6: triinv_reg_launch<6>(R, ldr, n, M, ldm, st); break;
    case 7: triinv_reg_launch<7>(R, ldr, n, M, ldm, st); break;
    case 8: triinv_reg_launch<8>(R, ldr, n, M, ldm, st); break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {

// Third-sweep kernels: they run only when bit 8 of *gate is set by the
// second Cholesky (see needs_third_sweep); otherwise R = R2 R1.
__global__ __launch_bounds__(256) void gram_gated_kernel(const int* __restrict__ gate,
                                                         const double* __restrict__ A, int crows,
                                                         int ldq, double* __restrict__ G) {
  if (!(*gate & 8)) return;
  gram_body(A, crows, ldq, G, blockIdx.x);
}

__global__ __launch_bounds__(64) void trsm_tile_gated_kernel(const int* __restrict__ gate,
                                                             double* __restrict__ A, int ldq, int q,
                                                             const double* __restrict__ R) {
  if (!(*gate & 8)) return;
  trsm_tile_body(A, ldq, q, R, blockIdx.x);
}

// Row i of T = R3 R2 when the third sweep ran, else of T = R2.
template <int NT>
__global__ __launch_bounds__(NT) void trmm_gated_kernel(const int* __restrict__ gate,
                                                        const double* __restrict__ R3,
                                                        const double* __restrict__ R2, int q,
                                                        double* __restrict__ T) {
  if (*gate & 8) {
    trmm_body<NT>(R3, R2, q, T, blockIdx.x);
    return;
  }
  const size_t row = static_cast<size_t>(blockIdx.x) * q;
  for (int k = threadIdx.x; k < q; k += NT) T[row + k] = R2[row + k];
}

}  // namespace

hipError_t launch_qr(double* A, int crows, int q, int ldq, int rank_cols, int sweeps, double* R,
                     double* G, double* R1, double* R2, int* status, hipStream_t st) {
  if (crows % 16 != 0 || ldq % 16 != 0 || q > ldq || q < 1 || sweeps < 1 || sweeps > 3)
    return hipErrorInvalidValue;
  const int nt = ldq / 16;
  double* R3 = G + static_cast<size_t>(ldq) * ldq;
  double* T = R3 + static_cast<size_t>(q) * q;
  double* Rs[3] = {sweeps == 1 ? R : R1, R2, R3};
  // the third sweep is gated on status bit 8 from the second Cholesky
  const bool gate3 = sweeps == 3 && ldq <= 1024;
  const size_t trsm_shm = (16 * (ldq + 1) + 16 * ldq) * sizeof(double);
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    const bool gated = gate3 && sweep == 2;
    if (gated)
      hipLaunchKernelGGL(gram_gated_kernel, dim3(nt * nt), dim3(256), 0, st, status, A, crows, ldq, G);
    else
      hipLaunchKernelGGL(gram_kernel, dim3(nt * nt), dim3(256), 0, st, A, crows, ldq, G);
    chol_launch(G, ldq, q, crows, sweep == 0 ? 1 : 2, Rs[sweep], status, sweep == 0 ? 1 : 2,
                rank_cols, gated ? status : nullptr, st);
    if (sweep == sweeps - 1) break;
    if (ldq <= 1024) {
      if (gate3 && sweep == 1)
        hipLaunchKernelGGL(trsm_tile_gated_kernel, dim3(crows / 16), dim3(64), trsm_shm, st, status,
                           A, ldq, q, Rs[sweep]);
      else
        hipLaunchKernelGGL(trsm_tile_kernel, dim3(crows / 16), dim3(64), trsm_shm, st, A, ldq, q,
                           Rs[sweep]);
    } else {
      hipLaunchKernelGGL(trsm_global_kernel, dim3((crows + 63) / 64), dim3(64), 0, st, A, crows,
                         ldq, q, Rs[sweep]);
    }
  }
  if (sweeps == 3) {
    if (gate3)
      hipLaunchKernelGGL((trmm_gated_kernel<256>), dim3(q), dim3(256), 0, st, status, R3, R2, q, T);
    else
      hipLaunchKernelGGL((trmm_kernel<256>), dim3(q), dim3(256), 0, st, R3, R2, q, T);
    hipLaunchKernelGGL((trmm_kernel<256>), dim3(q), dim3(256), 0, st, T, R1, q, R);
  } else if (sweeps == 2) {
    hipLaunchKernelGGL((trmm_kernel<256>), dim3(q), dim3(256), 0, st, R2, R1, q, R);
  }
  hipLaunchKernelGGL(rank_test_kernel, dim3(1), dim3(64), 0, st, R, q, rank_cols, status);
  return hipGetLastError();
}

hipError_t launch_triinv(const double* R, int q, int p, double* M, double* Mt, double* phi0,
                         int* status, hipStream_t st) {
  if (p < 1 || q < p) return hipErrorInvalidValue;
  if (reg_tiles(p) != 0) {
    hipError_t e = tri_inverse(R, q, p, M, p, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((triinv_finish_kernel<256>), dim3(1), dim3(256), 0, st, R, q, p, M, Mt, phi0,
                       status);
  } else {
    hipLaunchKernelGGL((triinv_kernel<256>), dim3(1), dim3(256), 0, st, R, q, p, M, Mt, phi0,
                       status);
  }
  return hipGetLastError();
}

}  // namespace tls

// ---- batched launches ---------------------------------------------------------
namespace tls {
namespace {

// gated: the third sweep of the final factorisation, run only for fits whose
// second Cholesky set status bit 8.
__global__ __launch_bounds__(256) void gram_b_kernel(const Item* __restrict__ items,
                                                     const FitDesc* __restrict__ D, int gated) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  if (gated && !(d.status[0] & 8)) return;
  gram_body(d.A, d.crows, d.ldq, d.G, it.idx);
}

// sweep 0..2 of the three-sweep factorisation, or sweep -1: the single shifted
// sweep of the stage-1 sketch (into R, rank bits to status[2]).
__device__ __forceinline__ void chol_target(const FitDesc& d, int sweep, double** R, int** status,
                                            int* shift_mode, int* fail_bit) {
  double* R3 = d.G + static_cast<size_t>(d.ldq) * d.ldq;
  *R = sweep < 0 ? d.R : (sweep == 0 ? d.R1 : (sweep == 1 ? d.R2 : R3));
  *status = sweep < 0 ? d.status + 2 : d.status;
  *shift_mode = sweep <= 0 ? 1 : 2;
  *fail_bit = sweep <= 0 ? 1 : 2;
}

template <int QT>
__global__ __launch_bounds__(256) void chol_b_kernel(const Item* __restrict__ items,
                                                     const FitDesc* __restrict__ D, int sweep) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  if (sweep == 2 && !(d.status[0] & 8)) return;
  double* R;
  int* status;
  int shift_mode, fail_bit;
  chol_target(d, sweep, &R, &status, &shift_mode, &fail_bit);
  if (QT > 0)
    chol_reg_body<(QT > 0 ? QT : 1)>(d.G, d.ldq, d.q, d.crows, shift_mode, R, status, fail_bit, d.p);
  else
    chol_body<256>(d.G, d.ldq, d.q, d.crows, shift_mode, R, status, fail_bit, d.p);
}

// 128 < q <= 224: the 32 x 32 thread grid
template <int QT>
__global__ __launch_bounds__(1024) void chol_b32_kernel(const Item* __restrict__ items,
                                                        const FitDesc* __restrict__ D, int sweep) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  if (sweep == 2 && !(d.status[0] & 8)) return;
  double* R;
  int* status;
  int shift_mode, fail_bit;
  chol_target(d, sweep, &R, &status, &shift_mode, &fail_bit);
  chol_reg_body<QT, 32>(d.G, d.ldq, d.q, d.crows, shift_mode, R, status, fail_bit, d.p);
}

__global__ __launch_bounds__(64) void trsm_b_kernel(const Item* __restrict__ items,
                                                    const FitDesc* __restrict__ D, int which) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  if (which == 1 && !(d.status[0] & 8)) return;  // only feeds the third sweep
  trsm_tile_body(d.A, d.ldq, d.q, which == 0 ? d.R1 : d.R2, it.idx);
}

__global__ __launch_bounds__(256) void trmm_b_kernel(const Item* __restrict__ items,
                                                     const FitDesc* __restrict__ D, int variant) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  double* R3 = d.G + static_cast<size_t>(d.ldq) * d.ldq;
  double* T = R3 + static_cast<size_t>(d.q) * d.q;
  if (variant == 0) {
    if (d.status[0] & 8) {
      trmm_body<256>(R3, d.R2, d.q, T, it.idx);
    } else {
      const size_t row = static_cast<size_t>(it.idx) * d.q;
      for (int k = threadIdx.x; k < d.q; k += 256) T[row + k] = d.R2[row + k];
    }
  } else
    trmm_body<256>(T, d.R1, d.q, d.R, it.idx);
}

__global__ __launch_bounds__(64) void rank_test_b_kernel(const Item* __restrict__ items,
                                                         const FitDesc* __restrict__ D, int stage) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  rank_test_body(d.R, d.q, d.p, stage == 1 ? d.status + 2 : d.status);
}

// max and min |R_ii| over the first p diagonal entries (one wavefront)
__device__ __forceinline__ void diag_range(const FitDesc& d) {
  if (threadIdx.x >= 64) return;
  double a = 0.0, b = INFINITY;
  for (int i = threadIdx.x; i < d.p; i += 64) {
    const double v = fabs(d.R[static_cast<size_t>(i) * d.q + i]);
    a = fmax(a, v);
    b = fmin(b, v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, 64));
    b = fmin(b, __shfl_xor(b, off, 64));
  }
  if (threadIdx.x == 0) {
    d.dminmax[0] = a;
    d.dminmax[1] = b;
  }
}

template <int QT>
__global__ __launch_bounds__(256) void triinv_b_kernel(const Item* __restrict__ items,
                                                       const FitDesc* __restrict__ D, int stage) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  double* M = stage == 1 ? d.M0 : d.M;
  double* Mt = stage == 1 ? d.Mt0 : d.Mt;
  if (QT > 0)
    triinv_reg_body<(QT > 0 ? QT : 1)>(d.R, d.q, d.p, M, d.p);
  else
    triinv_body<256>(d.R, d.q, d.p, M, Mt, stage == 1 ? nullptr : d.phi0,
                     stage == 1 ? d.status + 3 : d.status + 1);
  __syncthreads();
  if (QT > 0)
    triinv_finish_body<256>(d.R, d.q, d.p, M, Mt, stage == 1 ? nullptr : d.phi0,
                            stage == 1 ? d.status + 3 : d.status + 1);
  if (stage == 2) diag_range(d);
}

// 128 < p <= 224: the 32 x 32 thread grid
template <int QT>
__global__ __launch_bounds__(1024) void triinv_b32_kernel(const Item* __restrict__ items,
                                                          const FitDesc* __restrict__ D, int stage) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  double* M = stage == 1 ? d.M0 : d.M;
  double* Mt = stage == 1 ? d.Mt0 : d.Mt;
  triinv_reg32_body<QT>(d.R, d.q, d.p, M, d.p);
  __syncthreads();
  triinv_finish_body<1024>(d.R, d.q, d.p, M, Mt, stage == 1 ? nullptr : d.phi0,
                           stage == 1 ? d.status + 3 : d.status + 1);
  if (stage == 2) diag_range(d);
}

template <int QT>
hipError_t qr_b_qt(int stage, const Item* tiles, int ntiles, const Item* rowtiles, int nrowtiles,
                   const Item* rows, int nrows, const Item* fits, int nfits, int ldqmax,
                   const FitDesc* D, hipStream_t st) {
  const size_t trsm_shm = (16 * static_cast<size_t>(ldqmax + 1) + 16 * static_cast<size_t>(ldqmax)) *
                          sizeof(double);
  const int sweeps = stage == 1 ? 1 : 3;
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    hipLaunchKernelGGL(gram_b_kernel, dim3(ntiles), dim3(256), 0, st, tiles, D,
                       stage == 2 && sweep == 2 ? 1 : 0);
    if constexpr (QT > 100)
      hipLaunchKernelGGL((chol_b32_kernel<(QT > 100 ? QT - 100 : 1)>), dim3(nfits), dim3(1024), 0, st,
                         fits, D, stage == 1 ? -1 : sweep);
    else
      hipLaunchKernelGGL((chol_b_kernel<QT>), dim3(nfits), dim3(256), 0, st, fits, D,
                         stage == 1 ? -1 : sweep);
    if (sweep < sweeps - 1)
      hipLaunchKernelGGL(trsm_b_kernel, dim3(nrowtiles), dim3(64), trsm_shm, st, rowtiles, D, sweep);
  }
  if (stage == 2) {
    hipLaunchKernelGGL(trmm_b_kernel, dim3(nrows), dim3(256), 0, st, rows, D, 0);
    hipLaunchKernelGGL(trmm_b_kernel, dim3(nrows), dim3(256), 0, st, rows, D, 1);
  }
  hipLaunchKernelGGL(rank_test_b_kernel, dim3(nfits), dim3(64), 0, st, fits, D, stage);
  return hipGetLastError();
}

template <int QT>
hipError_t triinv_b_qt(int stage, const Item* fits, int nfits, int pmax, const FitDesc* D,
                       hipStream_t st) {
  if constexpr (QT > 100) {
    const size_t shm = static_cast<size_t>(pmax) * 33 * sizeof(double);
    hipLaunchKernelGGL((triinv_b32_kernel<(QT > 100 ? QT - 100 : 1)>), dim3(nfits), dim3(1024), shm, st,
                       fits, D, stage);
  } else {
    const size_t shm = QT > 0 ? static_cast<size_t>(pmax) * (pmax + 1) * sizeof(double) : 0;
    hipLaunchKernelGGL((triinv_b_kernel<QT>), dim3(nfits), dim3(256), shm, st, fits, D, stage);
  }
  return hipGetLastError();
}

}  // namespace

// qt = reg_tiles(q) of every fit of the launch.
hipError_t launch_qr_b(int stage, int qt, const Item* tiles, int ntiles, const Item* rowtiles,
                       int nrowtiles, const Item* rows, int nrows, const Item* fits, int nfits,
                       int ldqmax, const FitDesc* D, hipStream_t st) {
  if (nfits < 1) return hipSuccess;
  switch (qt) {
    case 0: return qr_b_qt<0>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 1: return qr_b_qt<1>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 2: return qr_b_qt<2>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 3: return qr_b_qt<3>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 4: return qr_b_qt<4>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 5: return qr_b_qt<5>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 6: return qr_b_qt<6>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 7: return qr_b_qt<7>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 8: return qr_b_qt<8>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 105: return qr_b_qt<105>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 106: return qr_b_qt<106>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    case 107: return qr_b_qt<107>(stage, tiles, ntiles, rowtiles, nrowtiles, rows, nrows, fits, nfits, ldqmax, D, st);
    default: return hipErrorInvalidValue;
  }
}

// pt = reg_tiles(p) of every fit of the launch.
hipError_t launch_triinv_b(int stage, int pt, const Item* fits, int nfits, int pmax,
                           const FitDesc* D, hipStream_t st) {
  if (nfits < 1) return hipSuccess;
  switch (pt) {
    case 0: return triinv_b_qt<0>(stage, fits, nfits, pmax, D, st);
    case 1: return triinv_b_qt<1>(stage, fits, nfits, pmax, D, st);
    case 2: return triinv_b_qt<2>(stage, fits, nfits, pmax, D, st);
    case 3: return triinv_b_qt<3>(stage, fits, nfits, pmax, D, st);
    case 4: return triinv_b_qt<4>(stage, fits, nfits, pmax, D, st);
    case 5: return triinv_b_qt<5>(stage, fits, nfits, pmax, D, st);
    case 6: return triinv_b_qt<6>(stage, fits, nfits, pmax, D, st);
    case 7: return triinv_b_qt<7>(stage, fits, nfits, pmax, D, st);
    case 8: return triinv_b_qt<8>(stage, fits, nfits, pmax, D, st);
    case 105: return triinv_b_qt<105>(stage, fits, nfits, pmax, D, st);
    case 106: return triinv_b_qt<106>(stage, fits, nfits, pmax, D, st);
    case 107: return triinv_b_qt<107>(stage, fits, nfits, pmax, D, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tls
