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
  // eight row steps per round so that their loads are in flight together
  // (the accumulation order is the plain one)
  int r0 = wv * 4;
  for (; r0 + 7 * 16 < crows; r0 += 8 * 16) {
    double a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double* row = A + static_cast<size_t>(r0 + 16 * k + kr) * ldq;
      a[k] = row[ci];
      b[k] = row[cj];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k], b[k], acc, 0, 0, 0);
  }
  for (; r0 < crows; r0 += 16) {
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
    // eight terms' loads in flight, summed in the plain order
    double acc = 0.0;
    int k = i;
    for (; k + 7 <= j; k += 8) {
      double rb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) rb[u] = Rb[static_cast<size_t>(k + u) * q + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += ra[k + u] * rb[u];
    }
    for (; k <= j; ++k) acc += ra[k] * Rb[static_cast<size_t>(k) * q + j];
    C[static_cast<size_t>(i) * q + j] = acc;
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void trmm_kernel(const double* __restrict__ Ra,
                                                  const double* __restrict__ Rb, int q,
                                                  double* __restrict__ C) {
  trmm_body<NT>(Ra, Rb, q, C, blockIdx.x);
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
  __shared__ double pub[2][TD * QT + 1];
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
    // an unshifted attempt that will be redone with the shift stops at its
    // first failed pivot (d is the same LDS word in every thread, so the
    // whole workgroup leaves the column loop together)
    const bool stop_on_fail = shift_mode == 2 && attempt == 0;
    bool stopped = false;
    // column j = TD a0 + jj: tiles left of / above tile a0 are final (row j's
    // multipliers vanish there), so the register tile indices are static
#pragma unroll
    for (int a0 = 0; a0 < QT; ++a0) {
      for (int jj = 0; jj < TD; ++jj) {
        const int j = TD * a0 + jj;
        if (j >= q) break;
        double* pj = pub[j & 1];
        // row j beyond the diagonal (entries up to j published as zero, so
        // the multipliers need no masks), the pivot in its own word
        if (ty == jj) {
#pragma unroll
          for (int b = a0; b < QT; ++b) {
            const int k = tx + TD * b;
            pj[k] = k > j ? reg[a0][b] : 0.0;
            if (k == j) pj[TD * QT] = reg[a0][b];
          }
        }
        __syncthreads();
        double d = pj[TD * QT];
        if (!(d > floor_)) {
          if (j < rank_cols && threadIdx.x == 0) s_fail = 1;
          if (j < rank_cols && stop_on_fail) {
            stopped = true;
            break;
          }
          d = floor_;
        }
        if (j < rank_cols) {
          dmin = fmin(dmin, d);
          dmax = fmax(dmax, d);
        }
        // 1/sqrt(d) from the hardware estimate and three Newton steps
        // (relative error of the estimate below 2^-20: 2^-60 after two,
        // the third settles the last bit), sqrt(d) and 1/d from it
        double isd = __builtin_amdgcn_rsq(d);
        isd = fma(0.5 * isd, fma(-d * isd, isd, 1.0), isd);
        isd = fma(0.5 * isd, fma(-d * isd, isd, 1.0), isd);
        isd = fma(0.5 * isd, fma(-d * isd, isd, 1.0), isd);
        const double sd = d * isd;
        const double invd = isd * isd;
        // row j of R stays in the registers of its owner (not updated again);
        // R is written once after the last column
        if (ty == jj) {
#pragma unroll
          for (int b = a0; b < QT; ++b) {
            const int k = tx + TD * b;
            reg[a0][b] = k < j ? 0.0 : (k == j ? sd : reg[a0][b] * isd);
          }
        }
        // rank-one update of the trailing rows and columns (index > j) on
        // the tiles on and above the diagonal (the factor reads only the
        // upper triangle: row j's entries right of the pivot are also its
        // column's entries below it); pub entries beyond q are zero
        double fi[QT], fk[QT];
#pragma unroll
        for (int a = a0; a < QT; ++a) fi[a] = pj[ty + TD * a] * invd;
#pragma unroll
        for (int b = a0; b < QT; ++b) fk[b] = pj[tx + TD * b];
#pragma unroll
        for (int a = a0; a < QT; ++a)
#pragma unroll
          for (int b = a; b < QT; ++b) reg[a][b] = fma(-fi[a], fk[b], reg[a][b]);
      }
      if (stopped) break;
    }
    __syncthreads();
    const int failed = s_fail;
    if (stopped) continue;  // redone with the shift; R is written by that attempt
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
                                                         double* __restrict__ M, int ldm,
                                                         double* __restrict__ Mt) {
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
      if (r < ldm && c < ldm) {
        const double x = (r < n && c < n) ? reg[a][b] : 0.0;
        M[static_cast<size_t>(r) * ldm + c] = x;
        if (Mt) Mt[static_cast<size_t>(c) * ldm + r] = x;
      }
    }
  // rows / columns of the ldm block beyond 16 QT (only when ldm > 16 QT)
  if (ldm > 16 * QT)
    for (int e = threadIdx.x; e < ldm * ldm; e += 256) {
      const int r = e / ldm, c = e % ldm;
      if (r >= 16 * QT || c >= 16 * QT) {
        M[e] = 0.0;
        if (Mt) Mt[e] = 0.0;
      }
    }
}

template <int QT>
__global__ __launch_bounds__(256) void triinv_reg_kernel(const double* __restrict__ R, int ldr, int n,
                                                         double* __restrict__ M, int ldm,
                                                         double* __restrict__ Mt) {
  triinv_reg_body<QT>(R, ldr, n, M, ldm, Mt);
}

// A <- A R^{-1} on the first q columns, 16 rows per wavefront (rows are
// independent).  Blocked by 16 columns as in LAPACK's triangular solve: the
// 16 x 16 diagonal block by forward substitution (one lane per row), then the
// trailing columns A[:, K] -= X[:, J] R[J, K] on the FP64 matrix cores.
// RALL (ldq <= 128): all of R is staged in LDS once, ahead of the column
// blocks, instead of 16 rows per block.  With ldq <= TRSM_DINV_LDQ the 16 x 16
// diagonal blocks are inverted first (one column per lane, back substitution,
// all blocks at once) and each block step is X_J = T_J R_JJ^{-1} on the
// matrix cores, as GPU triangular solves commonly do: the per-row
// substitution chain (16 dependent divides per block) is the solve's
// critical path otherwise.  Its error is bounded by u kappa(R_JJ) per block
// instead of u; the Cholesky QR sweeps that follow re-orthogonalise.
// diagonal-block inverses fit in LDS beside all of R up to this ldq
constexpr int TRSM_DINV_LDQ = 112;

template <bool RALL>
__device__ __forceinline__ void trsm_tile_body(double* __restrict__ A, int ldq, int q,
                                                       const double* __restrict__ R, int rt) {
  // 16 x (ldq + 1) rows of A, then 16 (RALL: ldq) x ldq rows of R
  extern __shared__ double T[];
  const int ld = ldq + 1;
  double* const Rbase = T + 16 * ld;
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
  // rows j0 .. j0+15 of R from column j0 on into dst (zero outside q x q;
  // R is upper triangular, so nothing left of j0 is read)
  auto stage_rows = [&](int j0, double* dst) {
    for (int cc = j0 + lane; cc < ldq; cc += 64) {
      double v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r)
        v[r] = (j0 + r < q && cc < q) ? R[static_cast<size_t>(j0 + r) * q + cc] : 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) dst[r * ldq + cc] = v[r];
    }
  };
  const bool dinv = RALL && ldq <= TRSM_DINV_LDQ;
  double* const Dinv = Rbase + static_cast<size_t>(ldq) * ldq;  // nt x 16 x 16 (dinv)
  if constexpr (RALL) {
    for (int J = 0; J < nt; ++J) stage_rows(J * 16, Rbase + static_cast<size_t>(J) * 16 * ldq);
    if (dinv) {
      __syncthreads();
      // column c of R_JJ^{-1}: U x = e_c from the last row up (rows past q:
      // the identity)
      for (int col = lane; col < nt * 16; col += 64) {
        const int J = col >> 4, c = col & 15, j0 = J * 16;
        const double* U = Rbase + static_cast<size_t>(j0) * ldq + j0;
        double x[16];
#pragma unroll
        for (int i = 15; i >= 0; --i) {
          double acc = i == c ? 1.0 : 0.0;
#pragma unroll
          for (int k = i + 1; k < 16; ++k) acc -= U[i * ldq + k] * x[k];
          x[i] = j0 + i < q ? acc / U[i * ldq + i] : (i == c ? 1.0 : 0.0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Dinv[J * 256 + i * 16 + c] = x[i];
      }
    }
  }
  for (int J = 0; J < nt; ++J) {
    const int j0 = J * 16;
    double* const Rp = RALL ? Rbase + static_cast<size_t>(j0) * ldq : Rbase;
    if constexpr (!RALL) stage_rows(j0, Rp);
    __syncthreads();
    if (dinv) {
      // X_J = T_J R_JJ^{-1}: all reads of T_J precede the writes
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      double xa[4];
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) xa[k4] = T[(lane & 15) * ld + j0 + 4 * k4 + (lane >> 4)];
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        const double db = Dinv[J * 256 + (4 * k4 + (lane >> 4)) * 16 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k4], db, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) T[(4 * v + (lane >> 4)) * ld + j0 + (lane & 15)] = acc[v];
    } else if (lane < 16) {
      // the row's 16 entries of this block in registers (R rows read as
      // LDS broadcasts): the same operations in the same order as a
      // substitution in place, without an LDS round trip per step
      double* row = T + lane * ld;
      const int nj = min(16, q - j0);
      double xr[16];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) xr[kk] = row[j0 + kk];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        if (jj < nj) {
          const double* rj = Rp + jj * ldq;
          const double x = xr[jj] / rj[j0 + jj];
          xr[jj] = x;
#pragma unroll
          for (int kk = jj + 1; kk < 16; ++kk)
            if (kk < nj) xr[kk] -= x * rj[j0 + kk];
        }
      }
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) row[j0 + kk] = xr[kk];
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

template <bool RALL>
__global__ __launch_bounds__(64) void trsm_tile_kernel(double* __restrict__ A, int ldq, int q,
                                                       const double* __restrict__ R) {
  trsm_tile_body<RALL>(A, ldq, q, R, blockIdx.x);
}

// LDS of the tiled solve: 16 rows of A (ldq + 1 padded), then 16 rows of R
// or (ldq <= 128) all of R, and the inverted diagonal blocks for
// ldq <= TRSM_DINV_LDQ; within 160 KiB up to ldq = TRSM_TILE_LDQ_MAX.
constexpr bool trsm_rall(int ldq) { return ldq <= 128; }
constexpr size_t trsm_lds_bytes(int ldq) {
  return (16 * static_cast<size_t>(ldq + 1) +
          (trsm_rall(ldq) ? static_cast<size_t>(ldq) : size_t{16}) * ldq +
          (ldq <= TRSM_DINV_LDQ ? 16 * static_cast<size_t>(ldq) : 0)) *
         sizeof(double);
}
static_assert(trsm_lds_bytes(TRSM_TILE_LDQ_MAX) <= 160 * 1024 &&
                  trsm_lds_bytes(TRSM_TILE_LDQ_MAX + 16) > 160 * 1024,
              "TRSM_TILE_LDQ_MAX is the largest ldq whose tile TRSM fits in LDS");

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
                                                  double* __restrict__ M, int ldm,
                                                  double* __restrict__ Mt) {
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
      if (r < ldm && c < ldm) {
        const double x = (r < n && c < n) ? reg[a][b] : 0.0;
        M[static_cast<size_t>(r) * ldm + c] = x;
        if (Mt) Mt[static_cast<size_t>(c) * ldm + r] = x;
      }
    }
}

template <int QT>
__global__ __launch_bounds__(1024) void triinv_reg32_kernel(const double* __restrict__ R, int ldr,
                                                            int n, double* __restrict__ M, int ldm,
                                                            double* __restrict__ Mt) {
  triinv_reg32_body<QT>(R, ldr, n, M, ldm, Mt);
}

// After a register inverse (which also wrote M^T): phi0 = M R[:p, p] (the
// compressed problem's solution), the rank test min|R_ii| <= p u max|R_ii|,
// and (when dminmax is given) that max and min.
template <int NT>
__device__ __forceinline__ void triinv_finish_body(const double* __restrict__ R, int q,
                                                           int p, const double* __restrict__ M,
                                                           double* __restrict__ phi0,
                                                           int* __restrict__ status,
                                                           double* __restrict__ dminmax = nullptr) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (phi0 && q > p) {
    // phi0_i = M[i, i:] R[i:, p]: one wavefront per row, lanes over the row
    for (int i = wid; i < p; i += NT / 64) {
      double acc = 0.0;
      for (int j = i + lane; j < p; j += 64)
        acc += M[static_cast<size_t>(i) * p + j] * R[static_cast<size_t>(j) * q + p];
      acc = wave_sum(acc);
      if (lane == 0) phi0[i] = acc;
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
    if (threadIdx.x == 0 && dminmax) {
      dminmax[0] = a;
      dminmax[1] = b;
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void triinv_finish_kernel(const double* __restrict__ R, int q,
                                                           int p, const double* __restrict__ M,
                                                           double* __restrict__ phi0,
                                                           int* __restrict__ status,
                                                           double* __restrict__ dminmax) {
  triinv_finish_body<NT>(R, q, p, M, phi0, status, dminmax);
}


// ---- blocked Cholesky and triangular inverse (order above 224) -------------
// Right-looking Cholesky on 32 x 32 blocks, one launch per block column k:
// every trailing block (i, j), k < i <= j, is updated by W_ij -= P_i^T P_j
// with P_i = D_k^T W_ki = R_ki (D_k = R_kk^{-1}, inverted once when R_kk is
// factored), and the workgroup of block (k+1, k+1) then factors that block
// and inverts its factor for launch k+1.  Every workgroup recomputes the two
// panel blocks it needs, so the panel solve needs no launch of its own.  The
// working matrix W (G plus the shift, padded with the identity to whole
// blocks), the block inverses and a control record (shift, pivot floor,
// pivot range, breakdown flag, liveness, retry flag) live in the QR scratch
// beyond R3 and T.  An unshifted factorisation (shift mode 2) that breaks
// down sets the retry flag, which enables a second, shifted chain.
constexpr int NBK = 32;

struct BlkScratch {
  double* W;
  double* Dinv;
  double* ctl;  // shift, floor, dmin, dmax, live, failed, retry
  int ldw, nbk;
};

__host__ __device__ inline BlkScratch blk_scratch(double* G, int ldq, int q) {
  BlkScratch s;
  s.nbk = (q + NBK - 1) / NBK;
  s.ldw = s.nbk * NBK;
  s.W = G + static_cast<size_t>(ldq) * ldq + 2 * static_cast<size_t>(q) * q;
  s.Dinv = s.W + static_cast<size_t>(s.ldw) * s.ldw;
  s.ctl = s.Dinv + static_cast<size_t>(s.nbk) * NBK * NBK;
  return s;
}

__host__ __device__ inline size_t blk_scratch_doubles(int q) {
  const size_t nbk = (q + NBK - 1) / NBK;
  return nbk * NBK * nbk * NBK + nbk * NBK * NBK + 8;
}

// t-th pair (a, b), 0 <= a <= b < m, in row order
__device__ __forceinline__ void upper_pair(int t, int m, int* a, int* b) {
  int r = 0;
  while (t >= m - r) {
    t -= m - r;
    ++r;
  }
  *a = r;
  *b = r + t;
}

// Lane src's value of x in every lane (src a compile-time constant: two
// scalar reads, no LDS).
__device__ __forceinline__ double lane_bcast(double x, int src) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Orders one wavefront's LDS writes before its later LDS reads of other
// lanes' data (a wavefront executes its LDS instructions in program order;
// this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_sched_barrier(0);
}

// One wavefront (wavefront 0 of the workgroup) factors the 32 x 32 block B
// (LDS, upper part), columns b*32 .. b*32+31 of the whole matrix, by
// symmetric elimination of the augmented matrix [B | I], lane l holding
// column l of it in registers: column jj's pivot (clamped to the floor; a
// breakdown when the column is below rank_cols) gives row jj of the factor
// U by scaling with its inverse square root, and every later row ii loses
// U[jj][ii] times that row.  Lane l < 32 ends with column l of U, lane
// 32 + r with row r of U^{-1} (the eliminated identity is U^{-T}).  R gets
// the block (zero below the diagonal, clipped to q), Dinv[b] its inverse.
__device__ __forceinline__ void wave_factor(const double (*B)[NBK + 1], double* pub, int b, int q,
                                            double floor_, int rank_cols, double* dmin,
                                            double* dmax, bool* failed, double* __restrict__ R,
                                            double* __restrict__ Dinv) {
  const int lane = threadIdx.x & 63;
  double v[NBK];
  double mn = *dmin, mx = *dmax;
  bool fl = *failed;
#pragma unroll
  for (int r = 0; r < NBK; ++r) {
    const double g = B[r][lane & (NBK - 1)];
    v[r] = lane < NBK ? g : (r == lane - NBK ? 1.0 : 0.0);
  }
  // branch-free steps (divergent branches here make the compiler keep far
  // more values live); row jj's diagonal entry goes to dg
#pragma unroll
  for (int jj = 0; jj < NBK; ++jj) {
    const bool track = b * NBK + jj < rank_cols;
    double d = lane_bcast(v[jj], jj);
    const bool ok = d > floor_;
    fl = fl || (track && !ok);
    d = ok ? d : floor_;
    mn = track ? fmin(mn, d) : mn;
    mx = track ? fmax(mx, d) : mx;
    const double rjj = sqrt(d);
    const double inv = 1.0 / rjj;
    v[jj] *= inv;
    double* pb = pub + (jj & 1) * 64;
    pb[lane] = v[jj];
    pub[128 + jj] = rjj;
    wave_lds_sync();
#pragma unroll
    for (int ii = jj + 1; ii < NBK; ++ii) v[ii] -= pb[ii] * v[jj];
  }
  *dmin = mn;
  *dmax = mx;
  *failed = fl;
  if (lane < NBK) {
    const int k = b * NBK + lane;
#pragma unroll
    for (int r = 0; r < NBK; ++r) {
      const int i = b * NBK + r;
      if (i < q && k < q)
        R[static_cast<size_t>(i) * q + k] = r < lane ? v[r] : (r == lane ? pub[128 + r] : 0.0);
    }
  } else {
    double* drow = Dinv + static_cast<size_t>(b) * NBK * NBK + (lane - NBK) * NBK;
#pragma unroll
    for (int c = 0; c < NBK; ++c) drow[c] = v[c];
  }
}

// One wavefront: X = T^{-1} for the upper-triangular 32 x 32 block T (LDS),
// lane c < 32 forming column c by right-looking back substitution (T's
// entries are uniform LDS reads).  X goes to LDS.
__device__ __forceinline__ void wave_tri_inv(const double (*T)[NBK + 1], double (*X)[NBK + 1]) {
  const int c = threadIdx.x & (NBK - 1);
  double acc[NBK];
#pragma unroll
  for (int r = 0; r < NBK; ++r) acc[r] = r == c ? 1.0 : 0.0;
#pragma unroll
  for (int i = NBK - 1; i >= 0; --i) {
    const double xi = acc[i] / T[i][i];
    acc[i] = xi;
#pragma unroll
    for (int r = 0; r < i; ++r) acc[r] -= T[r][i] * xi;
  }
  if ((threadIdx.x & 63) < NBK) {
#pragma unroll
    for (int r = 0; r < NBK; ++r) X[r][c] = acc[r];
  }
}

// Launch before the panels of one attempt (0: unshifted, shift mode 2 only;
// 1: shifted): workgroup t copies upper block pair t of G into W and zeroes
// the mirrored block of R; workgroup 0 also factors block 0 and sets up the
// control record.  gate: NULL, or run only when bit 8 of *gate is set.
__device__ __forceinline__ void chol_blk_init_body(const double* __restrict__ G, int ldq, int q,
                                                   int crows, int shift_mode, int attempt,
                                                   const int* __restrict__ gate,
                                                   double* __restrict__ R, int rank_cols,
                                                   const BlkScratch& s, int t) {
  __shared__ double red[4];
  __shared__ double B[NBK][NBK + 1], pub[128 + NBK];
  double* ctl = s.ctl;
  if (t >= s.nbk * (s.nbk + 1) / 2) return;
  const bool gate_on = !gate || (*gate & 8);
  // attempt 1 after an unshifted attempt runs only on its breakdown
  const bool live = (attempt == 1 && shift_mode == 2) ? ctl[6] != 0.0 : gate_on;
  if (!live) {
    if (t == 0 && threadIdx.x == 0) {
      ctl[4] = 0.0;
      if (attempt == 0) ctl[6] = 0.0;
    }
    return;
  }
  double tr = 0.0;
  for (int i = threadIdx.x; i < q; i += 256) tr += G[static_cast<size_t>(i) * ldq + i];
  tr = block_sum<256>(tr, red);
  const double shift =
      attempt ? 11.0 * (static_cast<double>(crows) * q + static_cast<double>(q) * (q + 1)) * 0x1p-53 * tr
              : 0.0;
  const double floor_ = tr > 0.0 ? tr * 0x1p-104 : 1e-300;
  int bi, bj;
  upper_pair(t, s.nbk, &bi, &bj);
  for (int e = threadIdx.x; e < NBK * NBK; e += 256) {
    const int r = e / NBK, c = e % NBK;
    const int i = bi * NBK + r, k = bj * NBK + c;
    const double v = (i < q && k < q) ? G[static_cast<size_t>(i) * ldq + k] + (i == k ? shift : 0.0)
                                      : (i == k ? 1.0 : 0.0);
    s.W[static_cast<size_t>(i) * s.ldw + k] = v;
    if (t == 0) B[r][c] = v;
    // block (bj, bi) of R lies below the diagonal
    const int i2 = bj * NBK + r, k2 = bi * NBK + c;
    if (bi < bj && i2 < q && k2 < q) R[static_cast<size_t>(i2) * q + k2] = 0.0;
  }
  if (t != 0) return;
  __syncthreads();
  if (threadIdx.x >= 64) return;
  double dmin = INFINITY, dmax = 0.0;
  bool failed = false;
  wave_factor(B, pub, 0, q, floor_, rank_cols, &dmin, &dmax, &failed, R, s.Dinv);
  if (threadIdx.x == 0) {
    ctl[0] = shift;
    ctl[1] = floor_;
    ctl[2] = dmin;
    ctl[3] = dmax;
    ctl[4] = 1.0;
    ctl[5] = failed ? 1.0 : 0.0;
    if (attempt == 0) ctl[6] = 0.0;
  }
}

// Launch k: workgroup t updates trailing block pair t (see above).
__device__ __forceinline__ void chol_blk_panel_body(int q, double* __restrict__ R, int rank_cols,
                                                    const BlkScratch& s, int k, int t) {
  __shared__ double Pi[NBK][NBK + 1], Pj[NBK][NBK + 1];
  __shared__ double B[NBK][NBK + 1], pub[128 + NBK];
  const double* ctl = s.ctl;
  const int m = s.nbk - 1 - k;
  if (m <= 0 || t >= m * (m + 1) / 2) return;
  if (ctl[4] == 0.0) return;
  int a, b;
  upper_pair(t, m, &a, &b);
  const int bi = k + 1 + a, bj = k + 1 + b;
  const bool diag_next = a == 0 && b == 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tr = wv >> 1, tc = wv & 1;
  const int l16 = lane & 15, l4 = lane >> 4;
  const double* Dk = s.Dinv + static_cast<size_t>(k) * NBK * NBK;
  const double* Wk = s.W + static_cast<size_t>(k) * NBK * s.ldw;
  // P_i, P_j tiles (tr, tc): P[r][c] = sum_s D_k[s][r] W_k[s][c]
  d4 pi = {0.0, 0.0, 0.0, 0.0}, pj = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s0 = 0; s0 < NBK; s0 += 4) {
    const int sr = s0 + l4;
    const double av = Dk[sr * NBK + tr * 16 + l16];
    const double* wrow = Wk + static_cast<size_t>(sr) * s.ldw;
    pi = __builtin_amdgcn_mfma_f64_16x16x4f64(av, wrow[bi * NBK + tc * 16 + l16], pi, 0, 0, 0);
    pj = __builtin_amdgcn_mfma_f64_16x16x4f64(av, wrow[bj * NBK + tc * 16 + l16], pj, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Pi[tr * 16 + 4 * v + l4][tc * 16 + l16] = pi[v];
    Pj[tr * 16 + 4 * v + l4][tc * 16 + l16] = pj[v];
  }
  __syncthreads();
  // W_ij -= P_i^T P_j
  d4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s0 = 0; s0 < NBK; s0 += 4) {
    const int sr = s0 + l4;
    u = __builtin_amdgcn_mfma_f64_16x16x4f64(Pi[sr][tr * 16 + l16], Pj[sr][tc * 16 + l16], u, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = tr * 16 + 4 * v + l4, c = tc * 16 + l16;
    double* w = s.W + static_cast<size_t>(bi * NBK + r) * s.ldw + bj * NBK + c;
    const double nv = *w - u[v];
    *w = nv;
    if (diag_next) B[r][c] = nv;
  }
  if (bi == bj) {
    // R_{k, bi} = P_i
    for (int e = threadIdx.x; e < NBK * NBK; e += 256) {
      const int r = e / NBK, c = e % NBK;
      const int i = k * NBK + r, kk = bi * NBK + c;
      if (i < q && kk < q) R[static_cast<size_t>(i) * q + kk] = Pi[r][c];
    }
  }
  if (!diag_next) return;
  __syncthreads();
  if (wv != 0) return;
  double dmin = ctl[2], dmax = ctl[3];
  bool failed = ctl[5] != 0.0;
  wave_factor(B, pub, bi, q, ctl[1], rank_cols, &dmin, &dmax, &failed, R, s.Dinv);
  if (lane == 0) {
    s.ctl[2] = dmin;
    s.ctl[3] = dmax;
    s.ctl[5] = failed ? 1.0 : 0.0;
  }
}

// After the panels of one attempt (one thread): status bits as the
// single-workgroup Cholesky sets them, or the retry flag.
__device__ __forceinline__ void chol_blk_finish_body(int shift_mode, int attempt,
                                                     int* __restrict__ status, int fail_bit,
                                                     const BlkScratch& s) {
  double* ctl = s.ctl;
  if (threadIdx.x != 0 || ctl[4] == 0.0) return;
  const bool failed = ctl[5] != 0.0;
  if (attempt == 0) {
    if (failed) {
      ctl[6] = 1.0;
      return;
    }
    if (needs_third_sweep(ctl[2], ctl[3])) atomicOr(status, 8);
    return;
  }
  if (failed) atomicOr(status, fail_bit);
  if (shift_mode == 2) atomicOr(status, 8);
}

__global__ __launch_bounds__(256) void chol_blk_init_kernel(double* G, int ldq, int q, int crows,
                                                            int shift_mode, int attempt,
                                                            const int* __restrict__ gate,
                                                            double* __restrict__ R, int rank_cols) {
  chol_blk_init_body(G, ldq, q, crows, shift_mode, attempt, gate, R, rank_cols,
                     blk_scratch(G, ldq, q), blockIdx.x);
}

__global__ __launch_bounds__(256) void chol_blk_panel_kernel(double* G, int ldq, int q,
                                                             double* __restrict__ R, int rank_cols,
                                                             int k) {
  chol_blk_panel_body(q, R, rank_cols, blk_scratch(G, ldq, q), k, blockIdx.x);
}

__global__ __launch_bounds__(64) void chol_blk_finish_kernel(double* G, int ldq, int q,
                                                             int shift_mode, int attempt,
                                                             int* __restrict__ status,
                                                             int fail_bit) {
  chol_blk_finish_body(shift_mode, attempt, status, fail_bit, blk_scratch(G, ldq, q));
}

// M = R[:p,:p]^{-1} by 32 x 32 blocks: the diagonal blocks are inverted first
// (one workgroup each, also kept in Dinv); launch d then forms every block at
// distance d above the diagonal, M_ij = -D_i sum_{i<k<=j} R_ik M_kj, from
// blocks of earlier launches.  Blocks beyond p are the identity.

// Diagonal block b of M, and the strictly lower blocks of its block row (zero).
__device__ __forceinline__ void inv_blk_diag_body(const double* __restrict__ R, int q, int p,
                                                  double* __restrict__ M,
                                                  double* __restrict__ Dinv, int b) {
  __shared__ double B[NBK][NBK + 1], X[NBK][NBK + 1];
  for (int e = threadIdx.x; e < NBK * NBK; e += 256) {
    const int r = e / NBK, c = e % NBK;
    const int i = b * NBK + r, k = b * NBK + c;
    B[r][c] = (i < p && k < p) ? R[static_cast<size_t>(i) * q + k] : (i == k ? 1.0 : 0.0);
  }
  __syncthreads();
  if (threadIdx.x < 64) wave_tri_inv(B, X);
  __syncthreads();
  for (int e = threadIdx.x; e < NBK * NBK; e += 256) {
    const int r = e / NBK, c = e % NBK;
    const int i = b * NBK + r, k = b * NBK + c;
    if (i < p && k < p) M[static_cast<size_t>(i) * p + k] = X[r][c];
    Dinv[static_cast<size_t>(b) * NBK * NBK + e] = X[r][c];
  }
  const int w = b * NBK;
  for (int e = threadIdx.x; e < NBK * w; e += 256) {
    const int i = b * NBK + e / w, k = e % w;
    if (i < p) M[static_cast<size_t>(i) * p + k] = 0.0;
  }
}

// Block (i, i + d) of M: wavefront w sums the terms kb = i + 1 + w, i + 5 + w,
// ... for all four 16 x 16 tiles, the partial sums meet in LDS in a fixed
// order, and the four wavefronts then apply -D_i, one tile each.
__device__ __forceinline__ void inv_blk_off_body(const double* __restrict__ R, int q, int p,
                                                 double* __restrict__ M,
                                                 const double* __restrict__ Dinv, int d, int i) {
  __shared__ double S[4][NBK][NBK + 1];
  const int j = i + d;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kb = i + 1 + wv; kb <= j; kb += 4) {
#pragma unroll
    for (int s0 = 0; s0 < NBK; s0 += 4) {
      const int col = kb * NBK + s0 + l4;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int row = i * NBK + a * 16 + l16;
        av[a] = (row < p && col < p) ? R[static_cast<size_t>(row) * q + col] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int mcol = j * NBK + b * 16 + l16;
        bv[b] = (col < p && mcol < p) ? M[static_cast<size_t>(col) * p + mcol] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) S[wv][a * 16 + 4 * v + l4][b * 16 + l16] = acc[a][b][v];
  __syncthreads();
  const int tr = wv >> 1, tc = wv & 1;
  const double* Di = Dinv + static_cast<size_t>(i) * NBK * NBK;
  d4 out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s0 = 0; s0 < NBK; s0 += 4) {
    const int sr = s0 + l4, sc = tc * 16 + l16;
    const double sv = ((S[0][sr][sc] + S[1][sr][sc]) + S[2][sr][sc]) + S[3][sr][sc];
    out = __builtin_amdgcn_mfma_f64_16x16x4f64(Di[(tr * 16 + l16) * NBK + sr], sv, out, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = i * NBK + tr * 16 + 4 * v + l4;
    const int mcol = j * NBK + tc * 16 + l16;
    if (r < p && mcol < p) M[static_cast<size_t>(r) * p + mcol] = -out[v];
  }
}

// Mt = M^T by 32 x 32 tiles (t < nbp^2), phi0 = M R[:p, p] by 32-row blocks
// (nbp workgroups after the tiles), and on the first of those the rank test
// min|R_ii| <= p u max|R_ii| (status bit 4) and the diagonal range.
__device__ __forceinline__ void inv_blk_finish_body(const double* __restrict__ R, int q, int p,
                                                    const double* __restrict__ M,
                                                    double* __restrict__ Mt,
                                                    double* __restrict__ phi0,
                                                    int* __restrict__ status,
                                                    double* __restrict__ dminmax, int t) {
  __shared__ double T[NBK][NBK + 1];
  const int nbp = (p + NBK - 1) / NBK;
  if (t < nbp * nbp) {
    const int bi = t / nbp, bj = t % nbp;
    for (int e = threadIdx.x; e < NBK * NBK; e += 256) {
      const int r = e / NBK, c = e % NBK;
      const int i = bi * NBK + r, k = bj * NBK + c;
      T[r][c] = (i < p && k < p) ? M[static_cast<size_t>(i) * p + k] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NBK * NBK; e += 256) {
      const int r = e / NBK, c = e % NBK;
      const int i = bj * NBK + r, k = bi * NBK + c;
      if (i < p && k < p) Mt[static_cast<size_t>(i) * p + k] = T[c][r];
    }
    return;
  }
  const int rb = t - nbp * nbp;
  if (rb >= nbp) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (phi0 && q > p) {
    for (int rr = 0; rr < NBK / 4; ++rr) {
      const int i = rb * NBK + wv * (NBK / 4) + rr;
      if (i >= p) break;
      double acc = 0.0;
      for (int j = i + lane; j < p; j += 64)
        acc += M[static_cast<size_t>(i) * p + j] * R[static_cast<size_t>(j) * q + p];
      acc = wave_sum(acc);
      if (lane == 0) phi0[i] = acc;
    }
  }
  if (rb == 0 && wv == 0) {
    double a = 0.0, b = INFINITY;
    for (int i = lane; i < p; i += 64) {
      const double d = fabs(R[static_cast<size_t>(i) * q + i]);
      a = fmax(a, d);
      b = fmin(b, d);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a = fmax(a, __shfl_xor(a, off, 64));
      b = fmin(b, __shfl_xor(b, off, 64));
    }
    if (lane == 0) {
      if (status && !(b > static_cast<double>(p) * 0x1p-53 * a)) atomicOr(status, 4);
      if (dminmax) {
        dminmax[0] = a;
        dminmax[1] = b;
      }
    }
  }
}

__global__ __launch_bounds__(256) void inv_blk_diag_kernel(const double* __restrict__ R, int q,
                                                           int p, double* __restrict__ M,
                                                           double* __restrict__ Dinv) {
  inv_blk_diag_body(R, q, p, M, Dinv, blockIdx.x);
}

__global__ __launch_bounds__(256) void inv_blk_off_kernel(const double* __restrict__ R, int q,
                                                          int p, double* __restrict__ M,
                                                          const double* __restrict__ Dinv, int d) {
  inv_blk_off_body(R, q, p, M, Dinv, d, blockIdx.x);
}

__global__ __launch_bounds__(256) void inv_blk_finish_kernel(const double* __restrict__ R, int q,
                                                             int p, const double* __restrict__ M,
                                                             double* __restrict__ Mt,
                                                             double* __restrict__ phi0,
                                                             int* __restrict__ status,
                                                             double* __restrict__ dminmax) {
  inv_blk_finish_body(R, q, p, M, Mt, phi0, status, dminmax, blockIdx.x);
}

void chol_blk_launch(double* G, int ldq, int q, int crows, int shift_mode, double* R, int* status,
                     int fail_bit, int rank_cols, const int* gate, hipStream_t st) {
  const int nbk = (q + NBK - 1) / NBK;
  for (int attempt = shift_mode == 1 ? 1 : 0; attempt < 2; ++attempt) {
    hipLaunchKernelGGL(chol_blk_init_kernel, dim3(nbk * (nbk + 1) / 2), dim3(256), 0, st, G, ldq, q,
                       crows, shift_mode, attempt, gate, R, rank_cols);
    for (int k = 0; k + 1 < nbk; ++k) {
      const int m = nbk - 1 - k;
      hipLaunchKernelGGL(chol_blk_panel_kernel, dim3(m * (m + 1) / 2), dim3(256), 0, st, G, ldq, q,
                         R, rank_cols, k);
    }
    hipLaunchKernelGGL(chol_blk_finish_kernel, dim3(1), dim3(64), 0, st, G, ldq, q, shift_mode,
                       attempt, status, fail_bit);
  }
}

// Mt doubles as the store of the diagonal block inverses until the finish.
void inv_blk_launch(const double* R, int q, int p, double* M, double* Mt, double* phi0,
                    int* status, double* dminmax, hipStream_t st) {
  const int nbp = (p + NBK - 1) / NBK;
  hipLaunchKernelGGL(inv_blk_diag_kernel, dim3(nbp), dim3(256), 0, st, R, q, p, M, Mt);
  for (int d = 1; d < nbp; ++d)
    hipLaunchKernelGGL(inv_blk_off_kernel, dim3(nbp - d), dim3(256), 0, st, R, q, p, M, Mt, d);
  hipLaunchKernelGGL(inv_blk_finish_kernel, dim3(nbp * nbp + nbp), dim3(256), 0, st, R, q, p, M, Mt,
                     phi0, status, dminmax);
}

}  // namespace

// Scratch: G holds ldq*ldq + 2*q*q doubles (Gram matrix, then R3 and R3 R2)
// and, for the blocked Cholesky (q above 224), its working matrix, block
// inverses and control record beyond that.
size_t qr_scratch_doubles(int crows, int q, int ldq) {
  (void)crows;
  return static_cast<size_t>(ldq) * ldq + 2 * static_cast<size_t>(q) * q +
         (reg_tiles(q) == 0 ? blk_scratch_doubles(q) : 0);
}

namespace {

template <int QT>
void chol_reg_launch(const double* G, int ldq, int q, int crows, int shift_mode, double* R,
                     int* status, int fail_bit, int rank_cols, const int* gate, hipStream_t st) {
  hipLaunchKernelGGL((chol_reg_kernel<QT>), dim3(1), dim3(256), 0, st, G, ldq, q, crows, shift_mode,
                     R, status, fail_bit, rank_cols, gate);
}

// gate: NULL, or run only when bit 8 of *gate is set (the third sweep).
void chol_launch(double* G, int ldq, int q, int crows, int shift_mode, double* R, int* status,
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
      chol_blk_launch(G, ldq, q, crows, shift_mode, R, status, fail_bit, rank_cols, gate, st);
  }
}

template <int QT>
void triinv_reg_launch(const double* R, int ldr, int n, double* M, int ldm, double* Mt,
                       hipStream_t st) {
  hipLaunchKernelGGL((triinv_reg_kernel<QT>), dim3(1), dim3(256),
                     static_cast<size_t>(n) * (n + 1) * sizeof(double), st, R, ldr, n, M, ldm, Mt);
}

}  // namespace

// Triangular inverse of R[:n,:n] into M (and its transpose into Mt when
// given) with leading dimension ldm >= n, zero-padded, for n <= 224 (register tiles on 16 x 16 or 32 x 32 thread
// grids; larger orders take the blocked kernels through launch_triinv).
hipError_t tri_inverse(const double* R, int ldr, int n, double* M, int ldm, double* Mt,
                       hipStream_t st) {
  const size_t shm32 = static_cast<size_t>(n) * 33 * sizeof(double);
  switch (reg_tiles(n)) {
#define TLS_TRI32(K)                                                                          \
  case 100 + K:                                                                               \
    hipLaunchKernelGGL((triinv_reg32_kernel<K>), dim3(1), dim3(1024), shm32, st, R, ldr, n, M, \
                       ldm, Mt);                                                                  \
    break;
    TLS_TRI32(5) TLS_TRI32(6) TLS_TRI32(7)
#undef TLS_TRI32
    case 1: triinv_reg_launch<1>(R, ldr, n, M, ldm, Mt, st); break;
    case 2: triinv_reg_launch<2>(R, ldr, n, M, ldm, Mt, st); break;
    case 3: triinv_reg_launch<3>(R, ldr, n, M, ldm, Mt, st); break;
    case 4: triinv_reg_launch<4>(R, ldr, n, M, ldm, Mt, st); break;
    case 5: triinv_reg_launch<5>(R, ldr, n, M, ldm, Mt, st); break;
    case 6: triinv_reg_launch<6>(R, ldr, n, M, ldm, Mt, st); break;
    case 7: triinv_reg_launch<7>(R, ldr, n, M, ldm, Mt, st); break;
    case 8: triinv_reg_launch<8>(R, ldr, n, M, ldm, Mt, st); break;
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

template <bool RALL>
__global__ __launch_bounds__(64) void trsm_tile_gated_kernel(const int* __restrict__ gate,
                                                             double* __restrict__ A, int ldq, int q,
                                                             const double* __restrict__ R) {
  if (!(*gate & 8)) return;
  trsm_tile_body<RALL>(A, ldq, q, R, blockIdx.x);
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
  // the tile TRSM where its LDS fits (ldq <= TRSM_TILE_LDQ_MAX), else the
  // global-memory one; the third sweep is gated on status bit 8 from the
  // second Cholesky (tile path)
  const bool tile = ldq <= TRSM_TILE_LDQ_MAX;
  const bool gate3 = sweeps == 3 && tile;
  const size_t trsm_shm = trsm_lds_bytes(ldq);
  const bool rall = trsm_rall(ldq);
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    const bool gated = gate3 && sweep == 2;
    if (gated)
      hipLaunchKernelGGL(gram_gated_kernel, dim3(nt * nt), dim3(256), 0, st, status, A, crows, ldq, G);
    else
      hipLaunchKernelGGL(gram_kernel, dim3(nt * nt), dim3(256), 0, st, A, crows, ldq, G);
    chol_launch(G, ldq, q, crows, sweep == 0 ? 1 : 2, Rs[sweep], status, sweep == 0 ? 1 : 2,
                rank_cols, gated ? status : nullptr, st);
    if (sweep == sweeps - 1) break;
    if (tile) {
      if (gate3 && sweep == 1) {
        if (rall)
          hipLaunchKernelGGL(trsm_tile_gated_kernel<true>, dim3(crows / 16), dim3(64), trsm_shm, st,
                             status, A, ldq, q, Rs[sweep]);
        else
          hipLaunchKernelGGL(trsm_tile_gated_kernel<false>, dim3(crows / 16), dim3(64), trsm_shm, st,
                             status, A, ldq, q, Rs[sweep]);
      } else if (rall) {
        hipLaunchKernelGGL(trsm_tile_kernel<true>, dim3(crows / 16), dim3(64), trsm_shm, st, A, ldq,
                           q, Rs[sweep]);
      } else {
        hipLaunchKernelGGL(trsm_tile_kernel<false>, dim3(crows / 16), dim3(64), trsm_shm, st, A, ldq,
                           q, Rs[sweep]);
      }
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
                         int* status, hipStream_t st, double* dminmax) {
  if (p < 1 || q < p) return hipErrorInvalidValue;
  if (reg_tiles(p) != 0) {
    hipError_t e = tri_inverse(R, q, p, M, p, Mt, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((triinv_finish_kernel<1024>), dim3(1), dim3(1024), 0, st, R, q, p, M, phi0,
                       status, dminmax);
  } else {
    inv_blk_launch(R, q, p, M, Mt, phi0, status, dminmax, st);
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
  chol_reg_body<QT>(d.G, d.ldq, d.q, d.crows, shift_mode, R, status, fail_bit, d.p);
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

template <bool RALL>
__global__ __launch_bounds__(64) void trsm_b_kernel(const Item* __restrict__ items,
                                                    const FitDesc* __restrict__ D, int which) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  if (which == 1 && !(d.status[0] & 8)) return;  // only feeds the third sweep
  trsm_tile_body<RALL>(d.A, d.ldq, d.q, which == 0 ? d.R1 : d.R2, it.idx);
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
                                                       const FitDesc* __restrict__ D) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  triinv_reg_body<QT>(d.R, d.q, d.p, d.M, d.p, d.Mt);
  __syncthreads();
  triinv_finish_body<256>(d.R, d.q, d.p, d.M, d.phi0, d.status + 1);
  diag_range(d);
}

// 128 < p <= 224: the 32 x 32 thread grid
template <int QT>
__global__ __launch_bounds__(1024) void triinv_b32_kernel(const Item* __restrict__ items,
                                                          const FitDesc* __restrict__ D) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  triinv_reg32_body<QT>(d.R, d.q, d.p, d.M, d.p, d.Mt);
  __syncthreads();
  triinv_finish_body<1024>(d.R, d.q, d.p, d.M, d.phi0, d.status + 1);
  diag_range(d);
}

// Blocked Cholesky and inverse of the fits of a launch with q (or p) above
// 224: workgroup w serves fit items[w / per] with index w % per; indices
// beyond that fit's block count return at once.
__global__ __launch_bounds__(256) void chol_blk_init_b_kernel(const Item* __restrict__ items,
                                                              const FitDesc* __restrict__ D,
                                                              int sweep, int attempt, int per) {
  const FitDesc& d = D[items[blockIdx.x / per].fit];
  double* R;
  int* status;
  int shift_mode, fail_bit;
  chol_target(d, sweep, &R, &status, &shift_mode, &fail_bit);
  chol_blk_init_body(d.G, d.ldq, d.q, d.crows, shift_mode, attempt, sweep == 2 ? d.status : nullptr,
                     R, d.p, blk_scratch(d.G, d.ldq, d.q), blockIdx.x % per);
}

__global__ __launch_bounds__(256) void chol_blk_panel_b_kernel(const Item* __restrict__ items,
                                                               const FitDesc* __restrict__ D,
                                                               int sweep, int k, int per) {
  const FitDesc& d = D[items[blockIdx.x / per].fit];
  double* R;
  int* status;
  int shift_mode, fail_bit;
  chol_target(d, sweep, &R, &status, &shift_mode, &fail_bit);
  chol_blk_panel_body(d.q, R, d.p, blk_scratch(d.G, d.ldq, d.q), k, blockIdx.x % per);
}

__global__ __launch_bounds__(64) void chol_blk_finish_b_kernel(const Item* __restrict__ items,
                                                               const FitDesc* __restrict__ D,
                                                               int sweep, int attempt) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  double* R;
  int* status;
  int shift_mode, fail_bit;
  chol_target(d, sweep, &R, &status, &shift_mode, &fail_bit);
  chol_blk_finish_body(shift_mode, attempt, status, fail_bit, blk_scratch(d.G, d.ldq, d.q));
}

void chol_blk_b(const Item* fits, int nfits, int ldqmax, int sweep, const FitDesc* D,
                hipStream_t st) {
  const int nbk = (ldqmax + NBK - 1) / NBK;
  const int per0 = nbk * (nbk + 1) / 2;
  for (int attempt = sweep <= 0 ? 1 : 0; attempt < 2; ++attempt) {
    hipLaunchKernelGGL(chol_blk_init_b_kernel, dim3(nfits * per0), dim3(256), 0, st, fits, D, sweep,
                       attempt, per0);
    for (int k = 0; k + 1 < nbk; ++k) {
      const int m = nbk - 1 - k;
      const int per = m * (m + 1) / 2;
      hipLaunchKernelGGL(chol_blk_panel_b_kernel, dim3(nfits * per), dim3(256), 0, st, fits, D,
                         sweep, k, per);
    }
    hipLaunchKernelGGL(chol_blk_finish_b_kernel, dim3(nfits), dim3(64), 0, st, fits, D, sweep,
                       attempt);
  }
}

__global__ __launch_bounds__(256) void inv_blk_diag_b_kernel(const Item* __restrict__ items,
                                                             const FitDesc* __restrict__ D,
                                                             int per) {
  const FitDesc& d = D[items[blockIdx.x / per].fit];
  const int b = blockIdx.x % per;
  if (b >= (d.p + NBK - 1) / NBK) return;
  inv_blk_diag_body(d.R, d.q, d.p, d.M, d.Mt, b);
}

__global__ __launch_bounds__(256) void inv_blk_off_b_kernel(const Item* __restrict__ items,
                                                            const FitDesc* __restrict__ D,
                                                            int dist, int per) {
  const FitDesc& d = D[items[blockIdx.x / per].fit];
  const int i = blockIdx.x % per;
  if (i + dist >= (d.p + NBK - 1) / NBK) return;
  inv_blk_off_body(d.R, d.q, d.p, d.M, d.Mt, dist, i);
}

__global__ __launch_bounds__(256) void inv_blk_finish_b_kernel(const Item* __restrict__ items,
                                                               const FitDesc* __restrict__ D,
                                                               int per) {
  const FitDesc& d = D[items[blockIdx.x / per].fit];
  inv_blk_finish_body(d.R, d.q, d.p, d.M, d.Mt, d.phi0, d.status + 1, d.dminmax, blockIdx.x % per);
}

void inv_blk_b(const Item* fits, int nfits, int pmax, const FitDesc* D, hipStream_t st) {
  const int nbp = (pmax + NBK - 1) / NBK;
  hipLaunchKernelGGL(inv_blk_diag_b_kernel, dim3(nfits * nbp), dim3(256), 0, st, fits, D, nbp);
  for (int dist = 1; dist < nbp; ++dist)
    hipLaunchKernelGGL(inv_blk_off_b_kernel, dim3(nfits * (nbp - dist)), dim3(256), 0, st, fits, D,
                       dist, nbp - dist);
  const int per = nbp * nbp + nbp;
  hipLaunchKernelGGL(inv_blk_finish_b_kernel, dim3(nfits * per), dim3(256), 0, st, fits, D, per);
}

template <int QT>
hipError_t qr_b_qt(int stage, const Item* tiles, int ntiles, const Item* rowtiles, int nrowtiles,
                   const Item* rows, int nrows, const Item* fits, int nfits, int ldqmax,
                   const FitDesc* D, hipStream_t st) {
  const size_t trsm_shm = trsm_lds_bytes(ldqmax);
  const int sweeps = stage == 1 ? 1 : 3;
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    hipLaunchKernelGGL(gram_b_kernel, dim3(ntiles), dim3(256), 0, st, tiles, D,
                       stage == 2 && sweep == 2 ? 1 : 0);
    if constexpr (QT > 100)
      hipLaunchKernelGGL((chol_b32_kernel<(QT > 100 ? QT - 100 : 1)>), dim3(nfits), dim3(1024), 0, st,
                         fits, D, stage == 1 ? -1 : sweep);
    else if constexpr (QT > 0)
      hipLaunchKernelGGL((chol_b_kernel<QT>), dim3(nfits), dim3(256), 0, st, fits, D,
                         stage == 1 ? -1 : sweep);
    else
      chol_blk_b(fits, nfits, ldqmax, stage == 1 ? -1 : sweep, D, st);
    if (sweep < sweeps - 1)
      hipLaunchKernelGGL((trsm_b_kernel<(QT >= 1 && QT <= 8)>), dim3(nrowtiles), dim3(64), trsm_shm,
                         st, rowtiles, D, sweep);
  }
  if (stage == 2) {
    hipLaunchKernelGGL(trmm_b_kernel, dim3(nrows), dim3(256), 0, st, rows, D, 0);
    hipLaunchKernelGGL(trmm_b_kernel, dim3(nrows), dim3(256), 0, st, rows, D, 1);
  }
  hipLaunchKernelGGL(rank_test_b_kernel, dim3(nfits), dim3(64), 0, st, fits, D, stage);
  return hipGetLastError();
}

template <int QT>
hipError_t triinv_b_qt(const Item* fits, int nfits, int pmax, const FitDesc* D, hipStream_t st) {
  if constexpr (QT > 100) {
    const size_t shm = static_cast<size_t>(pmax) * 33 * sizeof(double);
    hipLaunchKernelGGL((triinv_b32_kernel<(QT > 100 ? QT - 100 : 1)>), dim3(nfits), dim3(1024), shm, st,
                       fits, D);
  } else if constexpr (QT > 0) {
    const size_t shm = static_cast<size_t>(pmax) * (pmax + 1) * sizeof(double);
    hipLaunchKernelGGL((triinv_b_kernel<QT>), dim3(nfits), dim3(256), shm, st, fits, D);
  } else {
    inv_blk_b(fits, nfits, pmax, D, st);
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
hipError_t launch_triinv_b(int pt, const Item* fits, int nfits, int pmax, const FitDesc* D,
                           hipStream_t st) {
  if (nfits < 1) return hipSuccess;
  switch (pt) {
    case 0: return triinv_b_qt<0>(fits, nfits, pmax, D, st);
    case 1: return triinv_b_qt<1>(fits, nfits, pmax, D, st);
    case 2: return triinv_b_qt<2>(fits, nfits, pmax, D, st);
    case 3: return triinv_b_qt<3>(fits, nfits, pmax, D, st);
    case 4: return triinv_b_qt<4>(fits, nfits, pmax, D, st);
    case 5: return triinv_b_qt<5>(fits, nfits, pmax, D, st);
    case 6: return triinv_b_qt<6>(fits, nfits, pmax, D, st);
    case 7: return triinv_b_qt<7>(fits, nfits, pmax, D, st);
    case 8: return triinv_b_qt<8>(fits, nfits, pmax, D, st);
    case 105: return triinv_b_qt<105>(fits, nfits, pmax, D, st);
    case 106: return triinv_b_qt<106>(fits, nfits, pmax, D, st);
    case 107: return triinv_b_qt<107>(fits, nfits, pmax, D, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tls
