// QR factorisation of the sketch [S X | S b] (Section 2.1: the compressed
// problem is solved through a QR factorisation of SA) by shifted Cholesky QR
// in three sweeps (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J.
// Sci. Comput. 2020): G = A^T A + s I -> R1, A <- A R1^{-1}; G = A^T A -> R2,
// A <- A R2^{-1}; G = A^T A -> R3; R = R3 R2 R1.  The shift
// s = 11 (c q + q (q + 1)) u trace(A^T A) keeps the first Cholesky factorable
// up to condition numbers near 1/u; the later sweeps restore orthogonality.
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
__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ A, int crows, int ldq,
                                                   double* __restrict__ G) {
  const int nt = ldq / 16;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
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

// Right-looking Cholesky of G[:q,:q] (+ shift on the diagonal) into the upper
// factor R (row-major q x q, zero below the diagonal).  One workgroup; the
// working copy lives in R.
template <int NT>
__global__ __launch_bounds__(NT) void chol_kernel(const double* __restrict__ G, int ldq, int q,
                                                  int crows, int shift, double* __restrict__ R,
                                                  int* __restrict__ status, int fail_bit,
                                                  int rank_cols) {
  __shared__ double red[NT / 64];
  __shared__ double s_shift, s_floor;
  double tr = 0.0;
  for (int i = threadIdx.x; i < q; i += NT) tr += G[static_cast<size_t>(i) * ldq + i];
  tr = block_sum<NT>(tr, red);
  if (threadIdx.x == 0) {
    s_shift = shift ? 11.0 * (static_cast<double>(crows) * q + static_cast<double>(q) * (q + 1)) *
                          0x1p-53 * tr
                    : 0.0;
    s_floor = tr > 0.0 ? tr * 0x1p-104 : 1e-300;
  }
  for (int e = threadIdx.x; e < q * q; e += NT) {
    const int i = e / q, k = e % q;
    R[e] = (k >= i) ? G[static_cast<size_t>(i) * ldq + k] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 0; i < q; ++i) R[static_cast<size_t>(i) * q + i] += s_shift;
  __syncthreads();
  bool failed = false;
  for (int j = 0; j < q; ++j) {
    double d = R[static_cast<size_t>(j) * q + j];
    if (!(d > s_floor)) {
      if (j < rank_cols) failed = true;  // later columns may be exactly dependent (b in range)
      d = s_floor;
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
  if (failed && threadIdx.x == 0) atomicOr(status, fail_bit);
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
__global__ __launch_bounds__(64) void trsm_global_kernel(double* __restrict__ A, int crows, int ldq,
                                                         int q, const double* __restrict__ R) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= crows) return;
  double* row = A + static_cast<size_t>(t) * ldq;
  for (int j = 0; j < q; ++j) {
    const double* rj = R + static_cast<size_t>(j) * q;
    const double x = row[j] / rj[j];
    row[j] = x;
    for (int k = j + 1; k < q; ++k) row[k] -= x * rj[k];
  }
}

// C = Ra Rb for upper-triangular q x q (row-major); one workgroup per row.
template <int NT>
__global__ __launch_bounds__(NT) void trmm_kernel(const double* __restrict__ Ra,
                                                  const double* __restrict__ Rb, int q,
                                                  double* __restrict__ C) {
  const int i = blockIdx.x;
  const double* ra = Ra + static_cast<size_t>(i) * q;
  for (int j = threadIdx.x; j < q; j += NT) {
    double acc = 0.0;
    for (int k = i; k <= j; ++k) acc += ra[k] * Rb[static_cast<size_t>(k) * q + j];
    C[static_cast<size_t>(i) * q + j] = acc;
  }
}

// M = R[:p,:p]^{-1} (row-major, upper), Mt = M^T, phi0 = M R[:p, p] (the
// compressed problem's solution), and the rank test min|R_ii| <= p u max|R_ii|.
template <int NT>
__global__ __launch_bounds__(NT) void triinv_kernel(const double* __restrict__ R, int q, int p,
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
  for (int e = threadIdx.x; e < p * p; e += NT) {
    const int i = e / p, j = e % p;
    Mt[static_cast<size_t>(j) * p + i] = M[e];
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

// status |= 4 when min|R_ii| <= k u max|R_ii| over the first k = rank_cols
// diagonal entries (numerical rank of the leading columns below k).
__global__ void rank_test_kernel(const double* __restrict__ R, int q, int rank_cols,
                                 int* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = INFINITY;
  for (int i = 0; i < rank_cols; ++i) {
    const double d = fabs(R[static_cast<size_t>(i) * q + i]);
    a = fmax(a, d);
    b = fmin(b, d);
  }
  if (!(b > static_cast<double>(rank_cols) * 0x1p-53 * a)) atomicOr(status, 4);
}

}  // namespace

// G must hold ldq*ldq + 2*q*q doubles (Gram matrix, then R3 and R3 R2).
hipError_t launch_qr(double* A, int crows, int q, int ldq, int rank_cols, double* R, double* G,
                     double* R1, double* R2, int* status, hipStream_t st) {
  if (crows % 4 != 0 || ldq % 16 != 0 || q > ldq || q < 1) return hipErrorInvalidValue;
  const int nt = ldq / 16;
  double* R3 = G + static_cast<size_t>(ldq) * ldq;
  double* T = R3 + static_cast<size_t>(q) * q;
  double* Rs[3] = {R1, R2, R3};
  for (int sweep = 0; sweep < 3; ++sweep) {
    hipLaunchKernelGGL(gram_kernel, dim3(nt * nt), dim3(256), 0, st, A, crows, ldq, G);
    hipLaunchKernelGGL((chol_kernel<256>), dim3(1), dim3(256), 0, st, G, ldq, q, crows,
                       sweep == 0 ? 1 : 0, Rs[sweep], status, sweep == 0 ? 1 : 2, rank_cols);
    if (sweep == 2) break;
    if (q <= 128) {
      hipLaunchKernelGGL((trsm_kernel<64, 128>), dim3((crows + 63) / 64), dim3(64), 0, st, A,
                         crows, ldq, q, Rs[sweep]);
    } else {
      hipLaunchKernelGGL(trsm_global_kernel, dim3((crows + 63) / 64), dim3(64), 0, st, A, crows,
                         ldq, q, Rs[sweep]);
    }
  }
  hipLaunchKernelGGL((trmm_kernel<256>), dim3(q), dim3(256), 0, st, R3, R2, q, T);
  hipLaunchKernelGGL((trmm_kernel<256>), dim3(q), dim3(256), 0, st, T, R1, q, R);
  hipLaunchKernelGGL(rank_test_kernel, dim3(1), dim3(64), 0, st, R, q, rank_cols, status);
  return hipGetLastError();
}

hipError_t launch_triinv(const double* R, int q, int p, double* M, double* Mt, double* phi0,
                         int* status, hipStream_t st) {
  if (p < 1 || q < p) return hipErrorInvalidValue;
  hipLaunchKernelGGL((triinv_kernel<256>), dim3(1), dim3(256), 0, st, R, q, p, M, Mt, phi0,
                     status);
  return hipGetLastError();
}

}  // namespace tls
