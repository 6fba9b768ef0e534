// Randomized sketch kernels: Philox draws, row gathers of [X | b], leverage
// score sampling (Algorithm 2, eq. (ldist)) and the k-column JL map
// Omega = M Pi^T of eq. (glev) with a subsampled randomized Hadamard map
// (Definition 2.4, Algorithm 1) or a Gaussian map.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace tls {

namespace {

__global__ void philox_uniform_kernel(double* __restrict__ out, int64_t count, uint32_t stream,
                                      uint32_t fit, uint64_t seed, uint64_t start) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = philox_u01(start + static_cast<uint64_t>(i), stream, fit, seed);
}

// Row t of the sketch: scale * [X(idx,:), b(idx)], zero-padded to ldq columns;
// rows t >= c are zero.  mode 0: given idx/scale; 1: uniform trials (Algorithm
// 1: idx = floor(u m), scale sqrt(m/c)); 2: every row (c == m, scale 1).
__device__ __forceinline__ void gather_body(const double* __restrict__ y, int64_t m, int p,
                                                    int mode, const int64_t* __restrict__ idx,
                                                    const double* __restrict__ scale, int c,
                                                    int ldq, double* __restrict__ A,
                                                    int64_t* __restrict__ idx_out,
                                                    double* __restrict__ scale_out, uint64_t seed,
                                                    uint32_t fit, int t) {
  double* row = A + static_cast<size_t>(t) * ldq;
  if (t >= c) {
    for (int j = threadIdx.x; j < ldq; j += 64) row[j] = 0.0;
    return;
  }
  int64_t ii;
  double sc;
  if (mode == 0) {
    ii = idx[t];
    sc = scale[t];
  } else if (mode == 1) {
    const double u = philox_u01(static_cast<uint64_t>(t), RNG_UNIFORM_ROWS, fit, seed);
    ii = static_cast<int64_t>(floor(u * static_cast<double>(m)));
    if (ii > m - 1) ii = m - 1;
    sc = sqrt(static_cast<double>(m) / static_cast<double>(c));
  } else {
    ii = t;
    sc = 1.0;
  }
  for (int j = threadIdx.x; j < ldq; j += 64) {
    double v = 0.0;
    if (j < p)
      v = sc * y[p - 1 + ii - j];
    else if (j == p)
      v = sc * y[p + ii];
    row[j] = v;
  }
  if (threadIdx.x == 0) {
    if (idx_out) idx_out[t] = ii;
    if (scale_out) scale_out[t] = sc;
  }
}

__global__ __launch_bounds__(64) void gather_kernel(const double* __restrict__ y, int64_t m, int p,
                                                    int mode, const int64_t* __restrict__ idx,
                                                    const double* __restrict__ scale, int c,
                                                    int ldq, double* __restrict__ A,
                                                    int64_t* __restrict__ idx_out,
                                                    double* __restrict__ scale_out, uint64_t seed,
                                                    uint32_t fit) {
  gather_body(y, m, p, mode, idx, scale, c, ldq, A, idx_out, scale_out, seed, fit, blockIdx.x);
}

constexpr int CHUNK = 4096;

template <typename T, int NT>
__device__ __forceinline__ void chunk_sum_body(const T* __restrict__ s, int64_t m,
                                                       double* __restrict__ out, int chunk) {
  __shared__ double red[NT / 64];
  const int64_t base = static_cast<int64_t>(chunk) * CHUNK;
  double acc = 0.0;
  // all of the thread's loads in flight, added in row order
  constexpr int PER = CHUNK / NT;
  double v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t g = base + threadIdx.x + static_cast<int64_t>(k) * NT;
    v[k] = g < m ? static_cast<double>(s[g]) : 0.0;
  }
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (base + threadIdx.x + static_cast<int64_t>(k) * NT < m) acc += v[k];
  const double tot = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) out[chunk] = tot;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void chunk_sum_kernel(const T* __restrict__ s, int64_t m,
                                                       double* __restrict__ out) {
  chunk_sum_body<T, NT>(s, m, out, blockIdx.x);
}

// Exclusive prefix of the chunk sums in chunk order: pre[0] = 0, pre[k+1] =
// pre[k] + sums[k]; pre[nch] is the total.  One workgroup.
template <int NT>
__device__ __forceinline__ void chunk_prefix_body(const double* __restrict__ sums,
                                                          int nch, double* __restrict__ pre) {
  __shared__ double buf[NT];
  __shared__ double carry;
  if (threadIdx.x == 0) {
    carry = 0.0;
    pre[0] = 0.0;
  }
  __syncthreads();
  for (int base = 0; base < nch; base += NT) {
    const int i = base + threadIdx.x;
    buf[threadIdx.x] = i < nch ? sums[i] : 0.0;
    __syncthreads();
    // inclusive Hillis-Steele scan over NT entries
    for (int off = 1; off < NT; off <<= 1) {
      const double v = threadIdx.x >= off ? buf[threadIdx.x - off] : 0.0;
      __syncthreads();
      buf[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < nch) pre[i + 1] = carry + buf[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) carry += buf[NT - 1];
    __syncthreads();
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void chunk_prefix_kernel(const double* __restrict__ sums,
                                                          int nch, double* __restrict__ pre) {
  chunk_prefix_body<NT>(sums, nch, pre);
}

__device__ __forceinline__ double wave_incl_scan(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// One wavefront per draw: target = u * total; find the last chunk whose
// prefix is <= target by a 64-way search (each round probes 64 evenly spaced
// prefixes and keeps the bracket of the last one <= target), then the first
// row of the chunk whose running total exceeds the target.  The chunk is
// staged in LDS so that lane l owns rows 64 l .. 64 l + 63 of it: a wave
// scan of the lane totals gives each lane its starting total, every lane
// runs its 64 rows in order, and the lowest lane that crosses the target
// holds the draw.  scale = 1 / sqrt(c * s_i / total).
template <typename T>
__device__ __forceinline__ void draw_body(const T* __restrict__ s, int64_t m,
                                          const double* __restrict__ pre, int nch,
                                          const double* __restrict__ u, int c,
                                          int64_t* __restrict__ idx,
                                          double* __restrict__ scale, uint64_t seed,
                                          uint32_t fit, int t, uint64_t draw0 = 0) {
  __shared__ double seg[CHUNK + CHUNK / 64];  // row e of the chunk at e + e / 64
  const int lane = threadIdx.x;
  const double total = pre[nch];
  const double ut = u ? u[t] : philox_u01(draw0 + static_cast<uint64_t>(t), RNG_LEVERAGE, fit, seed);
  const double target = ut * total;
  int lo = 0, hi = nch - 1;  // invariant: pre[lo] <= target
  while (lo < hi) {
    const int step = (hi - lo + 64) / 64;
    const int k = lo + lane * step;
    const uint64_t le = __ballot(k <= hi && pre[k] <= target);
    // le has lane 0 unless the target is not a number (scores that are not
    // finite): then lo stays, so every index stays inside the chunks
    lo += (le ? 63 - __builtin_clzll(le) : 0) * step;
    hi = min(hi, lo + step - 1);
  }
  const int64_t base = static_cast<int64_t>(lo) * CHUNK;
  // the chunk's rows, 32 loads in flight per lane before any is stored
#pragma unroll
  for (int i0 = 0; i0 < 64; i0 += 32) {
    double tv[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int64_t g = base + (i0 + i) * 64 + lane;
      tv[i] = g < m ? static_cast<double>(s[g]) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) seg[(i0 + i) * 65 + lane] = tv[i];
  }
  __syncthreads();
  double v[64];
  double loc = 0.0;
  int lastk = -1;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    v[k] = seg[lane * 65 + k];
    loc += v[k];
    if (v[k] > 0.0) lastk = k;
  }
  const double incl = wave_incl_scan(loc);
  const double up = __shfl_up(incl, 1, 64);
  double running = pre[lo] + (lane ? up : 0.0);
  int hitk = -1;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    running += v[k];
    if (hitk < 0 && running > target && v[k] > 0.0) hitk = k;
  }
  int64_t found;
  const uint64_t hit = __ballot(hitk >= 0);
  if (hit) {
    const int L = __builtin_ctzll(hit);
    found = base + 64 * L + __shfl(hitk, L, 64);
  } else {
    // target within rounding of the chunk end: its last positive row
    const uint64_t pos = __ballot(lastk >= 0);
    if (pos) {
      const int L = 63 - __builtin_clzll(pos);
      found = base + 64 * L + __shfl(lastk, L, 64);
    } else {
      found = base;  // an all-zero chunk cannot be reached by a positive total
    }
  }
  if (lane == 0) {
    idx[t] = found;
    const double sv = static_cast<double>(s[found]);
    scale[t] = 1.0 / sqrt(static_cast<double>(c) * sv / total);
  }
}

template <typename T>
__global__ __launch_bounds__(64) void draw_kernel(const T* __restrict__ s, int64_t m,
                                                  const double* __restrict__ pre, int nch,
                                                  const double* __restrict__ u, int c,
                                                  int64_t* __restrict__ idx,
                                                  double* __restrict__ scale, uint64_t seed,
                                                  uint32_t fit, uint64_t draw0) {
  draw_body<T>(s, m, pre, nch, u, c, idx, scale, seed, fit, blockIdx.x, draw0);
}

// Repeated halving: zero the scores of the rows outside level `level` (row r
// is kept when its level draw u_r < 2^-level: nested uniform subsets of
// about m / 2^level rows).
template <typename T>
__global__ __launch_bounds__(256) void rh_mask_kernel(T* __restrict__ s, int64_t m, int level,
                                                      uint64_t seed, uint32_t fit) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (r >= m) return;
  const double u = philox_u01(static_cast<uint64_t>(r), RNG_RH_LEVEL, fit, seed);
  if (!(u < ldexp(1.0, -level))) s[r] = T(0);
}

// Entry j of row q of the k x p JL map Pi.  kind 0: subsampled randomized
// Hadamard map, Pi[q][j] = d_j (-1)^popcount(r_q & j) / sqrt(k) with
// d_j = +-1 from the sign stream and r_q uniform in [0, P), P the power of
// two >= p; kind 1: Gaussian N(0, 1/k) entries (Box-Muller).
struct JlRow {
  int kind;
  uint32_t rq;
  double invsk;
};

__device__ __forceinline__ JlRow jl_row(int p, int k, int kind, uint64_t seed, uint32_t fit,
                                        int q) {
  JlRow g{kind, 0u, 1.0 / sqrt(static_cast<double>(k))};
  if (kind == 0) {
    int P = 1;
    while (P < p) P <<= 1;
    const double ur = philox_u01(static_cast<uint64_t>(q), RNG_SRHT_ROWS, fit, seed);
    int64_t r = static_cast<int64_t>(floor(ur * static_cast<double>(P)));
    if (r > P - 1) r = P - 1;
    g.rq = static_cast<uint32_t>(r);
  }
  return g;
}

__device__ __forceinline__ double jl_entry(const JlRow& g, int p, int q, int j, uint64_t seed,
                                           uint32_t fit) {
  if (g.kind == 0) {
    const double us = philox_u01(static_cast<uint64_t>(j), RNG_SRHT_SIGNS, fit, seed);
    const double d = us < 0.5 ? 1.0 : -1.0;
    const double h = (__popc(g.rq & static_cast<uint32_t>(j)) & 1) ? -1.0 : 1.0;
    return d * h * g.invsk;
  }
  const uint64_t e = static_cast<uint64_t>(q) * p + j;
  const double u1 = philox_u01(2 * e, RNG_GAUSS, fit, seed);
  const double u2 = philox_u01(2 * e + 1, RNG_GAUSS, fit, seed);
  return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2) * g.invsk;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Rows c0 .. c0 + KC - 1 (those below k) of Pi and the same columns of
// Omega = R[:p,:p]^{-1} Pi^T (p x k, column-major; R upper triangular,
// row-major with leading dimension ldr) by back substitution, one wavefront
// for all of them: lane l holds b_j of every column for j = l + 64 t
// (t < T), step s takes x_s = b_s (1 / R_ss) of each column from the lane
// holding b_s (a register read with a uniform lane index) and updates the
// rows above it with column s of R, loaded once for all the columns.  The
// column loads and the reciprocals do not depend on the solution, so each
// block of U columns is prepared while the previous block is solved.

template <int T, int U, int KC>
__device__ __forceinline__ void jl_solve_body(const double* __restrict__ R, int ldr, int p, int k,
                                              int kind, double* __restrict__ Pi,
                                              double* __restrict__ Om, uint64_t seed,
                                              uint32_t fit, int c0) {
  const int lane = static_cast<int>(threadIdx.x);
  double b[T][KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int q = c0 + c;
    const JlRow g = jl_row(p, k, kind, seed, fit, q < k ? q : 0);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int j = lane + 64 * t;
      b[t][c] = (q < k && j < p) ? jl_entry(g, p, q, j, seed, fit) : 0.0;
      if (Pi && q < k && j < p) Pi[static_cast<size_t>(q) * p + j] = b[t][c];
    }
  }
  // column s of R above the diagonal (zero elsewhere) and 1 / R_ss
  auto load = [&](int s0, double (&rc)[U][T], double (&dg)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = s0 - u;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int j = lane + 64 * t;
        rc[u][t] = (s >= 0 && j < s) ? R[static_cast<size_t>(j) * ldr + s] : 0.0;
      }
      dg[u] = s >= 0 ? R[static_cast<size_t>(s) * ldr + s] : 1.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) dg[u] = 1.0 / dg[u];
  };
  auto solve = [&](int s0, const double (&rc)[U][T], const double (&dg)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = s0 - u;
      if (s < 0) break;
      const int ts = s >> 6, ls = s & 63;
      double xs[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        double bs = b[0][c];
#pragma unroll
        for (int t = 1; t < T; ++t)
          if (t == ts) bs = b[t][c];
        xs[c] = readlane_f64(bs * dg[u], ls);
      }
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          if (t == ts && lane == ls) b[t][c] = xs[c];
          b[t][c] = fma(-rc[u][t], xs[c], b[t][c]);
        }
    }
  };
  double ra[U][T], rb[U][T], da[U], db[U];
  load(p - 1, ra, da);
  for (int s0 = p - 1; s0 >= 0; s0 -= 2 * U) {
    load(s0 - U, rb, db);
    solve(s0, ra, da);
    load(s0 - 2 * U, ra, da);
    solve(s0 - U, rb, db);
  }
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int q = c0 + c;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int j = lane + 64 * t;
      if (q < k && j < p) Om[static_cast<size_t>(q) * p + j] = b[t][c];
    }
  }
}

// Columns per wavefront by rows per lane, as jl_cols of the order: batched
// fits take one wavefront for several columns (the column loads of R shared
// by all of them); a single fit, one wavefront per column (the k chains in
// parallel on separate CUs).
template <int T>
constexpr int jl_kc() {
  return T <= 2 ? 8 : (T <= 4 ? 4 : (T <= 8 ? 2 : 1));
}

template <int T, int U>
__global__ __launch_bounds__(64) void jl_solve_kernel(const double* __restrict__ R, int ldr, int p,
                                                      int k, int kind, double* __restrict__ Pi,
                                                      double* __restrict__ Om, uint64_t seed,
                                                      uint32_t fit) {
  jl_solve_body<T, U, 1>(R, ldr, p, k, kind, Pi, Om, seed, fit, blockIdx.x);
}

}  // namespace

hipError_t launch_philox_uniform(double* out, int64_t count, uint32_t stream, uint32_t fit,
                                 uint64_t seed, uint64_t start, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t nb = (count + 255) / 256;
  hipLaunchKernelGGL(philox_uniform_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, st,
                     out, count, stream, fit, seed, start);
  return hipGetLastError();
}

hipError_t launch_gather(const double* y, int64_t m, int p, int mode, const int64_t* idx,
                         const double* scale, int c, int crows, int ldq, double* A, int64_t* idx_out,
                         double* scale_out, uint64_t seed, uint32_t fit, hipStream_t st) {
  if (crows < c || ldq < p + 1 || crows < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_kernel, dim3(crows), dim3(64), 0, st, y, m, p, mode, idx, scale, c,
                     ldq, A, idx_out, scale_out, seed, fit);
  return hipGetLastError();
}

size_t sample_work_doubles(int64_t m) {
  const int64_t nch = (m + CHUNK - 1) / CHUNK;
  return static_cast<size_t>(2 * nch + 1);
}

hipError_t launch_rh_mask(int prec, void* scores, int64_t m, int level, uint64_t seed,
                          uint32_t fit, hipStream_t st) {
  if (m < 1 || level < 0) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((m + 255) / 256));
  if (prec == PREC_F64)
    hipLaunchKernelGGL((rh_mask_kernel<double>), grid, dim3(256), 0, st, static_cast<double*>(scores),
                       m, level, seed, fit);
  else
    hipLaunchKernelGGL((rh_mask_kernel<float>), grid, dim3(256), 0, st, static_cast<float*>(scores),
                       m, level, seed, fit);
  return hipGetLastError();
}

hipError_t launch_sample(int prec, const void* scores, int64_t m, const double* u, int c,
                         int64_t* idx, double* scale, double* work, uint64_t seed, uint32_t fit,
                         hipStream_t st, uint64_t draw0) {
  if (m < 1 || c < 1) return hipErrorInvalidValue;
  const int nch = static_cast<int>((m + CHUNK - 1) / CHUNK);
  double* sums = work;
  double* pre = work + nch;
  if (prec == PREC_F64) {
    hipLaunchKernelGGL((chunk_sum_kernel<double, 256>), dim3(nch), dim3(256), 0, st,
                       static_cast<const double*>(scores), m, sums);
  } else {
    hipLaunchKernelGGL((chunk_sum_kernel<float, 256>), dim3(nch), dim3(256), 0, st,
                       static_cast<const float*>(scores), m, sums);
  }
  hipLaunchKernelGGL((chunk_prefix_kernel<256>), dim3(1), dim3(256), 0, st, sums, nch, pre);
  if (prec == PREC_F64) {
    hipLaunchKernelGGL((draw_kernel<double>), dim3(c), dim3(64), 0, st,
                       static_cast<const double*>(scores), m, pre, nch, u, c, idx, scale, seed,
                       fit, draw0);
  } else {
    hipLaunchKernelGGL((draw_kernel<float>), dim3(c), dim3(64), 0, st,
                       static_cast<const float*>(scores), m, pre, nch, u, c, idx, scale, seed,
                       fit, draw0);
  }
  return hipGetLastError();
}

hipError_t launch_jl_solve(const double* R, int ldr, int p, int k, int kind, double* Pi,
                           double* Om, uint64_t seed, uint32_t fit, hipStream_t st) {
  if (p < 1 || k < 1 || p > 1024 || ldr < p) return hipErrorInvalidValue;
#define TLS_JL(T, U)                                                                             \
  hipLaunchKernelGGL((jl_solve_kernel<T, U>), dim3(k), dim3(64), 0, st, \
                     R, ldr, p, k, kind, Pi, \
                     Om, seed, fit)
  if (p <= 64)
    TLS_JL(1, 8);
  else if (p <= 128)
    TLS_JL(2, 8);
  else if (p <= 256)
    TLS_JL(4, 4);
  else if (p <= 512)
    TLS_JL(8, 4);
  else
    TLS_JL(16, 2);
#undef TLS_JL
  return hipGetLastError();
}

}  // namespace tls

// ---- batched launches ---------------------------------------------------------
namespace tls {
namespace {

// stage 1: uniform trials (every row when the sketch covers all rows);
// stage 2: the sampled rows and scales of the leverage stage.
__global__ __launch_bounds__(64) void gather_b_kernel(const Item* __restrict__ items,
                                                      const FitDesc* __restrict__ D, int stage,
                                                      uint64_t seed) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  const int mode = d.all_rows ? 2 : (stage == 1 ? 1 : 0);
  gather_body(d.y, d.m, d.p, mode, d.idx, d.scale, d.c, d.ldq, d.A, mode == 1 ? d.idx : nullptr,
              mode == 1 ? d.scale : nullptr, seed, d.fit, it.idx);
}

template <typename T>
__global__ __launch_bounds__(256) void chunk_sum_b_kernel(const Item* __restrict__ items,
                                                          const FitDesc* __restrict__ D) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  chunk_sum_body<T, 256>(static_cast<const T*>(d.u), d.m, d.swork, it.idx);
}

__global__ __launch_bounds__(256) void chunk_prefix_b_kernel(const Item* __restrict__ items,
                                                             const FitDesc* __restrict__ D) {
  const FitDesc& d = D[items[blockIdx.x].fit];
  chunk_prefix_body<256>(d.swork, d.nchunks, d.swork + d.nchunks);
}

template <typename T>
__global__ __launch_bounds__(64) void draw_b_kernel(const Item* __restrict__ items,
                                                    const FitDesc* __restrict__ D, uint64_t seed) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  draw_body<T>(static_cast<const T*>(d.u), d.m, d.swork + d.nchunks, d.nchunks, nullptr, d.c, d.idx,
               d.scale, seed, d.fit, it.idx);
}

// Omega of the stage-1 factor (in R after the stage-1 sweep), one
// wavefront per (fit, group of jl_cols(pmax) columns) item.
template <int T, int U>
__global__ __launch_bounds__(64) void jl_b_kernel(const Item* __restrict__ items,
                                                  const FitDesc* __restrict__ D, int kind,
                                                  uint64_t seed) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  jl_solve_body<T, U, jl_kc<T>()>(d.R, d.q, d.p, d.k, kind, d.Pi, d.Om, seed, d.fit,
                                  it.idx * jl_kc<T>());
}

}  // namespace

hipError_t launch_gather_b(int stage, const Item* items, int nitems, const FitDesc* D,
                           uint64_t seed, hipStream_t st) {
  if (nitems < 1) return hipSuccess;
  hipLaunchKernelGGL(gather_b_kernel, dim3(nitems), dim3(64), 0, st, items, D, stage, seed);
  return hipGetLastError();
}

// fit_items: one item per fit that samples (idx unused).
hipError_t launch_sample_b(int prec, const Item* chunk_items, int nchunk_items,
                           const Item* draw_items, int ndraw_items, const Item* fit_items,
                           int nfit_items, const FitDesc* D, uint64_t seed, hipStream_t st) {
  if (nfit_items < 1) return hipSuccess;
  if (prec == PREC_F64)
    hipLaunchKernelGGL((chunk_sum_b_kernel<double>), dim3(nchunk_items), dim3(256), 0, st,
                       chunk_items, D);
  else
    hipLaunchKernelGGL((chunk_sum_b_kernel<float>), dim3(nchunk_items), dim3(256), 0, st,
                       chunk_items, D);
  hipLaunchKernelGGL(chunk_prefix_b_kernel, dim3(nfit_items), dim3(256), 0, st, fit_items, D);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((draw_b_kernel<double>), dim3(ndraw_items), dim3(64), 0, st, draw_items, D,
                       seed);
  else
    hipLaunchKernelGGL((draw_b_kernel<float>), dim3(ndraw_items), dim3(64), 0, st, draw_items, D,
                       seed);
  return hipGetLastError();
}

hipError_t launch_jl_b(const Item* items, int nitems, const FitDesc* D, int kind, int pmax,
                       uint64_t seed, hipStream_t st) {
  if (nitems < 1) return hipSuccess;
  if (pmax > 1024) return hipErrorInvalidValue;
#define TLS_JL_B(T, U)                                                                       \
  hipLaunchKernelGGL((jl_b_kernel<T, U>), dim3(nitems), dim3(64), 0, st, items, D, kind, seed)
  if (pmax <= 64)
    TLS_JL_B(1, 8);
  else if (pmax <= 128)
    TLS_JL_B(2, 8);
  else if (pmax <= 256)
    TLS_JL_B(4, 4);
  else if (pmax <= 512)
    TLS_JL_B(8, 4);
  else
    TLS_JL_B(16, 2);
#undef TLS_JL_B
  return hipGetLastError();
}

}  // namespace tls
