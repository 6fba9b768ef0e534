// Shared device/host definitions for the Toeplitz least-squares library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tls {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulconj(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// The index of the calling thread within its group of NT threads (NT a power
// of two; NT = the workgroup size gives threadIdx.x), as a value the compiler
// cannot see through: index and address arithmetic derived from it in one
// phase of a kernel is then redone in the next rather than kept live in
// registers across the phases between.
template <int NT>
__device__ __forceinline__ int opaque_tid() {
  static_assert((NT & (NT - 1)) == 0, "thread groups are powers of two");
  int t = static_cast<int>(threadIdx.x) & (NT - 1);
  asm volatile("" : "+v"(t));
  return t;
}

// Make the accumulator x materialise here: the products folded into it are
// evaluated now instead of being deferred (with their operands kept live) to
// x's first later use.
__device__ __forceinline__ void settle(double& x) { asm volatile("" : "+v"(x)); }

__device__ __forceinline__ int bitrev(int k, int lg) {
  return static_cast<int>(__builtin_bitreverse32(static_cast<uint32_t>(k)) >> (32 - lg));
}

// Largest transform: real length 2^LG_BMAX (complex half-length 2^(LG_BMAX-1)).
constexpr int LG_BMAX = 14;
constexpr int BMAX = 1 << LG_BMAX;
constexpr int NMAX = BMAX / 2;

// Wave-level sum (64 lanes) using cross-lane shuffles.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-level sum in a fixed order (deterministic); `scratch` holds >= NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += scratch[i];
  return t;
}

// Sum of a column of nblocks partials in one fixed order for any workgroup
// of NT >= 256 threads: thread t < 256 adds rows t, t + 256, ..., then the
// four wavefront sums are added in order (the same result as block_sum<256>
// over those threads).  `scratch` holds >= 4 doubles.
template <int NT>
__device__ __forceinline__ double column_sum(const double* __restrict__ col, int nblocks,
                                             double* scratch) {
  static_assert(NT >= 256, "column_sum needs 256 threads");
  double s = 0.0;
  if (threadIdx.x < 256) {
    // up to 24 loads in flight per round (one round up to 6144 blocks),
    // added in the plain loop's order
    constexpr int U = 24;
    for (int b = threadIdx.x; b < nblocks; b += U * 256) {
      double v[U];
#pragma unroll
      for (int k = 0; k < U; ++k) v[k] = b + 256 * k < nblocks ? col[b + 256 * k] : 0.0;
#pragma unroll
      for (int k = 0; k < U; ++k) s += v[k];
    }
  }
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0 && wid < 4) scratch[wid] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) t += scratch[i];
  return t;
}

}  // namespace tls

namespace tls {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
// (c0,c1,c2,c3) <- (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)),
// key advanced by the Weyl constants between rounds.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(M0) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(M1) * c[2];
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Draw j of stream s for fit f under seed S: counter (j, 0, s, f), key
// (S mod 2^32, S >> 32); u = ((x0 << 32 | x1) >> 12 + 0.5) * 2^-52 in (0,1).
__host__ __device__ inline double philox_u01(uint64_t j, uint32_t stream, uint32_t fit, uint64_t seed) {
  uint32_t c[4] = {static_cast<uint32_t>(j), 0u, stream, fit};
  philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const uint64_t bits = ((static_cast<uint64_t>(c[0]) << 32) | c[1]) >> 12;
  return (static_cast<double>(bits) + 0.5) * 0x1p-52;
}

// Random-number streams of one fit.
enum RngStream : uint32_t {
  RNG_UNIFORM_ROWS = 0,  // stage-1 uniform row trials
  RNG_SRHT_SIGNS = 1,    // signs of the randomized Hadamard map
  RNG_SRHT_ROWS = 2,     // rows of the randomized Hadamard map
  RNG_LEVERAGE = 3,      // leverage-score draws
  RNG_GAUSS = 4,         // Gaussian JL map (Box-Muller pairs)
  RNG_RH_LEVEL = 5,      // repeated halving: row r belongs to level i when u_r < 2^-i
};

}  // namespace tls
