// Blocked circulant-embedding kernels for the lag matrix of eq. (xphi).
//
// Layout (0-based): X[i, j] = y[p-1+i-j], b[i] = y[p+i], m = n - p rows.
// Block k covers rows [kL, kL+L), L = B - p + 1, and owns the window
// y[kL .. kL+B) (zero past the end of y).  Inside the window, row i sits at
// position tau = i - kL + p - 1 in [p-1, B): the circular convolution of the
// window with v (zero-padded to B) at tau is exactly (X v)[i], and the
// circular correlation of the window with the block's rows placed at
// tau in [p-1, B) gives that block's share of (X^T u)[j] at j < p (no
// wrap-around in either, since every index difference stays in [0, B)).
//
// Spectra are stored packed: N = B/2 complex words per block, word 0 holding
// (X[0], X[N]) (both real) and word k the bin X[k] for 0 < k < N.
#pragma once

#include <type_traits>

#include "fft.h"
#include "kernels.h"

namespace tls {

template <typename T>
__device__ __forceinline__ void load_pair(const cx<T>* __restrict__ P, int k, int N, cx<T>& a,
                                          cx<T>& b) {
  if (k == 0) {
    const cx<T> w0 = P[0];
    a = {w0.x, T(0)};
    b = {w0.y, T(0)};
  } else {
    a = P[k];
    b = P[N - k];
  }
}

// The bin pairs (k, N-k) of a packed spectrum for k = tid + ip NT < N/2,
// plus the self-paired bin N/2, all loaded before any is used so that the
// whole set costs one memory round trip.  With `tab`, also the real-FFT
// twiddles exp(-2 pi i k / B) of those bins.
template <typename T, int LGN, int NT>
struct PairLoads {
  static constexpr int N = 1 << LGN;
  static constexpr int NP = (N / 2 + NT - 1) / NT;
  static constexpr bool FULL = NP * NT == N / 2;  // every (thread, ip) has a bin
  cx<T> a[NP], b[NP], w[NP], yh, wh;
  __device__ __forceinline__ void load(const cx<T>* __restrict__ P, const cx<T>* __restrict__ tab) {
    const int tid = opaque_tid<NT>();
#pragma unroll
    for (int ip = 0; ip < NP; ++ip) {
      int k = tid + ip * NT;
      if (!FULL) k = k < N / 2 ? k : 0;
      a[ip] = P[k];
      b[ip] = P[(N - k) & (N - 1)];
      if (tab) w[ip] = twiddle<T, false>(tab, k, LGN + 1);
    }
    yh = P[N / 2];
    if (tab) wh = twiddle<T, false>(tab, N / 2, LGN + 1);
  }
  // the twiddles alone (bins kept from an earlier load)
  __device__ __forceinline__ void load_tw(const cx<T>* __restrict__ tab) {
    const int tid = opaque_tid<NT>();
#pragma unroll
    for (int ip = 0; ip < NP; ++ip) {
      int k = tid + ip * NT;
      if (!FULL) k = k < N / 2 ? k : 0;
      w[ip] = twiddle<T, false>(tab, k, LGN + 1);
    }
    wh = twiddle<T, false>(tab, N / 2, LGN + 1);
  }
  // the bins k and N-k (bin 0 pairs with bin N: both real, packed in word 0)
  __device__ __forceinline__ void get(int ip, int k, cx<T>& xk, cx<T>& xnk) const {
    xk = a[ip];
    xnk = b[ip];
    if (k == 0) {
      xk = {a[ip].x, T(0)};
      xnk = {a[ip].y, T(0)};
    }
  }
};

// The bins of a PairLoads without its twiddles, kept between two uses.
template <typename T, int LGN, int NT>
struct PairBins {
  static constexpr int NP = PairLoads<T, LGN, NT>::NP;
  cx<T> a[NP], b[NP], yh;
  __device__ __forceinline__ void take(const PairLoads<T, LGN, NT>& l) {
#pragma unroll
    for (int ip = 0; ip < NP; ++ip) {
      a[ip] = l.a[ip];
      b[ip] = l.b[ip];
    }
    yh = l.yh;
  }
  __device__ __forceinline__ void give(PairLoads<T, LGN, NT>& l) const {
#pragma unroll
    for (int ip = 0; ip < NP; ++ip) {
      l.a[ip] = a[ip];
      l.b[ip] = b[ip];
    }
    l.yh = yh;
  }
};

// ---------------------------------------------------------------------------
// Block spectra of the series (computed in FP64, stored as TS).
template <int LGN, int NT, typename TS>
__device__ __forceinline__ void spectra_body(const double* __restrict__ y, int64_t n, int L,
                                                     cx<TS>* __restrict__ Yhat,
                                                     const cx<double>* __restrict__ tab, int blk) {
  constexpr int N = 1 << LGN;
  __shared__ cx<double> s[N];
  const int64_t start = static_cast<int64_t>(blk) * L;
  // up to 8 sample pairs per thread in flight before any is stored
  for (int t0 = threadIdx.x; t0 < N; t0 += 8 * NT) {
    cx<double> v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t i0 = start + 2 * (t0 + k * NT);
      v[k] = {t0 + k * NT < N && i0 < n ? y[i0] : 0.0,
              t0 + k * NT < N && i0 + 1 < n ? y[i0 + 1] : 0.0};
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (t0 + k * NT < N) s[swz<double>(t0 + k * NT)] = v[k];
  }
  __syncthreads();
  fft_dif<double, false, LGN, NT>(s, tab);
  cx<TS>* out = Yhat + static_cast<size_t>(blk) * N;
  for (int k = threadIdx.x; k <= N / 2; k += NT) {
    const cx<double> w = twiddle<double, false>(tab, k, LGN + 1);
    cx<double> Xk, Xnk;
    rfft_post(s[swz<double>(bitrev(k, LGN))], s[swz<double>(bitrev((N - k) & (N - 1), LGN))], w, Xk, Xnk);
    if (k == 0) {
      out[0] = {static_cast<TS>(Xk.x), static_cast<TS>(Xnk.x)};
    } else {
      out[k] = {static_cast<TS>(Xk.x), static_cast<TS>(Xk.y)};
      if (2 * k != N) out[N - k] = {static_cast<TS>(Xnk.x), static_cast<TS>(Xnk.y)};
    }
  }
}

template <int LGN, int NT, typename TS>
__global__ __launch_bounds__(NT) void spectra_kernel(const double* __restrict__ y, int64_t n, int L,
                                                     cx<TS>* __restrict__ Yhat,
                                                     const cx<double>* __restrict__ tab) {
  spectra_body<LGN, NT, TS>(y, n, L, Yhat, tab, blockIdx.x);
}

// Packed spectra (times `scale`) of short real columns zero-padded to B.
template <int LGN, int NT, typename TS>
__device__ __forceinline__ void small_rfft_body(const double* __restrict__ cols, int len,
                                                        int ld, double scale,
                                                        cx<TS>* __restrict__ out,
                                                        const cx<double>* __restrict__ tab,
                                                        const int* __restrict__ flag, int col_idx) {
  constexpr int N = 1 << LGN;
  __shared__ cx<double> s[N];
  if (flag && *flag) return;
  const double* col = cols + static_cast<size_t>(col_idx) * ld;
  for (int t = threadIdx.x; t < N; t += NT) {
    const int i0 = 2 * t;
    s[swz<double>(t)] = {i0 < len ? col[i0] : 0.0, i0 + 1 < len ? col[i0 + 1] : 0.0};
  }
  __syncthreads();
  fft_dif<double, false, LGN, NT>(s, tab);
  cx<TS>* o = out + static_cast<size_t>(col_idx) * N;
  for (int k = threadIdx.x; k <= N / 2; k += NT) {
    const cx<double> w = twiddle<double, false>(tab, k, LGN + 1);
    cx<double> Xk, Xnk;
    rfft_post(s[swz<double>(bitrev(k, LGN))], s[swz<double>(bitrev((N - k) & (N - 1), LGN))], w, Xk, Xnk);
    Xk = cscale(Xk, scale);
    Xnk = cscale(Xnk, scale);
    if (k == 0) {
      o[0] = {static_cast<TS>(Xk.x), static_cast<TS>(Xnk.x)};
    } else {
      o[k] = {static_cast<TS>(Xk.x), static_cast<TS>(Xk.y)};
      if (2 * k != N) o[N - k] = {static_cast<TS>(Xnk.x), static_cast<TS>(Xnk.y)};
    }
  }
}

template <int LGN, int NT, typename TS>
__global__ __launch_bounds__(NT) void small_rfft_kernel(const double* __restrict__ cols, int len,
                                                        int ld, double scale,
                                                        cx<TS>* __restrict__ out,
                                                        const cx<double>* __restrict__ tab,
                                                        const int* __restrict__ flag) {
  small_rfft_body<LGN, NT, TS>(cols, len, ld, scale, out, tab, flag, blockIdx.x);
}

// ---------------------------------------------------------------------------
// One pass over all blocks.  With v's packed spectrum pre-scaled by 1/B:
//   e = s1 * (X v) + s2 * w          (PM_MV; the w term when w_in != NULL)
//   u_out = e                        (when u_out != NULL; may alias w_in)
//   partial[j*ngroups + g] = share of (X^T e)[j] of block group g, j < p  (PM_RMV)
//   partial[p*ngroups + g] = share of ||e||^2 of block group g
// Without PM_MV the pass vector is u_in.  (s1, s2) = coef[0..1].
//
// A workgroup holds NW groups of NT threads; group `sub` transforms block
// g NW + sub in its own LDS region (blocks past the end contribute zero).
// X^T e needs only the first p outputs of the inverse transform of the sum
// over blocks of conj(Y_b) E_b (the transform is linear and the same for
// every block), so the NW product spectra are added in LDS in a fixed order
// and one inverse transform per workgroup replaces one per block.
template <typename T, int LGN, int NT, int NW, int MODE, bool KEEP_OK = true>
__device__ __forceinline__ void toep_pass_body(
    const cx<T>* __restrict__ Yhat, const cx<T>* __restrict__ Vhat, const T* w_in, T* u_out,
    const T* __restrict__ u_in, double* __restrict__ partial, const double* __restrict__ coef,
    const int* __restrict__ flag, const cx<T>* __restrict__ tab, int64_t m, int p, int L,
    int nblocks, int ngroups, int grp) {
  constexpr int N = 1 << LGN;
  constexpr int NEL = N / NT;
  constexpr int NTW = NT * NW;
  static_assert(N % NT == 0, "block transform must cover the thread group");
  __shared__ cx<T> s_all[NW * N];
  __shared__ double red[NTW / 64];
  if (flag && *flag) return;
  const int tid = static_cast<int>(threadIdx.x) & (NT - 1);
  const int sub = NW == 1 ? 0 : static_cast<int>(threadIdx.x) / NT;
  const int braw = grp * NW + sub;
  const bool valid = braw < nblocks;
  const int blk = valid ? braw : nblocks - 1;  // in-bounds loads; no rows below
  cx<T>* const s = s_all + sub * N;
  const cx<T>* Y = Yhat + static_cast<size_t>(blk) * N;
  const int64_t row0 = static_cast<int64_t>(blk) * L - (p - 1);  // row at tau = 0

  double nrm = 0.0;
  // Y kept in registers between its two uses in the FP64 passes of 1024-
  // and 4096-point blocks, where the pass's LDS already holds occupancy at
  // four waves per SIMD and the kept bins fit under that register budget
  // (126 and 125 VGPRs): at B = 1024 the second read had missed L2 (about
  // the whole 37 MB of spectra per AR(100) pass came from HBM twice)
  // (KEEP_OK false: the batched kernels, whose extra registers would cost
  // a wave per SIMD)
  constexpr bool KEEPY = KEEP_OK && sizeof(T) == 8 && (MODE & PM_MV) != 0 && (MODE & PM_RMV) != 0 &&
                         ((LGN == 9 && NT == 64 && NW == 4) || (LGN == 11 && NT == 256 && NW == 2));
  struct NoKeep {};
  std::conditional_t<KEEPY, PairBins<T, LGN, NT>, NoKeep> ykeep;
  if constexpr ((MODE & PM_MV) != 0) {
    // spectrum of X v on this block: Y * V (V pre-scaled by 1/B), in the
    // half-length complex form, bit-reversed for the inverse transform.
    // Every operand is loaded before any is used (one memory round trip).
    PairLoads<T, LGN, NT> ly, lv;
    ly.load(Y, tab);
    if constexpr (KEEPY) ykeep.take(ly);
    lv.load(Vhat, nullptr);
#pragma unroll
    for (int ip = 0; ip < PairLoads<T, LGN, NT>::NP; ++ip) {
      const int k = tid + ip * NT;
      if (PairLoads<T, LGN, NT>::FULL || k < N / 2) {
        cx<T> yk, ynk, vk, vnk;
        ly.get(ip, k, yk, ynk);
        lv.get(ip, k, vk, vnk);
        cx<T> Zk, Znk;
        irfft_pre(cmul(yk, vk), cmul(ynk, vnk), ly.w[ip], Zk, Znk);
        s[swz<T>(bitrev(k, LGN))] = Zk;
        if (k != 0) s[swz<T>(bitrev(N - k, LGN))] = Znk;
      }
    }
    if (tid == 0) {  // the self-paired bin N/2
      const cx<T> x = cmul(ly.yh, lv.yh);
      cx<T> Zk, Znk;
      irfft_pre(x, x, ly.wh, Zk, Znk);
      s[swz<T>(bitrev(N / 2, LGN))] = Zk;
    }
    group_sync<NT>();
  }
  // the rows of this block sit at window positions [p - 1, hi); they are
  // addressed by 32-bit offsets from the row at position 0 (the 64-bit base
  // is uniform; positions below p - 1 are never accessed).  A block past the
  // end has no rows (hi = 0): e = 0 there.
  const int hi = valid ? static_cast<int>(m - row0 < 2 * N ? m - row0 : 2 * N) : 0;
  T* const ub = u_out ? u_out + row0 : nullptr;
  // e at the rows of this block (zero outside them) from the inverse
  // transform value z = ((X v)[2t], (X v)[2t+1]) at packed position t
  auto emap = [&](int t, cx<T> z, T wa, T wb) -> cx<T> {
    const T s1 = static_cast<T>(coef[0]);
    const T s2 = static_cast<T>(coef[1]);
    T o0 = T(0), o1 = T(0);
    // explicit fused operations: the same rounding in every kernel that
    // inlines this pass, whatever the compiler knows about w_in there
    if (2 * t >= p - 1 && 2 * t < hi) {
      o0 = s1 * z.x;
      if (w_in) o0 = fma(s2, wa, o0);
      if (ub) ub[2 * t] = o0;
    }
    if (2 * t + 1 >= p - 1 && 2 * t + 1 < hi) {
      o1 = s1 * z.y;
      if (w_in) o1 = fma(s2, wb, o1);
      if (ub) ub[2 * t + 1] = o1;
    }
    nrm = fma(static_cast<double>(o0), static_cast<double>(o0), nrm);
    nrm = fma(static_cast<double>(o1), static_cast<double>(o1), nrm);
    return cx<T>{o0, o1};
  };

  // v[e]: the value at packed position tid + e NT between the transforms
  // (their outermost butterflies run on it in registers)
  cx<T> v[NEL];
  if constexpr ((MODE & PM_MV) != 0) {
    fft_dit_out<T, true, LGN, NT>(s, tab, v);
    // the butterflies finish before the w loads are issued (hoisted above
    // them, the loads would keep both sets of registers live)
#pragma unroll
    for (int e = 0; e < NEL; ++e) asm volatile("" : "+v"(v[e].x), "+v"(v[e].y));
    asm volatile("" ::: "memory");
    // the w terms of all this thread's rows are loaded before any is used
    // (one memory round trip rather than one per element)
    T w0[NEL], w1[NEL];
    const T* const wbase = w_in ? w_in + row0 : nullptr;
#pragma unroll
    for (int e = 0; e < NEL; ++e) {
      const int r = 2 * (tid + e * NT);
      w0[e] = (wbase && r >= p - 1 && r < hi) ? wbase[r] : T(0);
      w1[e] = (wbase && r + 1 >= p - 1 && r + 1 < hi) ? wbase[r + 1] : T(0);
    }
#pragma unroll
    for (int e = 0; e < NEL; ++e) v[e] = emap(tid + e * NT, v[e], w0[e], w1[e]);
    settle(nrm);
    if constexpr ((MODE & PM_RMV) != 0) fft_dif_in<T, false, LGN, NT>(s, tab, v);
  } else {
    const T* const uib = u_in + row0;
#pragma unroll
    for (int e = 0; e < NEL; ++e) {
      const int t = tid + e * NT;
      const T o0 = (2 * t >= p - 1 && 2 * t < hi) ? uib[2 * t] : T(0);
      const T o1 = (2 * t + 1 >= p - 1 && 2 * t + 1 < hi) ? uib[2 * t + 1] : T(0);
      nrm = fma(static_cast<double>(o0), static_cast<double>(o0), nrm);
      nrm = fma(static_cast<double>(o1), static_cast<double>(o1), nrm);
      v[e] = {o0, o1};
    }
    settle(nrm);
    fft_dif_in<T, false, LGN, NT>(s, tab, v);
  }
  if constexpr ((MODE & PM_RMV) != 0) {
    // this block's share of X^T e: correlation of the window with e, i.e.
    // conj(E) * Y per bin pair (Y kept, or reloaded), left in the inverse
    // transform's input form
    PairLoads<T, LGN, NT> ly;
    if constexpr (KEEPY) {
      ykeep.give(ly);
      ly.load_tw(tab);
    } else {
      ly.load(Y, tab);
    }
#pragma unroll
    for (int ip = 0; ip < PairLoads<T, LGN, NT>::NP; ++ip) {
      const int k = tid + ip * NT;
      if (PairLoads<T, LGN, NT>::FULL || k < N / 2) {
        const int bk = bitrev(k, LGN);
        const int bnk = bitrev((N - k) & (N - 1), LGN);
        cx<T> Xk, Xnk;
        rfft_post(s[swz<T>(bk)], s[swz<T>(bnk)], ly.w[ip], Xk, Xnk);
        cx<T> yk2, ynk2;
        ly.get(ip, k, yk2, ynk2);
        cx<T> Zk, Znk;
        irfft_pre(cmulconj(yk2, Xk), cmulconj(ynk2, Xnk), ly.w[ip], Zk, Znk);
        s[swz<T>(bk)] = Zk;
        if (k != 0) s[swz<T>(bnk)] = Znk;
      }
    }
    if (tid == 0) {  // the self-paired bin N/2
      const int bh = bitrev(N / 2, LGN);
      cx<T> Xk, Xnk;
      const cx<T> z = s[swz<T>(bh)];
      rfft_post(z, z, ly.wh, Xk, Xnk);
      cx<T> Zk, Znk;
      irfft_pre(cmulconj(ly.yh, Xk), cmulconj(ly.yh, Xnk), ly.wh, Zk, Znk);
      s[swz<T>(bh)] = Zk;
    }
    if constexpr (NW == 1) group_sync<NT>();
    if constexpr (NW > 1) {
      __syncthreads();
      // the group's product spectra summed into region 0, blocks in order
      // (every region is addressed through the same swizzle)
      for (int i = static_cast<int>(threadIdx.x); i < N; i += NTW) {
        cx<T> acc = s_all[i];
#pragma unroll
        for (int w = 1; w < NW; ++w) acc = cadd(acc, s_all[w * N + i]);
        s_all[i] = acc;
      }
      __syncthreads();
    }
    fft_dit<T, true, LGN, NTW>(s_all, tab);
    const double invB = 1.0 / static_cast<double>(2 * N);
    for (int t = static_cast<int>(threadIdx.x); 2 * t < p; t += NTW) {
      const cx<T> z = s_all[swz<T>(t)];
      partial[static_cast<size_t>(2 * t) * ngroups + grp] = static_cast<double>(z.x) * invB;
      if (2 * t + 1 < p)
        partial[static_cast<size_t>(2 * t + 1) * ngroups + grp] = static_cast<double>(z.y) * invB;
    }
  }
  const double tot = block_sum<NTW>(nrm, red);
  if (threadIdx.x == 0) partial[static_cast<size_t>(p) * ngroups + grp] = tot;
}

template <typename T, int LGN, int NT, int NW, int MODE>
__global__ __launch_bounds__(NT * NW) void toep_pass_kernel(
    const cx<T>* __restrict__ Yhat, const cx<T>* __restrict__ Vhat, const T* w_in, T* u_out,
    const T* __restrict__ u_in, double* __restrict__ partial, const double* __restrict__ coef,
    const int* __restrict__ flag, const cx<T>* __restrict__ tab, int64_t m, int p, int L,
    int nblocks, int ngroups) {
  toep_pass_body<T, LGN, NT, NW, MODE>(Yhat, Vhat, w_in, u_out, u_in, partial, coef, flag, tab, m,
                                       p, L, nblocks, ngroups, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Approximate generalised leverage scores (eq. (glev) in product form):
// scores[i] = sum_q ((X omega_q)[i])^2 for k packed column spectra (scaled 1/B).
template <typename T, int LGN, int NT>
__device__ __forceinline__ void scores_body(const cx<T>* __restrict__ Yhat,
                                                    const cx<T>* __restrict__ Om, int kcols,
                                                    T* __restrict__ scores,
                                                    const cx<T>* __restrict__ tab, int64_t m,
                                                    int p, int L, int blk) {
  constexpr int N = 1 << LGN;
  constexpr int NPAIR = (N / 2 + 1 + NT - 1) / NT;
  constexpr int NEL = N / NT;
  __shared__ cx<T> s[N];
  const int tid = threadIdx.x;
  const cx<T>* Y = Yhat + static_cast<size_t>(blk) * N;
  const int64_t row0 = static_cast<int64_t>(blk) * L - (p - 1);
  cx<T> yk[NPAIR], ynk[NPAIR];
#pragma unroll
  for (int ip = 0; ip < NPAIR; ++ip) {
    const int k = tid + ip * NT;
    if (k <= N / 2) load_pair(Y, k, N, yk[ip], ynk[ip]);
  }
  T acc0[NEL], acc1[NEL];
#pragma unroll
  for (int e = 0; e < NEL; ++e) acc0[e] = acc1[e] = T(0);
  for (int q = 0; q < kcols; ++q) {
    const cx<T>* V = Om + static_cast<size_t>(q) * N;
#pragma unroll
    for (int ip = 0; ip < NPAIR; ++ip) {
      const int k = tid + ip * NT;
      if (k <= N / 2) {
        cx<T> vk, vnk;
        load_pair(V, k, N, vk, vnk);
        const cx<T> w = twiddle<T, false>(tab, k, LGN + 1);
        cx<T> Zk, Znk;
        irfft_pre(cmul(yk[ip], vk), cmul(ynk[ip], vnk), w, Zk, Znk);
        s[swz<T>(bitrev(k, LGN))] = Zk;
        if (k != 0 && 2 * k != N) s[swz<T>(bitrev(N - k, LGN))] = Znk;
      }
    }
    __syncthreads();
    fft_dit<T, true, LGN, NT>(s, tab);
#pragma unroll
    for (int e = 0; e < NEL; ++e) {
      const cx<T> z = s[swz<T>(tid + e * NT)];
      acc0[e] += z.x * z.x;
      acc1[e] += z.y * z.y;
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < NEL; ++e) {
    const int t = tid + e * NT;
    const int64_t i0 = row0 + 2 * t;
    if (2 * t >= p - 1 && i0 < m) scores[i0] = acc0[e];
    if (2 * t + 1 >= p - 1 && i0 + 1 < m) scores[i0 + 1] = acc1[e];
  }
}

template <typename T, int LGN, int NT>
__global__ __launch_bounds__(NT) void scores_kernel(const cx<T>* __restrict__ Yhat,
                                                    const cx<T>* __restrict__ Om, int kcols,
                                                    T* __restrict__ scores,
                                                    const cx<T>* __restrict__ tab, int64_t m,
                                                    int p, int L) {
  scores_body<T, LGN, NT>(Yhat, Om, kcols, scores, tab, m, p, L, blockIdx.x);
}

}  // namespace tls
