// Workgroup FFT core on LDS for gfx950.
//
// A real sequence x of length B = 2N is transformed through the complex
// sequence z[t] = x[2t] + i x[2t+1] of length N.  The complex transforms are
// radix-2 decimation passes fused three levels at a time (8 points per
// thread in registers, one LDS round trip per three levels):
//   fft_dif: natural-order input  -> bit-reversed output (forward, e^{-i})
//   fft_dit: bit-reversed input   -> natural-order output (inverse, e^{+i})
// so a forward transform followed by a pointwise product and an inverse
// transform never needs a permutation pass.  Inverse transforms are
// unscaled.  Real <-> half-length complex conversion works on bin pairs
// (k, N-k) (rfft_post / irfft_pre), which every caller does in registers.
//
// Twiddles come from one table built once on the host in extended
// precision that holds, for every power of two L <= BMAX, the L/2 factors
// w_L^e = exp(-2 pi i e / L), e < L/2, contiguously from index L/2 - 1: the
// threads of a stage, which need consecutive exponents of one L, then read
// consecutive words.
#pragma once

#include "common.h"

namespace tls {

// LDS index swizzle: one 256-byte LDS row holds 16 complex doubles (32
// complex floats); XOR-ing the column with the row number spreads both
// power-of-two strides (small-span passes) and bit-reversed scatters across
// all banks.  A bijection on [0, N) for N >= one row.
template <typename T>
__device__ __forceinline__ int swz(int i) {
  constexpr int LG = sizeof(cx<T>) == 16 ? 4 : 5;
  return i ^ ((i >> LG) & ((1 << LG) - 1));
}

// Barrier of a group of NT threads that exchange data through LDS.  A
// group within one wavefront needs none: its LDS operations are performed in
// issue order, so the fences only keep the compiler from moving LDS
// accesses across this point.
template <int NT>
__device__ __forceinline__ void group_sync() {
  if constexpr (NT <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tab, int e, int lgL) {
  cx<T> w = tab[((1 << lgL) >> 1) - 1 + e];
  if (INV) w.y = -w.y;
  return w;
}

// Forward twiddles of one radix-R stage for the offset r within its span h:
// w1 = w_{2h}^r, w2 = w_{4h}^r (R >= 4), w3a = w_{8h}^r and
// w3b = w_{8h}^{r+h} (R = 8).  At h = 1 (r = 0) they are constants.  The
// inverse stages use the conjugates, so one set serves both directions.
template <typename T, int R, int LGH>
struct Tw {
  cx<T> w1, w2, w3a, w3b;
  __device__ __forceinline__ Tw(const cx<T>* __restrict__ tab, int r) {
    if constexpr (R == 8 && LGH == 0) {
      constexpr T c = T(0.70710678118654752440084436210484903928);
      w1 = {T(1), T(0)};
      w2 = {T(1), T(0)};
      w3a = {T(1), T(0)};
      w3b = {c, -c};
    } else {
      w1 = twiddle<T, false>(tab, r, LGH + 1);
      if constexpr (R >= 4) w2 = twiddle<T, false>(tab, r, LGH + 2);
      if constexpr (R == 8) {
        w3a = twiddle<T, false>(tab, r, LGH + 3);
        w3b = twiddle<T, false>(tab, r + (1 << LGH), LGH + 3);
      }
    }
  }
};

template <typename T, bool INV>
__device__ __forceinline__ cx<T> cj(cx<T> w) {
  return INV ? cx<T>{w.x, -w.y} : w;
}

// a * w, skipping the product when w is the constant 1 (exact either way).
template <typename T, bool ONE>
__device__ __forceinline__ cx<T> tmul(cx<T> a, cx<T> w) {
  if constexpr (ONE) return a;
  else return cmul(a, w);
}

// ---- butterflies on registers: points base + k*h, h = 2^LGH -----------------
// Decimation in time: levels of span h, 2h, 4h (radix 8), h, 2h (radix 4), h.
template <typename T, bool INV, int LGH>
__device__ __forceinline__ void bfly_dit8(cx<T> (&a)[8], const Tw<T, 8, LGH>& tw) {
  constexpr bool C = LGH == 0;
  const cx<T> w1 = cj<T, INV>(tw.w1), w2 = cj<T, INV>(tw.w2);
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    const cx<T> b = tmul<T, C>(a[k + 1], w1);
    a[k + 1] = csub(a[k], b);
    a[k] = cadd(a[k], b);
  }
#pragma unroll
  for (int k0 = 0; k0 < 8; k0 += 4) {
    cx<T> b = tmul<T, C>(a[k0 + 2], w2);
    a[k0 + 2] = csub(a[k0], b);
    a[k0] = cadd(a[k0], b);
    b = C ? rot90<T, INV>(a[k0 + 3]) : cmul(a[k0 + 3], rot90<T, INV>(w2));
    a[k0 + 3] = csub(a[k0 + 1], b);
    a[k0 + 1] = cadd(a[k0 + 1], b);
  }
  const cx<T> w3a = cj<T, INV>(tw.w3a), w3b = cj<T, INV>(tw.w3b);
  const cx<T> w3[4] = {w3a, w3b, rot90<T, INV>(w3a), rot90<T, INV>(w3b)};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const cx<T> b = (C && k == 0) ? a[k + 4] : (C && k == 2) ? rot90<T, INV>(a[k + 4])
                                                             : cmul(a[k + 4], w3[k]);
    a[k + 4] = csub(a[k], b);
    a[k] = cadd(a[k], b);
  }
}

template <typename T, bool INV, int LGH>
__device__ __forceinline__ void bfly_dit4(cx<T> (&a)[4], const Tw<T, 4, LGH>& tw) {
  const cx<T> w1 = cj<T, INV>(tw.w1), w2 = cj<T, INV>(tw.w2);
#pragma unroll
  for (int k = 0; k < 4; k += 2) {
    const cx<T> b = cmul(a[k + 1], w1);
    a[k + 1] = csub(a[k], b);
    a[k] = cadd(a[k], b);
  }
  cx<T> b = cmul(a[2], w2);
  a[2] = csub(a[0], b);
  a[0] = cadd(a[0], b);
  b = cmul(a[3], rot90<T, INV>(w2));
  a[3] = csub(a[1], b);
  a[1] = cadd(a[1], b);
}

template <typename T, bool INV, int LGH>
__device__ __forceinline__ void bfly_dit2(cx<T> (&a)[2], const Tw<T, 2, LGH>& tw) {
  const cx<T> b = cmul(a[1], cj<T, INV>(tw.w1));
  a[1] = csub(a[0], b);
  a[0] = cadd(a[0], b);
}

// Decimation in frequency: levels of span 4h, 2h, h (radix 8), 2h, h, h.
template <typename T, bool INV, int LGH>
__device__ __forceinline__ void bfly_dif8(cx<T> (&a)[8], const Tw<T, 8, LGH>& tw) {
  constexpr bool C = LGH == 0;
  const cx<T> w3a = cj<T, INV>(tw.w3a), w3b = cj<T, INV>(tw.w3b);
  const cx<T> w3[4] = {w3a, w3b, rot90<T, INV>(w3a), rot90<T, INV>(w3b)};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const cx<T> t = csub(a[k], a[k + 4]);
    a[k] = cadd(a[k], a[k + 4]);
    a[k + 4] = (C && k == 0) ? t : (C && k == 2) ? rot90<T, INV>(t) : cmul(t, w3[k]);
  }
  const cx<T> w1 = cj<T, INV>(tw.w1), w2 = cj<T, INV>(tw.w2);
#pragma unroll
  for (int k0 = 0; k0 < 8; k0 += 4) {
    cx<T> t = csub(a[k0], a[k0 + 2]);
    a[k0] = cadd(a[k0], a[k0 + 2]);
    a[k0 + 2] = tmul<T, C>(t, w2);
    t = csub(a[k0 + 1], a[k0 + 3]);
    a[k0 + 1] = cadd(a[k0 + 1], a[k0 + 3]);
    a[k0 + 3] = C ? rot90<T, INV>(t) : cmul(t, rot90<T, INV>(w2));
  }
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    const cx<T> t = csub(a[k], a[k + 1]);
    a[k] = cadd(a[k], a[k + 1]);
    a[k + 1] = tmul<T, C>(t, w1);
  }
}

template <typename T, bool INV, int LGH>
__device__ __forceinline__ void bfly_dif4(cx<T> (&a)[4], const Tw<T, 4, LGH>& tw) {
  const cx<T> w1 = cj<T, INV>(tw.w1), w2 = cj<T, INV>(tw.w2);
  cx<T> t = csub(a[0], a[2]);
  a[0] = cadd(a[0], a[2]);
  a[2] = cmul(t, w2);
  t = csub(a[1], a[3]);
  a[1] = cadd(a[1], a[3]);
  a[3] = cmul(t, rot90<T, INV>(w2));
#pragma unroll
  for (int k = 0; k < 4; k += 2) {
    t = csub(a[k], a[k + 1]);
    a[k] = cadd(a[k], a[k + 1]);
    a[k + 1] = cmul(t, w1);
  }
}

template <typename T, bool INV, int LGH>
__device__ __forceinline__ void bfly_dif2(cx<T> (&a)[2], const Tw<T, 2, LGH>& tw) {
  const cx<T> t = csub(a[0], a[1]);
  a[0] = cadd(a[0], a[1]);
  a[1] = cmul(t, cj<T, INV>(tw.w1));
}

template <typename T, bool DIT, bool INV, int R, int LGH>
__device__ __forceinline__ void bfly(cx<T> (&a)[R], const Tw<T, R, LGH>& tw) {
  if constexpr (R == 8) {
    if constexpr (DIT) bfly_dit8<T, INV, LGH>(a, tw);
    else bfly_dif8<T, INV, LGH>(a, tw);
  } else if constexpr (R == 4) {
    if constexpr (DIT) bfly_dit4<T, INV, LGH>(a, tw);
    else bfly_dif4<T, INV, LGH>(a, tw);
  } else {
    if constexpr (DIT) bfly_dit2<T, INV, LGH>(a, tw);
    else bfly_dif2<T, INV, LGH>(a, tw);
  }
}

// One radix-R stage over the LDS array: thread loop over the N/R point groups.
template <typename T, bool DIT, bool INV, int N, int NT, int R, int LGH>
__device__ __forceinline__ void stage(cx<T>* s, const cx<T>* __restrict__ tab) {
  constexpr int h = 1 << LGH;
  constexpr int LGR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  for (int q = opaque_tid<NT>(); q < N / R; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> LGH) << (LGH + LGR)) + r;
    cx<T> a[R];
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = s[swz<T>(base + k * h)];
    const Tw<T, R, LGH> tw(tab, r);
    bfly<T, DIT, INV, R, LGH>(a, tw);
#pragma unroll
    for (int k = 0; k < R; ++k) s[swz<T>(base + k * h)] = a[k];
  }
}

// Stage plans.  DIT: radix-8 stages from span 1 upward, then one radix-4 or
// radix-2 stage for the remaining levels; DIF: the mirror image.
template <int LGN>
struct Plan8 {
  static constexpr int REM = LGN % 3;
  static constexpr int RLAST = REM == 0 ? 8 : (REM == 2 ? 4 : 2);  // radix of the outer stage
  static constexpr int LGLAST = LGN - (REM == 0 ? 3 : REM);         // its span exponent
};

template <typename T, bool INV, int LGN, int NT, int LGH, bool SKIP_LAST>
__device__ __forceinline__ void dit_from(cx<T>* s, const cx<T>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  if constexpr (LGH + 3 <= LGN) {
    if constexpr (!(SKIP_LAST && LGH + 3 == LGN)) {
      stage<T, true, INV, N, NT, 8, LGH>(s, tab);
      group_sync<NT>();
    }
    dit_from<T, INV, LGN, NT, LGH + 3, SKIP_LAST>(s, tab);
  } else if constexpr (LGN - LGH == 2 && !SKIP_LAST) {
    stage<T, true, INV, N, NT, 4, LGH>(s, tab);
    group_sync<NT>();
  } else if constexpr (LGN - LGH == 1 && !SKIP_LAST) {
    stage<T, true, INV, N, NT, 2, LGH>(s, tab);
    group_sync<NT>();
  }
}

template <typename T, bool INV, int LGN, int NT, int LGH>
__device__ __forceinline__ void dif_down(cx<T>* s, const cx<T>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  if constexpr (LGH >= 0) {
    stage<T, false, INV, N, NT, 8, LGH>(s, tab);
    group_sync<NT>();
    dif_down<T, INV, LGN, NT, LGH - 3>(s, tab);
  }
}

// Full transforms on an LDS array addressed through swz<T>().  Callers
// synchronise before (input written by other threads) and index the array
// through swz<T>() too; the transforms end with a barrier.
template <typename T, bool INV, int LGN, int NT>
__device__ __forceinline__ void fft_dit(cx<T>* s, const cx<T>* __restrict__ tab) {
  dit_from<T, INV, LGN, NT, 0, false>(s, tab);
}

template <typename T, bool INV, int LGN, int NT>
__device__ __forceinline__ void fft_dif(cx<T>* s, const cx<T>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  using P = Plan8<LGN>;
  if constexpr (P::RLAST != 8) {
    stage<T, false, INV, N, NT, P::RLAST, P::LGLAST>(s, tab);
    group_sync<NT>();
  }
  dif_down<T, INV, LGN, NT, P::RLAST == 8 ? P::LGLAST : P::LGLAST - 3>(s, tab);
}

// The outermost stage of a transform (the last stage of fft_dit, the first of
// fft_dif) has radix R = RLAST and span H = N / R: its groups are q < H with
// points q + k H.  When H is a multiple of NT, thread tid owns the groups
// q = tid + c NT (c < H / NT), whose points are exactly tid + e NT with
// e = c + k (H / NT): the stage can leave its outputs in (or take its inputs
// from) the per-thread array v[e] <-> point tid + e NT, the layout of the
// pointwise step between an inverse and a forward transform, which then
// costs no LDS round trip.
template <int LGN, int NT>
struct Outer {
  using P = Plan8<LGN>;
  static constexpr int R = P::RLAST;
  static constexpr int LGH = P::LGLAST;
  static constexpr int H = 1 << LGH;
  static constexpr bool REGS = H % NT == 0;
  static constexpr int C = REGS ? H / NT : 1;
};
// fft_dit with the result in registers: v[e] = value at point tid + e NT.
// Ends without a barrier; the caller may then overwrite exactly these points
// of s (fft_dif_in does) without one.
template <typename T, bool INV, int LGN, int NT>
__device__ __forceinline__ void fft_dit_out(cx<T>* s, const cx<T>* __restrict__ tab,
                                            cx<T> (&v)[(1 << LGN) / NT]) {
  using O = Outer<LGN, NT>;
  const int tid = opaque_tid<NT>();
  if constexpr (O::REGS) {
    dit_from<T, INV, LGN, NT, 0, true>(s, tab);
#pragma unroll
    for (int c = 0; c < O::C; ++c) {
      const int q = tid + c * NT;
      cx<T> a[O::R];
#pragma unroll
      for (int k = 0; k < O::R; ++k) a[k] = s[swz<T>(q + k * O::H)];
      const Tw<T, O::R, O::LGH> tw(tab, q);
      bfly<T, true, INV, O::R, O::LGH>(a, tw);
#pragma unroll
      for (int k = 0; k < O::R; ++k) v[c + k * O::C] = a[k];
    }
  } else {
    fft_dit<T, INV, LGN, NT>(s, tab);
#pragma unroll
    for (int e = 0; e < (1 << LGN) / NT; ++e) v[e] = s[swz<T>(tid + e * NT)];
  }
}
// fft_dif with the input in registers (v[e] at point tid + e NT); no other
// thread may still read these points of s.  Ends with a barrier like fft_dif.
template <typename T, bool INV, int LGN, int NT>
__device__ __forceinline__ void fft_dif_in(cx<T>* s, const cx<T>* __restrict__ tab,
                                           const cx<T> (&v)[(1 << LGN) / NT]) {
  using O = Outer<LGN, NT>;
  const int tid = opaque_tid<NT>();
  if constexpr (O::REGS) {
#pragma unroll
    for (int c = 0; c < O::C; ++c) {
      const int q = tid + c * NT;
      cx<T> a[O::R];
#pragma unroll
      for (int k = 0; k < O::R; ++k) a[k] = v[c + k * O::C];
      const Tw<T, O::R, O::LGH> tw(tab, q);
      bfly<T, false, INV, O::R, O::LGH>(a, tw);
#pragma unroll
      for (int k = 0; k < O::R; ++k) s[swz<T>(q + k * O::H)] = a[k];
    }
    group_sync<NT>();
    dif_down<T, INV, LGN, NT, O::LGH - 3>(s, tab);
  } else {
#pragma unroll
    for (int e = 0; e < (1 << LGN) / NT; ++e) s[swz<T>(tid + e * NT)] = v[e];
    group_sync<NT>();
    fft_dif<T, INV, LGN, NT>(s, tab);
  }
}

// Forward real-FFT post-step for the bin pair (k, N-k): from Z[k], Z[N-k]
// (complex DFT_N of the packed sequence) give X[k], X[N-k] of the real DFT_B.
// w = exp(-2 pi i k / B).  For k = 0 pass zk == znk (Z[N] = Z[0]) and read
// X[0] = Xk, X[N] = Xnk (both real).
template <typename T>
__device__ __forceinline__ void rfft_post(cx<T> zk, cx<T> znk, cx<T> w, cx<T>& Xk, cx<T>& Xnk) {
  const cx<T> E = {T(0.5) * (zk.x + znk.x), T(0.5) * (zk.y - znk.y)};
  const cx<T> D = {T(0.5) * (zk.x - znk.x), T(0.5) * (zk.y + znk.y)};
  const cx<T> O = {D.y, -D.x};
  const cx<T> wO = cmul(w, O);
  Xk = cadd(E, wO);
  Xnk = cconj(csub(E, wO));
}

// Inverse real-FFT pre-step for the bin pair (k, N-k): from X[k], X[N-k] give
// Z[k], Z[N-k] such that the unscaled inverse DFT_N of Z equals
// B * (x[2t] + i x[2t+1]).  w = exp(-2 pi i k / B).
template <typename T>
__device__ __forceinline__ void irfft_pre(cx<T> Xk, cx<T> Xnk, cx<T> w, cx<T>& Zk, cx<T>& Znk) {
  const cx<T> E = {Xk.x + Xnk.x, Xk.y - Xnk.y};
  const cx<T> D = {Xk.x - Xnk.x, Xk.y + Xnk.y};
  const cx<T> O = cmulconj(w, D);  // conj(w) * D
  Zk = {E.x - O.y, E.y + O.x};     // E + i O
  Znk = {E.x + O.y, -E.y + O.x};   // conj(E) + i conj(O)
}

}  // namespace tls
