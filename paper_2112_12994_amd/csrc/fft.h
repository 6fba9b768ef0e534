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
// Twiddles come from one table tab[k] = exp(-2 pi i k / BMAX), k < BMAX/2,
// built once on the host in extended precision; w_L^e = tab[e * BMAX / L].
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

template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tab, int e, int lgL) {
  cx<T> w = tab[e << (LG_BMAX - lgL)];
  if (INV) w.y = -w.y;
  return w;
}

// ---- decimation-in-time passes (levels of span h, 2h, 4h) -----------------
template <typename T, bool INV, int N, int NT>
__device__ __forceinline__ void dit_pass3(cx<T>* s, const cx<T>* __restrict__ tab, int lgh) {
  const int h = 1 << lgh;
  for (int q = threadIdx.x; q < N / 8; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> lgh) << (lgh + 3)) + r;
    cx<T> a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = s[swz<T>(base + k * h)];
    const cx<T> w1 = twiddle<T, INV>(tab, r, lgh + 1);
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      const cx<T> b = cmul(a[k + 1], w1);
      a[k + 1] = csub(a[k], b);
      a[k] = cadd(a[k], b);
    }
    const cx<T> w2 = twiddle<T, INV>(tab, r, lgh + 2);
    const cx<T> w2b = rot90<T, INV>(w2);
#pragma unroll
    for (int k0 = 0; k0 < 8; k0 += 4) {
      cx<T> b = cmul(a[k0 + 2], w2);
      a[k0 + 2] = csub(a[k0], b);
      a[k0] = cadd(a[k0], b);
      b = cmul(a[k0 + 3], w2b);
      a[k0 + 3] = csub(a[k0 + 1], b);
      a[k0 + 1] = cadd(a[k0 + 1], b);
    }
    cx<T> w3[4];
    w3[0] = twiddle<T, INV>(tab, r, lgh + 3);
    w3[1] = twiddle<T, INV>(tab, r + h, lgh + 3);
    w3[2] = rot90<T, INV>(w3[0]);
    w3[3] = rot90<T, INV>(w3[1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const cx<T> b = cmul(a[k + 4], w3[k]);
      a[k + 4] = csub(a[k], b);
      a[k] = cadd(a[k], b);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) s[swz<T>(base + k * h)] = a[k];
  }
}

template <typename T, bool INV, int N, int NT>
__device__ __forceinline__ void dit_pass2(cx<T>* s, const cx<T>* __restrict__ tab, int lgh) {
  const int h = 1 << lgh;
  for (int q = threadIdx.x; q < N / 4; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> lgh) << (lgh + 2)) + r;
    cx<T> a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = s[swz<T>(base + k * h)];
    const cx<T> w1 = twiddle<T, INV>(tab, r, lgh + 1);
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
      const cx<T> b = cmul(a[k + 1], w1);
      a[k + 1] = csub(a[k], b);
      a[k] = cadd(a[k], b);
    }
    const cx<T> w2 = twiddle<T, INV>(tab, r, lgh + 2);
    const cx<T> w2b = rot90<T, INV>(w2);
    cx<T> b = cmul(a[2], w2);
    a[2] = csub(a[0], b);
    a[0] = cadd(a[0], b);
    b = cmul(a[3], w2b);
    a[3] = csub(a[1], b);
    a[1] = cadd(a[1], b);
#pragma unroll
    for (int k = 0; k < 4; ++k) s[swz<T>(base + k * h)] = a[k];
  }
}

template <typename T, bool INV, int N, int NT>
__device__ __forceinline__ void dit_pass1(cx<T>* s, const cx<T>* __restrict__ tab, int lgh) {
  const int h = 1 << lgh;
  for (int q = threadIdx.x; q < N / 2; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> lgh) << (lgh + 1)) + r;
    const cx<T> a0 = s[swz<T>(base)];
    const cx<T> b = cmul(s[swz<T>(base + h)], twiddle<T, INV>(tab, r, lgh + 1));
    s[swz<T>(base)] = cadd(a0, b);
    s[swz<T>(base + h)] = csub(a0, b);
  }
}

// ---- decimation-in-frequency passes (levels of span 4h, 2h, h) -----------
template <typename T, bool INV, int N, int NT>
__device__ __forceinline__ void dif_pass3(cx<T>* s, const cx<T>* __restrict__ tab, int lgh) {
  const int h = 1 << lgh;
  for (int q = threadIdx.x; q < N / 8; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> lgh) << (lgh + 3)) + r;
    cx<T> a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = s[swz<T>(base + k * h)];
    cx<T> w3[4];
    w3[0] = twiddle<T, INV>(tab, r, lgh + 3);
    w3[1] = twiddle<T, INV>(tab, r + h, lgh + 3);
    w3[2] = rot90<T, INV>(w3[0]);
    w3[3] = rot90<T, INV>(w3[1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const cx<T> t = csub(a[k], a[k + 4]);
      a[k] = cadd(a[k], a[k + 4]);
      a[k + 4] = cmul(t, w3[k]);
    }
    const cx<T> w2 = twiddle<T, INV>(tab, r, lgh + 2);
    const cx<T> w2b = rot90<T, INV>(w2);
#pragma unroll
    for (int k0 = 0; k0 < 8; k0 += 4) {
      cx<T> t = csub(a[k0], a[k0 + 2]);
      a[k0] = cadd(a[k0], a[k0 + 2]);
      a[k0 + 2] = cmul(t, w2);
      t = csub(a[k0 + 1], a[k0 + 3]);
      a[k0 + 1] = cadd(a[k0 + 1], a[k0 + 3]);
      a[k0 + 3] = cmul(t, w2b);
    }
    const cx<T> w1 = twiddle<T, INV>(tab, r, lgh + 1);
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      const cx<T> t = csub(a[k], a[k + 1]);
      a[k] = cadd(a[k], a[k + 1]);
      a[k + 1] = cmul(t, w1);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) s[swz<T>(base + k * h)] = a[k];
  }
}

template <typename T, bool INV, int N, int NT>
__device__ __forceinline__ void dif_pass2(cx<T>* s, const cx<T>* __restrict__ tab, int lgh) {
  const int h = 1 << lgh;
  for (int q = threadIdx.x; q < N / 4; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> lgh) << (lgh + 2)) + r;
    cx<T> a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = s[swz<T>(base + k * h)];
    const cx<T> w2 = twiddle<T, INV>(tab, r, lgh + 2);
    const cx<T> w2b = rot90<T, INV>(w2);
    cx<T> t = csub(a[0], a[2]);
    a[0] = cadd(a[0], a[2]);
    a[2] = cmul(t, w2);
    t = csub(a[1], a[3]);
    a[1] = cadd(a[1], a[3]);
    a[3] = cmul(t, w2b);
    const cx<T> w1 = twiddle<T, INV>(tab, r, lgh + 1);
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
      t = csub(a[k], a[k + 1]);
      a[k] = cadd(a[k], a[k + 1]);
      a[k + 1] = cmul(t, w1);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s[swz<T>(base + k * h)] = a[k];
  }
}

template <typename T, bool INV, int N, int NT>
__device__ __forceinline__ void dif_pass1(cx<T>* s, const cx<T>* __restrict__ tab, int lgh) {
  const int h = 1 << lgh;
  for (int q = threadIdx.x; q < N / 2; q += NT) {
    const int r = q & (h - 1);
    const int base = ((q >> lgh) << (lgh + 1)) + r;
    const cx<T> a0 = s[swz<T>(base)], a1 = s[swz<T>(base + h)];
    s[swz<T>(base)] = cadd(a0, a1);
    s[swz<T>(base + h)] = cmul(csub(a0, a1), twiddle<T, INV>(tab, r, lgh + 1));
  }
}

// Full transforms on an LDS array addressed through swz<T>().  Callers
// synchronise before (input written by other threads) and index the array
// through swz<T>() too; the transforms end with a barrier.
template <typename T, bool INV, int LGN, int NT>
__device__ __forceinline__ void fft_dit(cx<T>* s, const cx<T>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  int lgh = 0;
#pragma unroll
  for (int it = 0; it < LGN / 3; ++it, lgh += 3) {
    dit_pass3<T, INV, N, NT>(s, tab, lgh);
    __syncthreads();
  }
  if constexpr (LGN % 3 == 2) {
    dit_pass2<T, INV, N, NT>(s, tab, lgh);
    __syncthreads();
  } else if constexpr (LGN % 3 == 1) {
    dit_pass1<T, INV, N, NT>(s, tab, lgh);
    __syncthreads();
  }
}

template <typename T, bool INV, int LGN, int NT>
__device__ __forceinline__ void fft_dif(cx<T>* s, const cx<T>* __restrict__ tab) {
  constexpr int N = 1 << LGN;
  int lgh = LGN;
  if constexpr (LGN % 3 == 2) {
    lgh -= 2;
    dif_pass2<T, INV, N, NT>(s, tab, lgh);
    __syncthreads();
  } else if constexpr (LGN % 3 == 1) {
    lgh -= 1;
    dif_pass1<T, INV, N, NT>(s, tab, lgh);
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < LGN / 3; ++it) {
    lgh -= 3;
    dif_pass3<T, INV, N, NT>(s, tab, lgh);
    __syncthreads();
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
