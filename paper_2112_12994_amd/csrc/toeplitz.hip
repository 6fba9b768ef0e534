// Launch wrappers for the blocked Toeplitz kernels (see toeplitz_impl.h).
#include "toeplitz_impl.h"

namespace tls {

namespace {

constexpr int nt_for(int lgn) {
  return ((1 << lgn) / 8) < 64 ? 64 : (((1 << lgn) / 8) > 256 ? 256 : (1 << lgn) / 8);
}

constexpr int LGN_MIN = 6;   // B = 128
constexpr int LGN_MAX = 13;  // B = 16384

template <typename T>
const cx<T>* tab_of(const Twiddles& tw);
template <>
const cx<double>* tab_of<double>(const Twiddles& tw) {
  return static_cast<const cx<double>*>(tw.d64);
}
template <>
const cx<float>* tab_of<float>(const Twiddles& tw) {
  return static_cast<const cx<float>*>(tw.d32);
}

template <typename T, int LGN, int MODE>
hipError_t toep_one(const void* Yhat, const void* Vhat, const void* w_in, void* u_out,
                    const void* u_in, double* partial, const double* coef, const int* flag,
                    const Twiddles& tw, int64_t m, int p, int L, int nblocks, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  hipLaunchKernelGGL((toep_pass_kernel<T, LGN, NT, MODE>), dim3(nblocks), dim3(NT), 0, st,
                     static_cast<const cx<T>*>(Yhat), static_cast<const cx<T>*>(Vhat),
                     static_cast<const T*>(w_in), static_cast<T*>(u_out),
                     static_cast<const T*>(u_in), partial, coef, flag, tab_of<T>(tw), m, p, L,
                     nblocks);
  return hipGetLastError();
}

template <typename T, int LGN>
hipError_t toep_modes(int mode, const void* Yhat, const void* Vhat, const void* w_in, void* u_out,
                      const void* u_in, double* partial, const double* coef, const int* flag,
                      const Twiddles& tw, int64_t m, int p, int L, int nblocks, hipStream_t st) {
#define TLS_MODE_CASE(MD)                                                                       \
  case MD:                                                                                      \
    return toep_one<T, LGN, MD>(Yhat, Vhat, w_in, u_out, u_in, partial, coef, flag, tw, m, p, \
                                L, nblocks, st);
  switch (mode) {
    TLS_MODE_CASE(MODE_FUSED)
    TLS_MODE_CASE(MODE_MV)
    TLS_MODE_CASE(MODE_RMV)
    default:
      return hipErrorInvalidValue;
  }
#undef TLS_MODE_CASE
}

template <typename T>
hipError_t toep_dispatch(int lgn, int mode, const void* Yhat, const void* Vhat, const void* w_in,
                         void* u_out, const void* u_in, double* partial, const double* coef,
                         const int* flag, const Twiddles& tw, int64_t m, int p, int L, int nblocks,
                         hipStream_t st) {
#define TLS_LGN_CASE(LG)                                                                       \
  case LG:                                                                                     \
    return toep_modes<T, LG>(mode, Yhat, Vhat, w_in, u_out, u_in, partial, coef, flag, tw, m, \
                             p, L, nblocks, st);
  switch (lgn) {
    TLS_LGN_CASE(6)
    TLS_LGN_CASE(7)
    TLS_LGN_CASE(8)
    TLS_LGN_CASE(9)
    TLS_LGN_CASE(10)
    TLS_LGN_CASE(11)
    TLS_LGN_CASE(12)
    TLS_LGN_CASE(13)
    default:
      return hipErrorInvalidValue;
  }
#undef TLS_LGN_CASE
}

template <int LGN, typename TS>
hipError_t spectra_one(const double* y, int64_t n, int L, int nblocks, void* Yhat,
                       const Twiddles& tw, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  hipLaunchKernelGGL((spectra_kernel<LGN, NT, TS>), dim3(nblocks), dim3(NT), 0, st, y, n, L,
                     static_cast<cx<TS>*>(Yhat), static_cast<const cx<double>*>(tw.d64));
  return hipGetLastError();
}

template <int LGN, typename TS>
hipError_t small_rfft_one(const double* cols, int len, int ld, int ncols, double scale, void* out,
                          const Twiddles& tw, const int* flag, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  hipLaunchKernelGGL((small_rfft_kernel<LGN, NT, TS>), dim3(ncols), dim3(NT), 0, st, cols, len, ld,
                     scale, static_cast<cx<TS>*>(out), static_cast<const cx<double>*>(tw.d64),
                     flag);
  return hipGetLastError();
}

template <typename T, int LGN>
hipError_t scores_one(const void* Yhat, const void* Om, int k, void* scores, const Twiddles& tw,
                      int64_t m, int p, int L, int nblocks, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  hipLaunchKernelGGL((scores_kernel<T, LGN, NT>), dim3(nblocks), dim3(NT), 0, st,
                     static_cast<const cx<T>*>(Yhat), static_cast<const cx<T>*>(Om), k,
                     static_cast<T*>(scores), tab_of<T>(tw), m, p, L);
  return hipGetLastError();
}

template <int NT>
__global__ __launch_bounds__(NT) void colsum_kernel(const double* __restrict__ partial,
                                                    int nblocks, double* __restrict__ out,
                                                    const int* __restrict__ flag) {
  __shared__ double red[NT / 64];
  if (flag && *flag) return;
  const double* col = partial + static_cast<size_t>(blockIdx.x) * nblocks;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += NT) s += col[b];
  const double tot = block_sum<NT>(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// Direct FP64 residual r_i = b_i - sum_j phi_j X[i, j] = y[p+i] - sum_j phi_j y[p-1+i-j],
// summed over j in order, row by row (the error of each row is bounded by
// the row's own terms rather than by whole-window norms as in the FFT
// products).  Each workgroup stages its rows' samples and phi in LDS and
// writes one partial of ||r||^2.
template <int NT, int RPT>
__global__ __launch_bounds__(NT) void resid_direct_kernel(const double* __restrict__ y, int64_t m,
                                                          int p, const double* __restrict__ phi,
                                                          double* __restrict__ partial) {
  extern __shared__ double sh[];
  double* sphi = sh;
  double* sy = sh + p;
  __shared__ double red[NT / 64];
  constexpr int TILE = NT * RPT;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * TILE;
  for (int j = threadIdx.x; j < p; j += NT) sphi[j] = phi[j];
  // samples y[row0 .. row0 + TILE + p) (rows use y[i .. i + p])
  for (int t = threadIdx.x; t < TILE + p; t += NT) {
    const int64_t g = row0 + t;
    sy[t] = g < m + p ? y[g] : 0.0;
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int t = threadIdx.x + k * NT;
    if (row0 + t < m) {
      double r = sy[t + p];
      for (int j = 0; j < p; ++j) r -= sphi[j] * sy[t + p - 1 - j];
      acc += r * r;
    }
  }
  const double tot = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

}  // namespace

int resid_direct_blocks(int64_t m) { return static_cast<int>((m + 1023) / 1024); }

hipError_t launch_resid_direct(const double* y, int64_t m, int p, const double* phi,
                               double* partial, hipStream_t st) {
  const int nb = resid_direct_blocks(m);
  const size_t shm = (static_cast<size_t>(p) + 1024 + p) * sizeof(double);
  hipLaunchKernelGGL((resid_direct_kernel<256, 4>), dim3(nb), dim3(256), shm, st, y, m, p, phi,
                     partial);
  return hipGetLastError();
}

hipError_t launch_toep(int prec, int lgn, int mode, const void* Yhat, const void* Vhat,
                       const void* w_in, void* u_out, const void* u_in, double* partial,
                       const double* coef, const int* flag, const Twiddles& tw, int64_t m, int p,
                       int L, int nblocks, hipStream_t st) {
  if (lgn < LGN_MIN || lgn > LGN_MAX || nblocks < 1) return hipErrorInvalidValue;
  if (prec == PREC_F64)
    return toep_dispatch<double>(lgn, mode, Yhat, Vhat, w_in, u_out, u_in, partial, coef, flag,
                                 tw, m, p, L, nblocks, st);
  return toep_dispatch<float>(lgn, mode, Yhat, Vhat, w_in, u_out, u_in, partial, coef, flag, tw,
                              m, p, L, nblocks, st);
}

#define TLS_SIZE_SWITCH(FN, TARG, ARGS)     \
  switch (lgn) {                            \
    case 6: return FN<6, TARG> ARGS;        \
    case 7: return FN<7, TARG> ARGS;        \
    case 8: return FN<8, TARG> ARGS;        \
    case 9: return FN<9, TARG> ARGS;        \
    case 10: return FN<10, TARG> ARGS;      \
    case 11: return FN<11, TARG> ARGS;      \
    case 12: return FN<12, TARG> ARGS;      \
    case 13: return FN<13, TARG> ARGS;      \
    default: return hipErrorInvalidValue;   \
  }

hipError_t launch_spectra(int prec, int lgn, const double* y, int64_t n, int L, int nblocks,
                          void* Yhat, const Twiddles& tw, hipStream_t st) {
  if (nblocks < 1) return hipErrorInvalidValue;
  if (prec == PREC_F64) {
    TLS_SIZE_SWITCH(spectra_one, double, (y, n, L, nblocks, Yhat, tw, st))
  }
  TLS_SIZE_SWITCH(spectra_one, float, (y, n, L, nblocks, Yhat, tw, st))
}

hipError_t launch_small_rfft(int prec, int lgn, const double* cols, int len, int ld, int ncols,
                             double scale, void* out, const Twiddles& tw, const int* flag,
                             hipStream_t st) {
  if (ncols < 1 || len > (2 << lgn)) return hipErrorInvalidValue;
  if (prec == PREC_F64) {
    TLS_SIZE_SWITCH(small_rfft_one, double, (cols, len, ld, ncols, scale, out, tw, flag, st))
  }
  TLS_SIZE_SWITCH(small_rfft_one, float, (cols, len, ld, ncols, scale, out, tw, flag, st))
}

template <int LGN, typename T>
hipError_t scores_sw(const void* Yhat, const void* Om, int k, void* scores, const Twiddles& tw,
                     int64_t m, int p, int L, int nblocks, hipStream_t st) {
  return scores_one<T, LGN>(Yhat, Om, k, scores, tw, m, p, L, nblocks, st);
}

hipError_t launch_scores(int prec, int lgn, const void* Yhat, const void* Om, int k, void* scores,
                         const Twiddles& tw, int64_t m, int p, int L, int nblocks, hipStream_t st) {
  if (nblocks < 1 || k < 1) return hipErrorInvalidValue;
  if (prec == PREC_F64) {
    TLS_SIZE_SWITCH(scores_sw, double, (Yhat, Om, k, scores, tw, m, p, L, nblocks, st))
  }
  TLS_SIZE_SWITCH(scores_sw, float, (Yhat, Om, k, scores, tw, m, p, L, nblocks, st))
}

hipError_t launch_colsum(const double* partial, int nblocks, int ncols, double* out,
                         const int* flag, hipStream_t st) {
  if (ncols < 1 || nblocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((colsum_kernel<256>), dim3(ncols), dim3(256), 0, st, partial, nblocks, out,
                     flag);
  return hipGetLastError();
}

}  // namespace tls
