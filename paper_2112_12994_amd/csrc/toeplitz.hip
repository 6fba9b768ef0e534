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
  constexpr int NT = pass_nt(LGN);
  constexpr int NW = pass_nw(LGN);
  const int ngroups = pass_groups(LGN, nblocks);
  hipLaunchKernelGGL((toep_pass_kernel<T, LGN, NT, NW, MODE>), dim3(ngroups), dim3(NT * NW), 0, st,
                     static_cast<const cx<T>*>(Yhat), static_cast<const cx<T>*>(Vhat),
                     static_cast<const T*>(w_in), static_cast<T*>(u_out),
                     static_cast<const T*>(u_in), partial, coef, flag, tab_of<T>(tw), m, p, L,
                     nblocks, ngroups);
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
__device__ __forceinline__ void colsum_body(const double* __restrict__ partial,
                                                    int nblocks, double* __restrict__ out,
                                                    const int* __restrict__ flag, int j) {
  __shared__ double red[4];
  if (flag && *flag) return;
  const double tot = column_sum<NT>(partial + static_cast<size_t>(j) * nblocks, nblocks, red);
  if (threadIdx.x == 0) out[j] = tot;
}

template <int NT>
__global__ __launch_bounds__(NT) void colsum_kernel(const double* __restrict__ partial,
                                                    int nblocks, double* __restrict__ out,
                                                    const int* __restrict__ flag) {
  colsum_body<NT>(partial, nblocks, out, flag, blockIdx.x);
}

// Direct FP64 residual r_i = b_i - sum_j phi_j X[i, j] = y[p+i] - sum_j phi_j y[p-1+i-j],
// summed over j in order, row by row (the error of each row is bounded by
// the row's own terms rather than by whole-window norms as in the FFT
// products).  Each workgroup stages its rows' samples in LDS (one pad word
// per R samples, so that lanes R samples apart hit different banks) and
// writes one partial of ||r||^2.  Thread k owns R consecutive rows: at lag
// j they need samples t .. t + R - 1, t = kR + p - 1 - j, so one new sample
// per lag enters a register ring and every lag costs one LDS read for R
// FMAs; phi_j is a uniform (scalar) load.
constexpr int RESID_R = 8;

__host__ __device__ __forceinline__ int resid_skew(int t) { return t + t / RESID_R; }

template <int NT>
__device__ __forceinline__ void resid_direct_body(const double* __restrict__ y, int64_t m,
                                                  int p, const double* __restrict__ phi,
                                                  double* __restrict__ partial, int tile) {
  constexpr int R = RESID_R;
  extern __shared__ double sy[];
  __shared__ double red[NT / 64];
  constexpr int TILE = NT * R;
  const int64_t row0 = static_cast<int64_t>(tile) * TILE;
  // samples y[row0 .. row0 + TILE + p) (row i uses y[i .. i + p]), up to 16
  // loads per thread in flight before any is stored
  for (int t0 = threadIdx.x; t0 < TILE + p; t0 += 16 * NT) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int t = t0 + k * NT;
      const int64_t g = row0 + t;
      v[k] = (t < TILE + p && g < m + p) ? y[g] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int t = t0 + k * NT;
      if (t < TILE + p) sy[resid_skew(t)] = v[k];
    }
  }
  __syncthreads();
  const int w = threadIdx.x * R + p - 1;  // sample of row 0 at lag 0
  double acc[R], ring[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    acc[r] = sy[resid_skew(w + 1 + r)];  // b of row r
    ring[r] = sy[resid_skew(w + r)];     // lag 0 sample of row r, in slot r
  }
  // at lag j the sample of row r sits in slot (r - j) mod R
  for (int jb = 0; jb < p; jb += R) {
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
      const int j = jb + jj;
      if (j < p) {
        const double f = phi[j];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] -= f * ring[(r - jj + R) % R];
        // the sample entering at lag j + 1 (row 0) replaces row R-1's
        const int tn = w - j - 1;
        ring[(R - 1 - jj + R) % R] = tn >= 0 ? sy[resid_skew(tn)] : 0.0;
      }
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (row0 + threadIdx.x * R + r < m) ss += acc[r] * acc[r];
  const double tot = block_sum<NT>(ss, red);
  if (threadIdx.x == 0) partial[tile] = tot;
}

template <int NT>
__global__ __launch_bounds__(NT) void resid_direct_kernel(const double* __restrict__ y, int64_t m,
                                                          int p, const double* __restrict__ phi,
                                                          double* __restrict__ partial) {
  resid_direct_body<NT>(y, m, p, phi, partial, blockIdx.x);
}

}  // namespace

constexpr int RESID_NT = 256;
constexpr int RESID_TILE = RESID_NT * RESID_R;

int resid_direct_blocks(int64_t m) {
  return static_cast<int>((m + RESID_TILE - 1) / RESID_TILE);
}

// LDS of one residual workgroup: the skewed samples of its rows
size_t resid_lds_bytes(int p) {
  return static_cast<size_t>(resid_skew(RESID_TILE + p) + 1) * sizeof(double);
}

hipError_t launch_resid_direct(const double* y, int64_t m, int p, const double* phi,
                               double* partial, hipStream_t st) {
  const int nb = resid_direct_blocks(m);
  hipLaunchKernelGGL((resid_direct_kernel<RESID_NT>), dim3(nb), dim3(RESID_NT), resid_lds_bytes(p),
                     st, y, m, p, phi, partial);
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

// ---- batched launches: one workgroup per work item {fit, local index} -------
namespace tls {
namespace {

template <int LGN, int NT, typename TS>
__global__ __launch_bounds__(NT) void spectra_b_kernel(const Item* __restrict__ items,
                                                       const FitDesc* __restrict__ D, int to64,
                                                       const cx<double>* __restrict__ tab) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  spectra_body<LGN, NT, TS>(d.y, d.n, d.L, static_cast<cx<TS>*>(to64 ? d.Yhat64 : d.Yhat), tab,
                            it.idx);
}

// A pointer the compiler cannot see through: the batched passes hand the
// pass body their vectors this way, so that it compiles to the same code as
// in the single-fit kernel (which gets them as plain arguments) and gives
// bit-identical results.
template <typename P>
__device__ __forceinline__ P opaque_ptr(P x) {
  asm volatile("" : "+s"(x));
  return x;
}

template <typename T, int LGN, int NT, int VARIANT>
__global__ __launch_bounds__(NT * pass_nw(LGN)) void toep_b_kernel(const Item* __restrict__ items,
                                                    const FitDesc* __restrict__ D,
                                                    const double* __restrict__ consts,
                                                    const cx<T>* __restrict__ tab) {
  constexpr int NW = pass_nw(LGN);
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  // the LSQR passes run for the fits whose products have their precision
  if constexpr (VARIANT == BP_LSQR_FIRST || VARIANT == BP_LSQR) {
    if (d.st->f32) return;
  } else if constexpr (VARIANT == BP_LSQR32) {
    if (!d.st->f32) return;
  }
  if constexpr (VARIANT == BP_LSQR_FIRST || VARIANT == BP_LSQR) {
    const T* w = VARIANT == BP_LSQR_FIRST ? reinterpret_cast<const T*>(d.y + d.p)
                                          : static_cast<const T*>(d.u);
    toep_pass_body<T, LGN, NT, NW, MODE_FUSED, false>(static_cast<const cx<T>*>(d.Yhat64),
                                           static_cast<const cx<T>*>(d.Vhat), opaque_ptr(w),
                                           opaque_ptr(static_cast<T*>(d.u)),
                                           opaque_ptr(static_cast<const T*>(nullptr)), d.partial,
                                           d.st->coef, &d.st->done, tab, d.m, d.p, d.L,
                                           d.nblocks, d.ngroups, it.idx);
  } else if constexpr (VARIANT == BP_LSQR32) {
    toep_pass_body<T, LGN, NT, NW, MODE_FUSED, false>(
        static_cast<const cx<T>*>(d.Yhat), static_cast<const cx<T>*>(d.Vhat),
        opaque_ptr(static_cast<const T*>(d.u)), opaque_ptr(static_cast<T*>(d.u)),
        opaque_ptr(static_cast<const T*>(nullptr)), d.partial, d.st->coef, &d.st->done, tab, d.m,
        d.p, d.L, d.nblocks, d.ngroups, it.idx);
  } else if constexpr (VARIANT == BP_OUTER64) {
    toep_pass_body<T, LGN, NT, NW, MODE_FUSED, false>(
        static_cast<const cx<T>*>(d.Yhat64), static_cast<const cx<T>*>(d.Vhat),
        opaque_ptr(reinterpret_cast<const T*>(d.y + d.p)), opaque_ptr(static_cast<T*>(nullptr)),
        opaque_ptr(static_cast<const T*>(nullptr)), d.partial, consts, &d.rst->done, tab, d.m,
        d.p, d.L, d.nblocks, d.ngroups, it.idx);
  } else {
    toep_pass_body<T, LGN, NT, NW, MODE_FUSED, false>(
        static_cast<const cx<T>*>(d.Yhat), static_cast<const cx<T>*>(d.Vhat32),
        opaque_ptr(static_cast<const T*>(nullptr)), opaque_ptr(static_cast<T*>(nullptr)),
        opaque_ptr(static_cast<const T*>(nullptr)), d.partial, consts + 2, &d.rst->inner_done,
        tab, d.m, d.p, d.L, d.nblocks, d.ngroups, it.idx);
  }
}

template <int LGN, int NT, typename TS>
__global__ __launch_bounds__(NT) void small_rfft_b_kernel(const Item* __restrict__ items,
                                                          const FitDesc* __restrict__ D,
                                                          int variant,
                                                          const cx<double>* __restrict__ tab) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  const double scale = 1.0 / static_cast<double>(2 << LGN);
  // variant 1 (v's spectrum for LSQR) in the precision of the fit's products
  if (variant == 1 && (sizeof(TS) == 4) != (d.st->f32 != 0)) return;
  if (variant == 0)
    small_rfft_body<LGN, NT, TS>(d.Om, d.p, d.p, scale, static_cast<cx<TS>*>(d.Omhat), tab,
                                 nullptr, it.idx);
  else
    small_rfft_body<LGN, NT, TS>(variant == 1 ? d.phi0 : d.phi, d.p, d.p, scale,
                                 static_cast<cx<TS>*>(d.Vhat), tab, nullptr, 0);
}

template <typename T, int LGN, int NT>
__global__ __launch_bounds__(NT) void scores_b_kernel(const Item* __restrict__ items,
                                                      const FitDesc* __restrict__ D,
                                                      const cx<T>* __restrict__ tab) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  // FP64 scores from the FP64 spectra (Yhat64 is Yhat unless mixed)
  scores_body<T, LGN, NT>(static_cast<const cx<T>*>(sizeof(T) == 8 ? d.Yhat64 : d.Yhat),
                          static_cast<const cx<T>*>(d.Omhat),
                          d.k, static_cast<T*>(d.u), tab, d.m, d.p, d.L, it.idx);
}

template <int NT>
__global__ __launch_bounds__(NT) void colsum_b_kernel(const Item* __restrict__ items,
                                                      const FitDesc* __restrict__ D, int variant) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  if (variant == 3) {
    colsum_body<NT>(d.rpart, static_cast<int>((d.m + RESID_TILE - 1) / RESID_TILE), d.rr, nullptr,
                    it.idx);
    return;
  }
  const int* flag = variant == 0 ? &d.st->done : (variant == 1 ? &d.rst->done : &d.rst->inner_done);
  colsum_body<NT>(d.partial, d.ngroups, d.g, flag, it.idx);
}

template <int NT>
__global__ __launch_bounds__(NT) void resid_b_kernel(const Item* __restrict__ items,
                                                     const FitDesc* __restrict__ D) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  resid_direct_body<NT>(d.y, d.m, d.p, d.phi, d.rpart, it.idx);
}

template <int LGN>
hipError_t toep_b_sel(int prec, int variant, const Item* items, int nitems, const FitDesc* D,
                      const double* consts, const Twiddles& tw, hipStream_t st) {
  constexpr int NT = pass_nt(LGN);
  switch (variant) {
    case BP_LSQR_FIRST:
      hipLaunchKernelGGL((toep_b_kernel<double, LGN, NT, BP_LSQR_FIRST>), dim3(nitems), dim3(NT * pass_nw(LGN)), 0,
                         st, items, D, consts, tab_of<double>(tw));
      break;
    case BP_LSQR:
      hipLaunchKernelGGL((toep_b_kernel<double, LGN, NT, BP_LSQR>), dim3(nitems), dim3(NT * pass_nw(LGN)), 0,
                         st, items, D, consts, tab_of<double>(tw));
      break;
    case BP_OUTER64:
      hipLaunchKernelGGL((toep_b_kernel<double, LGN, NT, BP_OUTER64>), dim3(nitems), dim3(NT * pass_nw(LGN)), 0,
                         st, items, D, consts, tab_of<double>(tw));
      break;
    case BP_LSQR32:
      hipLaunchKernelGGL((toep_b_kernel<float, LGN, NT, BP_LSQR32>), dim3(nitems),
                         dim3(NT * pass_nw(LGN)), 0, st, items, D, consts, tab_of<float>(tw));
      break;
    case BP_INNER32:
      hipLaunchKernelGGL((toep_b_kernel<float, LGN, NT, BP_INNER32>), dim3(nitems), dim3(NT * pass_nw(LGN)), 0,
                         st, items, D, consts, tab_of<float>(tw));
      break;
    default:
      return hipErrorInvalidValue;
  }
  (void)prec;
  return hipGetLastError();
}

template <int LGN>
hipError_t spectra_b_sel(int prec, const Item* items, int nitems, const FitDesc* D, int to64,
                         const Twiddles& tw, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  if (prec == PREC_F64 || to64)
    hipLaunchKernelGGL((spectra_b_kernel<LGN, NT, double>), dim3(nitems), dim3(NT), 0, st, items, D,
                       to64, static_cast<const cx<double>*>(tw.d64));
  else
    hipLaunchKernelGGL((spectra_b_kernel<LGN, NT, float>), dim3(nitems), dim3(NT), 0, st, items, D,
                       to64, static_cast<const cx<double>*>(tw.d64));
  return hipGetLastError();
}

template <int LGN>
hipError_t small_rfft_b_sel(int prec, int variant, const Item* items, int nitems, const FitDesc* D,
                            const Twiddles& tw, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  if (prec == PREC_F64 || variant == 2)
    hipLaunchKernelGGL((small_rfft_b_kernel<LGN, NT, double>), dim3(nitems), dim3(NT), 0, st, items,
                       D, variant, static_cast<const cx<double>*>(tw.d64));
  else
    hipLaunchKernelGGL((small_rfft_b_kernel<LGN, NT, float>), dim3(nitems), dim3(NT), 0, st, items,
                       D, variant, static_cast<const cx<double>*>(tw.d64));
  return hipGetLastError();
}

template <int LGN>
hipError_t scores_b_sel(int prec, const Item* items, int nitems, const FitDesc* D,
                        const Twiddles& tw, hipStream_t st) {
  constexpr int NT = nt_for(LGN);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((scores_b_kernel<double, LGN, NT>), dim3(nitems), dim3(NT), 0, st, items, D,
                       tab_of<double>(tw));
  else
    hipLaunchKernelGGL((scores_b_kernel<float, LGN, NT>), dim3(nitems), dim3(NT), 0, st, items, D,
                       tab_of<float>(tw));
  return hipGetLastError();
}

}  // namespace

#define TLS_B_SWITCH(CALL)                    \
  switch (lgn) {                              \
    case 6: return CALL(6);                   \
    case 7: return CALL(7);                   \
    case 8: return CALL(8);                   \
    case 9: return CALL(9);                   \
    case 10: return CALL(10);                 \
    case 11: return CALL(11);                 \
    case 12: return CALL(12);                 \
    case 13: return CALL(13);                 \
    default: return hipErrorInvalidValue;     \
  }

hipError_t launch_spectra_b(int prec, int lgn, const Item* items, int nitems, const FitDesc* D,
                            int to64, const Twiddles& tw, hipStream_t st) {
  if (nitems < 1) return hipSuccess;
#define TLS_C(LG) spectra_b_sel<LG>(prec, items, nitems, D, to64, tw, st)
  TLS_B_SWITCH(TLS_C)
#undef TLS_C
}

hipError_t launch_toep_b(int prec, int lgn, int variant, const Item* items, int nitems,
                         const FitDesc* D, const double* consts, const Twiddles& tw,
                         hipStream_t st) {
  if (nitems < 1) return hipSuccess;
#define TLS_C(LG) toep_b_sel<LG>(prec, variant, items, nitems, D, consts, tw, st)
  TLS_B_SWITCH(TLS_C)
#undef TLS_C
}

hipError_t launch_small_rfft_b(int prec, int lgn, int variant, const Item* items, int nitems,
                               const FitDesc* D, const Twiddles& tw, hipStream_t st) {
  if (nitems < 1) return hipSuccess;
#define TLS_C(LG) small_rfft_b_sel<LG>(prec, variant, items, nitems, D, tw, st)
  TLS_B_SWITCH(TLS_C)
#undef TLS_C
}

hipError_t launch_scores_b(int prec, int lgn, const Item* items, int nitems, const FitDesc* D,
                           const Twiddles& tw, hipStream_t st) {
  if (nitems < 1) return hipSuccess;
#define TLS_C(LG) scores_b_sel<LG>(prec, items, nitems, D, tw, st)
  TLS_B_SWITCH(TLS_C)
#undef TLS_C
}

hipError_t launch_colsum_b(int variant, const Item* items, int nitems, const FitDesc* D,
                           hipStream_t st) {
  if (nitems < 1) return hipSuccess;
  hipLaunchKernelGGL((colsum_b_kernel<256>), dim3(nitems), dim3(256), 0, st, items, D, variant);
  return hipGetLastError();
}

hipError_t launch_resid_b(const Item* items, int nitems, const FitDesc* D, int pmax,
                          hipStream_t st) {
  if (nitems < 1) return hipSuccess;
  hipLaunchKernelGGL((resid_b_kernel<RESID_NT>), dim3(nitems), dim3(RESID_NT),
                     resid_lds_bytes(pmax), st, items, D);
  return hipGetLastError();
}

}  // namespace tls
