// Host-side launch wrappers of the HIP kernels (one library, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tls {

enum Prec : int { PREC_F64 = 0, PREC_F32 = 1 };

// Compile-time modes of the blocked Toeplitz pass (the pass always forms the
// per-block partials of ||e||^2; w_in / u_out are used when non-NULL).
enum PassMode : int {
  PM_MV = 1,   // e = s1 X v + s2 w (needs the packed spectrum of v)
  PM_RMV = 2,  // apply X^T to e (or to u_in without PM_MV)
};
constexpr int MODE_FUSED = PM_MV | PM_RMV;  // LSQR step, residual + gradient, X^T X v
constexpr int MODE_MV = PM_MV;              // e = s1 Xv + s2 w, ||e||^2
constexpr int MODE_RMV = PM_RMV;            // X^T u, ||u||^2

struct Twiddles {
  const void* d64 = nullptr;  // cx<double>[NMAX]
  const void* d32 = nullptr;  // cx<float>[NMAX]
};

// threads per workgroup used for a transform of complex length 2^lgn
inline int fft_threads(int lgn) {
  int n8 = (1 << lgn) / 8;
  return n8 < 64 ? 64 : (n8 > 256 ? 256 : n8);
}

hipError_t launch_spectra(int prec, int lgn, const double* y, int64_t n, int L, int nblocks,
                          void* Yhat, const Twiddles& tw, hipStream_t st);
hipError_t launch_toep(int prec, int lgn, int mode, const void* Yhat, const void* Vhat,
                       const void* w_in, void* u_out, const void* u_in, double* partial,
                       const double* coef, const int* flag, const Twiddles& tw, int64_t m, int p,
                       int L, int nblocks, hipStream_t st);
hipError_t launch_small_rfft(int prec, int lgn, const double* cols, int len, int ld, int ncols,
                             double scale, void* out, const Twiddles& tw, const int* flag,
                             hipStream_t st);
hipError_t launch_scores(int prec, int lgn, const void* Yhat, const void* Om, int k, void* scores,
                         const Twiddles& tw, int64_t m, int p, int L, int nblocks, hipStream_t st);
// ||y[p:] - X phi||^2 partials, one per 1024 rows (direct FP64 sums).
int resid_direct_blocks(int64_t m);
hipError_t launch_resid_direct(const double* y, int64_t m, int p, const double* phi,
                               double* partial, hipStream_t st);
hipError_t launch_colsum(const double* partial, int nblocks, int ncols, double* out,
                         const int* flag, hipStream_t st);

// sketch
hipError_t launch_philox_uniform(double* out, int64_t count, uint32_t stream, uint32_t fit,
                                 uint64_t seed, uint64_t start, hipStream_t st);
hipError_t launch_gather(const double* y, int64_t m, int p, int mode, const int64_t* idx,
                         const double* scale, int c, int crows, int ldq, double* A, int64_t* idx_out,
                         double* scale_out, uint64_t seed, uint32_t fit, hipStream_t st);
hipError_t launch_sample(int prec, const void* scores, int64_t m, const double* u, int c,
                         int64_t* idx, double* scale, double* work, uint64_t seed, uint32_t fit,
                         hipStream_t st);
size_t sample_work_doubles(int64_t m);
hipError_t launch_jl_omega(const double* M, int p, int k, int kind, double* Pi, double* Om,
                           uint64_t seed, uint32_t fit, hipStream_t st);

// QR of the sketch and triangular helpers
// rank_cols: leading columns whose breakdown or tiny pivot means rank
// deficiency (the sketch [S X | S b] passes p: b may lie in the range of X).
// A: crows x ldq row-major, crows % 16 == 0.  G: qr_scratch_doubles() doubles.
size_t qr_scratch_doubles(int crows, int q, int ldq);
// sweeps: 3 = shifted Cholesky QR then two refining sweeps (R accurate to
// O(u) orthogonality); 1 = the shifted sweep alone (a rougher R, enough for
// approximate leverage scores).
hipError_t launch_qr(double* A, int crows, int q, int ldq, int rank_cols, int sweeps, double* R,
                     double* G, double* R1, double* R2, int* status, hipStream_t st);
hipError_t launch_triinv(const double* R, int q, int p, double* M, double* Mt, double* phi0,
                         int* status, hipStream_t st);

// LSQR p-side step and state
struct LsqrState {
  double alpha, beta, rhobar, phibar, anorm2, bnorm, rnorm, arnorm, znorm, tol;
  double coef[2];
  int iter, istop, done, max_iter, phase, pad_;
};
hipError_t launch_lsqr_step(int prec, int lgn, int p, LsqrState* st, const double* g,
                            const double* M, const double* Mt, double* v, double* w, double* z,
                            const double* phi0, double* phi, void* Vhat, const Twiddles& tw,
                            hipStream_t stream);
// Mixed-precision refinement (FP64 outer residual, FP32 inner CG on the
// preconditioned normal equations).
struct RefineState {
  double rho, rho0, tol, inner_tol, rnorm, hnorm, hprev;
  int outer, inner, max_refine, inner_max, done, inner_done, total_inner, stop;
};
// g64: X^T r (p) and ||r||^2 ([p]) for r = b - X phi.  Checks convergence
// (||M^T g|| <= tol ||r||), else starts CG: w = 0, res = d = M^T g, and
// writes the packed FP32 spectrum of M d (scaled 1/B) to Vhat32.
hipError_t launch_refine_outer(int lgn, int p, RefineState* st, const double* g64, const double* M,
                               const double* Mt, double* w, double* res, double* d,
                               void* Vhat32, const Twiddles& tw, hipStream_t s);
// g: X^T X (M d) (p) from the FP32 Gram pass.  One CG step; when the inner
// solve ends, phi += M w.
hipError_t launch_refine_cg(int lgn, int p, RefineState* st, const double* g, const double* M,
                            const double* Mt, double* w, double* res, double* d, double* phi,
                            void* Vhat32, const Twiddles& tw, hipStream_t s);

hipError_t launch_vec_axpy_small(const double* M, const double* x, const double* y0, int p,
                                 double* out, hipStream_t st);

}  // namespace tls
