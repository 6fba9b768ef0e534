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
  const void* d64 = nullptr;  // cx<double>[BMAX], see build_twiddles
  const void* d32 = nullptr;  // cx<float>[BMAX]
};

// Threads per block transform of the Toeplitz pass at complex length 2^lgn:
// eight points each (one radix-8 butterfly per stage), at most 256.
constexpr int pass_nt(int lgn) {
  return (1 << lgn) / 8 < 8 ? 8 : ((1 << lgn) / 8 > 256 ? 256 : (1 << lgn) / 8);
}

// Blocks per workgroup of the Toeplitz pass: that many blocks are
// transformed side by side (each by pass_nt(lgn) threads; short blocks fill
// a 256-thread workgroup) and their X^T products share one inverse
// transform; the pass writes its partials per group of pass_nw(lgn)
// consecutive blocks.
constexpr int pass_nw(int lgn) {
  return lgn <= 9 ? 256 / pass_nt(lgn) : (lgn <= 11 ? 2 : 1);
}
inline int pass_groups(int lgn, int nblocks) {
  return (nblocks + pass_nw(lgn) - 1) / pass_nw(lgn);
}

hipError_t launch_spectra(int prec, int lgn, const double* y, int64_t n, int L, int nblocks,
                          void* Yhat, const Twiddles& tw, hipStream_t st);
// partial: (p + 1) x pass_groups(lgn, nblocks) doubles, column-major.
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
// draw0: counter of the first Philox draw (draw t uses counter draw0 + t)
hipError_t launch_sample(int prec, const void* scores, int64_t m, const double* u, int c,
                         int64_t* idx, double* scale, double* work, uint64_t seed, uint32_t fit,
                         hipStream_t st, uint64_t draw0 = 0);
// Repeated halving: scores of rows outside level `level` set to zero.
hipError_t launch_rh_mask(int prec, void* scores, int64_t m, int level, uint64_t seed,
                          uint32_t fit, hipStream_t st);
size_t sample_work_doubles(int64_t m);
// Pi (k x p JL map) and Omega = R[:p,:p]^{-1} Pi^T (p x k, column-major) for
// upper-triangular R (row-major, leading dimension ldr >= p), p <= 1024.
// JL columns solved together by one wavefront at order p (fewer for long
// columns, so that the right-hand sides stay in registers).
constexpr int jl_cols(int p) { return p <= 128 ? 8 : (p <= 256 ? 4 : (p <= 512 ? 2 : 1)); }
hipError_t launch_jl_solve(const double* R, int ldr, int p, int k, int kind, double* Pi,
                           double* Om, uint64_t seed, uint32_t fit, hipStream_t st);

// Largest leading dimension (a multiple of 16) of the sketch whose TRSM runs
// on LDS tiles; larger ones take the global-memory TRSM (single fits) or run
// one fit at a time (batched calls).
constexpr int TRSM_TILE_LDQ_MAX = 624;

// QR of the sketch and triangular helpers
// rank_cols: leading columns whose breakdown or tiny pivot means rank
// deficiency (the sketch [S X | S b] passes p: b may lie in the range of X).
// A: crows x ldq row-major, crows % 16 == 0.  G: qr_scratch_doubles() doubles.
size_t qr_scratch_doubles(int crows, int q, int ldq);
// sweeps: 3 = shifted Cholesky QR then one refining sweep, and a second one
// only when the first refining Cholesky needed the shift (A R^{-1}
// orthonormal to about 1e-6 or better); 1 = the shifted sweep alone (a
// rougher R, enough for approximate leverage scores).
// Register-tile class of the Cholesky (order q) and triangular inverse
// (order p) kernels: ceil(n/16) for n <= 128 (16 x 16 threads), 100 +
// ceil(n/32) for 128 < n <= 224 (32 x 32 threads), 0 above (blocked kernels on
// 32 x 32 blocks, one launch per block column).
inline int reg_tiles(int n) {
  if (n <= 128) return (n + 15) / 16;
  if (n <= 224) return 100 + (n + 31) / 32;
  return 0;
}
hipError_t launch_qr(double* A, int crows, int q, int ldq, int rank_cols, int sweeps, double* R,
                     double* G, double* R1, double* R2, int* status, hipStream_t st);
// dminmax (optional): max and min |R_ii| over the first p diagonal entries.
hipError_t launch_triinv(const double* R, int q, int p, double* M, double* Mt, double* phi0,
                         int* status, hipStream_t st, double* dminmax = nullptr);

// LSQR p-side step and state
struct LsqrState {
  double alpha, beta, rhobar, phibar, anorm2, bnorm, rnorm, arnorm, znorm, tol;
  double coef[2];
  double best_ratio;  // smallest ||A^T r|| / (||A|| ||r||) estimate so far (2x steps)
  int iter, istop, done, max_iter, phase, best_iter;
  int f32;  // mixed precision: 1 when the fit's LSQR products are FP32
};
// q: p doubles of scratch for the wide step (p > 128 with M in global
// memory: the products over many workgroups); NULL keeps one workgroup.
// snap: NULL, or host-mapped memory (pinned) that receives the state after
// this step, also when the iteration had stopped before it.
hipError_t launch_lsqr_step(int prec, int lgn, int p, LsqrState* st, const double* g,
                            const double* M, const double* Mt, double* v, double* w, double* z,
                            const double* phi0, double* phi, void* Vhat, double* q,
                            LsqrState* snap, const Twiddles& tw, hipStream_t stream);
// Mixed-precision refinement (FP64 outer residual, FP32 inner CG on the
// preconditioned normal equations).
struct RefineState {
  double rho, rho0, tol, inner_tol, rnorm, hnorm, hprev, hbest;
  int outer, inner, max_refine, inner_max, done, inner_done, total_inner, stop;
  int path;  // mixed precision: the fit's path (MixedPath in engine.h)
};
// g64: X^T r (p) and ||r||^2 ([p]) for r = b - X phi.  Keeps the iterate with
// the smallest preconditioned gradient in phib.  Checks convergence
// (||M^T g|| <= tol ||r||), else starts CG: w = 0, res = d = M^T g, and
// writes the packed FP32 spectrum of M d (scaled 1/B) to Vhat32.
hipError_t launch_refine_outer(int lgn, int p, RefineState* st, const double* g64, const double* M,
                               const double* Mt, const double* phi, double* phib, double* w,
                               double* res, double* d, void* Vhat32, const Twiddles& tw,
                               hipStream_t s);
// g: X^T X (M d) (p) from the FP32 Gram pass.  One CG step; when the inner
// solve ends, phi += M w.
hipError_t launch_refine_cg(int lgn, int p, RefineState* st, const double* g, const double* M,
                            const double* Mt, double* w, double* res, double* d, double* phi,
                            void* Vhat32, const Twiddles& tw, hipStream_t s);

// ---- batched fits -----------------------------------------------------------
// Device descriptor of one fit of a batch: its sizes and its slice of the
// batch workspace.  Every fit of one batched run shares the FFT block length,
// the precision and the options.
struct FitDesc {
  const double* y;
  int64_t n, m;
  double tol;
  int p, q, ldq, c, crows, k, L, nblocks, ngroups, nchunks, all_rows;
  uint32_t fit;
  void* Yhat;
  void* Yhat64;
  void* u;
  double *partial, *g, *A, *G, *R1, *R2, *R, *M, *Mt, *Pi, *Om;
  void* Omhat;
  void* Vhat;
  void* Vhat32;
  double *v, *w, *z, *phi0, *phi, *phib;
  int64_t* idx;
  double *scale, *swork;
  LsqrState* st;
  RefineState* rst;
  int* status;
  double *rpart, *rr, *dminmax, *cw, *cres, *cd;
};

// Work items {fit, local index} of a batched launch (one workgroup each).
struct Item {
  int fit, idx;
};

// Variants of the batched Toeplitz pass.
enum BatchPass : int {
  BP_LSQR_FIRST = 0,  // FP64: e = b - X phi0 into u, X^T e (FP64 spectra)
  BP_LSQR = 1,        // FP64: e = X (M v) - (alpha/beta) u in place, X^T e
  BP_OUTER64 = 2,     // FP64: r = b - X phi, X^T r (nothing stored)
  BP_INNER32 = 3,     // FP32: X^T X (M d) (nothing stored)
  BP_LSQR32 = 4,      // FP32 products: e = X (M v) + s2 u in place (u in FP32; it holds b
                      // before the first step), X^T e
};

hipError_t launch_spectra_b(int prec, int lgn, const Item* items, int nitems, const FitDesc* D,
                            int to64, const Twiddles& tw, hipStream_t st);
hipError_t launch_toep_b(int prec, int lgn, int variant, const Item* items, int nitems,
                         const FitDesc* D, const double* consts, const Twiddles& tw,
                         hipStream_t st);
hipError_t launch_small_rfft_b(int prec, int lgn, int variant, const Item* items, int nitems,
                               const FitDesc* D, const Twiddles& tw, hipStream_t st);
hipError_t launch_scores_b(int prec, int lgn, const Item* items, int nitems, const FitDesc* D,
                           const Twiddles& tw, hipStream_t st);
// variant 0: LSQR partials -> g (flag st->done); 1: outer64 (flag rst->done);
// 2: inner32 (flag rst->inner_done); 3: residual partials -> rr
hipError_t launch_colsum_b(int variant, const Item* items, int nitems, const FitDesc* D,
                           hipStream_t st);
hipError_t launch_resid_b(const Item* items, int nitems, const FitDesc* D, int pmax,
                          hipStream_t st);
hipError_t launch_gather_b(int stage, const Item* items, int nitems, const FitDesc* D,
                           uint64_t seed, hipStream_t st);
hipError_t launch_sample_b(int prec, const Item* chunk_items, int nchunk_items,
                           const Item* draw_items, int ndraw_items, const Item* fit_items,
                           int nfit_items, const FitDesc* D, uint64_t seed, hipStream_t st);
hipError_t launch_jl_b(const Item* items, int nitems, const FitDesc* D, int kind, int pmax,
                       uint64_t seed, hipStream_t st);
// stage 1: one shifted sweep into R (rank bits to status[2]); stage 2: three
// sweeps into R (status[0]).  Item lists: Gram tiles (fit, tile of the
// ldq/16 x ldq/16 grid), 16-row tiles (fit, tile), rows of R (fit, row), and
// one item per fit.  qt = ceil(qmax/16) <= 8, or 0 for the blocked kernels.
hipError_t launch_qr_b(int stage, int qt, const Item* tiles, int ntiles, const Item* rowtiles,
                       int nrowtiles, const Item* rows, int nrows, const Item* fits, int nfits,
                       int ldqmax, const FitDesc* D, hipStream_t st);
// M, Mt, phi0 of the final factor (rank bits to status[1]), |R_ii| range.
hipError_t launch_triinv_b(int pt, const Item* fits, int nfits, int pmax, const FitDesc* D,
                           hipStream_t st);
// One workgroup per item of `fits` (item.fit indexes D).  counts[0] += 1 for
// each fit that finishes (LSQR) or is finished (refinement outer step);
// counts[1] += 1 for each fit whose inner CG solve is finished; the LSQR step
// appends each fit it finishes to done_list (when non-null; length in
// counts[2]).  mlds must equal lsqr_step_lds(lgn, p) for every fit (the
// single-fit kernel's choice).
bool lsqr_step_lds(int lgn, int p);
hipError_t launch_lsqr_step_b(int prec, int lgn, const Item* fits, int nfits, int pmax, bool mlds,
                              const FitDesc* D, int* counts, int* done_list, const Twiddles& tw,
                              hipStream_t st);
hipError_t launch_refine_outer_b(int lgn, const Item* fits, int nfits, int pmax, const FitDesc* D,
                                 int* counts, const Twiddles& tw, hipStream_t st);
hipError_t launch_refine_cg_b(int lgn, const Item* fits, int nfits, int pmax, const FitDesc* D,
                              int* counts, const Twiddles& tw, hipStream_t st);

hipError_t launch_vec_axpy_small(const double* M, const double* x, const double* y0, int p,
                                 double* out, hipStream_t st);

}  // namespace tls
