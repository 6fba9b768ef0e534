/* tls.h - Toeplitz least squares for AR(p) fitting on AMD MI355X (gfx950).
 *
 * The problem (Section 3, eq. (xphi); Definition 2.1): given a series
 * y_1..y_n and an order p, find phi minimising ||X phi - b||_2, where row t of
 * X holds the p lags (y_{t-1}, ..., y_{t-p}) and b_t = y_t, t = p+1..n.  X is
 * (n-p) x p and Toeplitz (constant descending diagonals), so only the series
 * is ever stored.  By Theorem 2.2 the minimiser solves the normal equations
 * and is unique when X has full column rank.
 *
 * Method: a randomized sketch of [X | b] (uniform row trials, then
 * approximate generalised leverage scores (Definition 3.6, eq. (glev)) and
 * leverage-score row sampling (Algorithm 2, eq. (ldist))) is QR-factored to
 * give R; LSQR preconditioned by R^{-1} then converges to the exact
 * least-squares solution, applying X and X^T by blocked FFT convolution.
 *
 * Conventions for every entry point:
 *  - Coefficients are returned in lag order phi_1..phi_p (eq. (xphi)).
 *  - The caller owns every buffer.  Host pointers are read or written only
 *    during the call.  Device pointers (the *_device and tls_op_* calls) must
 *    be device memory of the context's device and stay valid until the work
 *    queued on `stream` has finished; the library never frees them.
 *  - A stream argument is a hipStream_t passed as void*; NULL means the
 *    context's own stream.  tls_op_* calls only enqueue work; tls_fit* calls
 *    return after the fit is complete.
 *  - Every call returns a tls_status; no exception crosses the ABI.  On any
 *    status other than TLS_OK, TLS_ENOCONV, TLS_ESTALL and TLS_ERANK, outputs
 *    are left unwritten.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef TLS_H_
#define TLS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tls_status;
#define TLS_OK 0          /* success */
#define TLS_EINVAL 1      /* invalid argument: NULL pointer, p < 1, n < 2p + 1, tol not in (0,1), non-finite data */
#define TLS_ERANK 2       /* X numerically rank deficient (Theorem 2.2's singular case), or the preconditioned
                             iteration broke down numerically, or a returned coefficient is not
                             finite (overflow on finite data); outputs hold the last iterate */
#define TLS_ENOCONV 3     /* iteration limit reached; outputs hold the last iterate */
#define TLS_ENOMEM 4      /* device allocation failed */
#define TLS_EDEVICE 5     /* HIP runtime error */
#define TLS_EUNSUPPORTED 6 /* size outside the supported range (p > 1024 or FFT block limits) */
#define TLS_EAGAIN 7      /* served request not finished yet (tls_poll) */
#define TLS_ESTALL 8      /* tol was not met: the iteration stopped improving first (istop 5: the
                             rounding of the FFT products was reached, i.e. the conditioning of X
                             is beyond the working precision); outputs hold the best iterate */

/* Static description of a status code. */
const char* tls_status_string(tls_status s);

#define TLS_PREC_F64 0    /* every step in FP64 */
#define TLS_PREC_MIXED 1  /* FP32 FFT matvecs for the fits whose sketch factor allows them
                             (tls_result.mixed_path); FP64 sketch scores, QR, recurrences and
                             residual */

#define TLS_SKETCH_LEVERAGE 0 /* uniform trials -> generalised leverage scores -> leverage sampling */
#define TLS_SKETCH_UNIFORM 1  /* uniform trials only (Algorithm 1's sampling without the transform) */
#define TLS_SKETCH_RH 2       /* repeated halving (Algorithm 4): nested uniform halvings of the rows
                                 (row r is in level i when its stream-5 draw is below 2^-i), the
                                 uniform sketch standing for the smallest; each level's rows are
                                 scored (eq. (glev)) w.r.t. the sketch of the level below and sampled
                                 into the next sketch, up to all rows.  Batched calls run such fits
                                 one at a time; servers reject it (TLS_EUNSUPPORTED) */

#define TLS_JL_SRHT 0     /* k x p subsampled randomized Hadamard map (Definition 2.4, Algorithm 1) */
#define TLS_JL_GAUSS 1    /* k x p Gaussian map, entries N(0, 1/k) (eq. (glev)) */

/* What a fit returns.  OLS: the least-squares solution of Theorem 2.2,
 * reached by LSQR preconditioned with the sketch's R.  SKETCH: the compressed
 * (sketch-and-solve) estimator of Section 2.1, the solution of eq. (OLSc)
 * min ||S X phi - S b|| on the sampled, rescaled rows, from the same QR of
 * [S X | S b] (no LSQR iterations; resid_norm is still the FP64 residual of
 * the full problem, so resid_norm / (the OLS residual) is the paper's
 * residual ratio). */
#define TLS_EST_OLS 0
#define TLS_EST_SKETCH 1

/* Autotuned block lengths: one log2 B per (precision, order bucket ceil(log2 p),
 * length bucket ceil(log2 (n - p)), clamped to 40); 0 = not tuned. */
#define TLS_TUNE_PRECS 2
#define TLS_TUNE_PBUCKETS 11
#define TLS_TUNE_MBUCKETS 41
#define TLS_TUNE_ENTRIES (TLS_TUNE_PRECS * TLS_TUNE_PBUCKETS * TLS_TUNE_MBUCKETS)

typedef struct tls_options {
  int32_t precision;   /* TLS_PREC_* (default F64) */
  int32_t sketch;      /* TLS_SKETCH_* (default LEVERAGE) */
  int32_t jl_kind;     /* TLS_JL_* (default SRHT) */
  int32_t gamma;       /* sketch rows c = gamma * p (default 8); all rows when c >= n - p */
  int32_t jl_k;        /* columns of the JL map (default 8) */
  int32_t max_iter;    /* LSQR / inner iteration limit (default 1000) */
  int32_t block_lg;    /* log2 of the FFT block length B, 7..14; 0 = automatic */
  int32_t warm_start;  /* 1: start from the compressed problem's solution (default 1) */
  int32_t max_refine;  /* mixed precision: outer FP64 refinement steps for fits too
                          ill-conditioned for FP32 products alone (default 0: those fits
                          run FP64 LSQR; see tls_result.mixed_path) */
  int32_t profile;     /* 1: time every Toeplitz pass with HIP events (tls_result.pass_ms);
                          batched calls then run their launch classes one at a time, so
                          each launch's time is not shared with another class's kernels */
  uint64_t seed;       /* random seed (default 0) */
  uint64_t request_id; /* selects the random streams of one fit (default 0) */
  int32_t no_graph;    /* batched calls: 1 launches every step directly; 0 (default) captures
                          each chunk of LSQR (or inner refinement) steps of a launch class once
                          as a HIP graph and replays it (not while profile = 1) */
  int32_t tick_steps;  /* servers: LSQR steps each fit in flight takes per worker tick (0 =
                          default 24: most fits then finish in the tick that sets them up; fewer
                          steps make shorter ticks but more of them per request) */
  int32_t estimator;   /* TLS_EST_* (default OLS) */
  int32_t reserved1;
  int64_t reserved[2];
} tls_options;

typedef struct tls_result {
  double resid_norm;   /* FP64 ||b - X phi||_2 of the returned phi */
  double kappa_est;    /* max|R_ii| / min|R_ii| of the sketch factor (cheap condition estimate) */
  double lsqr_rnorm;   /* LSQR's own residual estimate */
  double lsqr_arnorm;  /* LSQR's ||A^T r|| estimate */
  int32_t iters;       /* total inner iterations */
  int32_t istop;       /* stop reason: 1, 2 converged; 3 exact; 4 breakdown; 5 the
                          ||A^T r|| estimate stopped decreasing (30 iterations without
                          halving: the rounding of the FFT products was reached before
                          tol; the best iterate is returned with TLS_ESTALL); 7 iteration
                          limit.  Mixed precision: see mixed_path; LSQR's code is
                          reported, and for refinement 2 when it converged (when it
                          stopped contracting or hit its step limit, FP64 LSQR finishes
                          from the best refinement iterate and its code is reported) */
  int32_t refine_steps;/* outer refinement steps (mixed precision), else 0 */
  int32_t sketch_rows; /* c */
  int32_t block_len;   /* FFT block length B used */
  int32_t n_blocks;    /* FFT blocks per pass */
  double t_total_ms;   /* wall time of the call */
  double pass_ms;      /* profile = 1: summed device time of every launch of the dominant
                          Toeplitz pass (pass_kind says which), including launches queued
                          after the fit had converged, which exit at once */
  int32_t pass_count;  /* profile = 1: number of those launches (batched calls: pass_ms and
                          pass_count cover the whole batch's launches, the same in every
                          fit's result) */
  int32_t pass_worked; /* profile = 1: how many of them did work */
  int32_t pass_kind;   /* which pass the three fields above cover: 0 the fused FP64 LSQR
                          pass, 1 the FP32 normal-equation pass of the mixed refinement,
                          2 the fused LSQR pass with FP32 products (mixed_path 1).  A mixed
                          single fit reports the pass of its path (with refinement and an
                          FP64 finish, whichever took more device time); batched mixed
                          calls time the launches of both product precisions and report 2 */
  int32_t mixed_path;  /* mixed precision: the path the fit took, chosen from
                          kappa_F = ||R||_F ||R^{-1}||_F of the sketch factor (>= kappa(R)):
                          1 LSQR with FP32 products (FP32 spectra, u and v's spectrum) and
                          FP64 recurrences to max(tol, 1e-7), when kappa_F <= 300 (the
                          FP32 result is then within about 1e-5 of the FP64 one); 2 FP64
                          refinement around FP32 inner solves, when max_refine > 0 and
                          kappa_F <= 1e8; 3 FP64 LSQR otherwise.  0 for FP64 fits and for
                          the compressed estimator */
} tls_result;

typedef struct tls_ctx tls_ctx;

/* Fill `opt` with the defaults listed above. */
void tls_options_default(tls_options* opt);

/* Create a context on HIP device `device` (its own stream, FFT twiddle
 * tables, a reusable device workspace).  opt may be NULL (defaults).
 * Errors: TLS_EINVAL (ctx NULL), TLS_EDEVICE, TLS_ENOMEM. */
tls_status tls_create(tls_ctx** ctx, int device, const tls_options* opt);

/* Release a context and everything it allocated.  NULL is ignored. */
void tls_destroy(tls_ctx* ctx);

/* Fit AR(p) to the host series y[0..n-1] (Section 3, eq. (xphi)) with the
 * default context (device 0, default options, created on first use).
 * coef: host, p doubles out.  resid_norm: host, 1 double out (FP64
 * ||b - X phi||).  iters: host, 1 int out (LSQR iterations).  tol: LSQR
 * stopping tolerance in (0, 1).  Not thread-safe. */
tls_status tls_fit(const double* series, int64_t n, int32_t p, double tol, double* coef,
                   double* resid_norm, int32_t* iters);

/* Same with an explicit context and options (opt NULL = the context's).
 * series is host memory; coef host, p doubles; out may be NULL. */
tls_status tls_fit_ex(tls_ctx* ctx, const double* series, int64_t n, int32_t p, double tol,
                      const tls_options* opt, double* coef, tls_result* out);

/* Same, with the series already in device memory (d_series, n doubles),
 * work queued on `stream`; coef and out are host memory. */
tls_status tls_fit_device(tls_ctx* ctx, const double* d_series, int64_t n, int32_t p, double tol,
                          const tls_options* opt, void* stream, double* coef, tls_result* out);

/* Batched fits of `count` independent host series: series[i] has n[i]
 * samples and order p[i]; coefficients of fit i go to
 * coef_packed[coef_offset[i] .. + p[i]).  resid_norm, iters, per_fit_status:
 * host arrays of count entries (any may be NULL).  Each fit gives the same
 * result as tls_fit_ex with the same options and request_id = opt.request_id + i.
 * Returns TLS_OK when every fit's status is TLS_OK, else the first failing
 * status; per-fit statuses say which. */
tls_status tls_fit_batch(tls_ctx* ctx, int32_t count, const double* const* series, const int64_t* n,
                         const int32_t* p, double tol, const tls_options* opt, double* coef_packed,
                         const int64_t* coef_offset, double* resid_norm, int32_t* iters,
                         tls_status* per_fit_status);

/* Batched fits of `count` series already in device memory: d_series is a
 * host array of device pointers (series i: n[i] doubles, order p[i]), work
 * queued on `stream` (NULL = the context's stream; the call returns after it
 * has finished).  coef_packed, coef_offset, out (count tls_result entries,
 * may be NULL) and per_fit_status (may be NULL) are host memory.  The fits
 * are grouped by FFT block length and order class and each group runs its
 * kernels as single launches over all of its fits (orders above 623, whose
 * sketch TRSM exceeds the tiles' LDS, and the repeated-halving sketch run
 * one fit at a time inside the call); fit i gives the same result, bit for
 * bit, as tls_fit_device with request_id = opt.request_id + i.
 * The series must stay valid and unmodified until the call returns.
 * Returns TLS_OK when every fit is TLS_OK, else the first failing status. */
tls_status tls_fit_batch_device(tls_ctx* ctx, int32_t count, const double* const* d_series,
                                const int64_t* n, const int32_t* p, double tol,
                                const tls_options* opt, void* stream, double* coef_packed,
                                const int64_t* coef_offset, tls_result* out,
                                tls_status* per_fit_status);

/* ---- block-length autotuner ---------------------------------------------------
 * The FFT block length B of the overlap-save products (eq. (xphi) through
 * circulant embedding) trades FFT work per sample against the p - 1 samples
 * each block re-reads.  tls_autotune measures, on the device and on synthetic
 * data, the per-iteration fused LSQR pass with FP64 products and its column
 * sums (also for the mixed table: a class's B is fixed before each fit's
 * mixed_path is known, and the FP64-product pass is the costlier one) at
 * every admissible B (2p <= B <= 2^14, B no longer than needed for m) for the
 * order buckets covering [p_min, p_max] (measured at p = 2^bucket) and the
 * length buckets covering [n_min, n_max] (measured at m = 2^bucket, at most
 * 2^26; longer buckets take the 2^26 result), and records the fastest in the
 * context.  Fits on this context whose options leave block_lg = 0 then take
 * B from the table (or the built-in rule where the table has no entry), so
 * single, batched and served fits of one context agree bit for bit.  Uses the
 * context's stream and workspace and synchronises; *entries (optional)
 * receives the number of table entries written.  TLS_EINVAL for a bad
 * precision or range (1 <= p_min <= p_max <= 1024, 2 p_max + 1 <= n_min <=
 * n_max). */
tls_status tls_autotune(tls_ctx* ctx, int32_t precision, int32_t p_min, int32_t p_max,
                        int64_t n_min, int64_t n_max, int32_t* entries);
/* Copy the table out (table: TLS_TUNE_ENTRIES bytes, index
 * (prec * TLS_TUNE_PBUCKETS + pbucket) * TLS_TUNE_MBUCKETS + mbucket, prec 0 =
 * F64, 1 = mixed), or replace it, so that a tuned choice can be stored and
 * reused by another process with identical results.  tls_set_tuning rejects
 * (TLS_EINVAL, table unchanged) entries other than 0 or 7..14. */
tls_status tls_get_tuning(const tls_ctx* ctx, int8_t* table);
tls_status tls_set_tuning(tls_ctx* ctx, const int8_t* table);

/* ---- partial autocorrelations and order selection --------------------------
 * The PACF at lags 1..pmax (Definition of the PACF; Algorithm 3's loop over
 * orders): for lag h, the AR(h) fit on the series prefix of n - pmax + h
 * samples (every fit has n - pmax rows), tau_h = its last coefficient
 * phi_{h,h}.  All pmax fits run as one batched call with the options given
 * (estimator OLS: exact PACF; estimator SKETCH: the compressed estimates of
 * Algorithm 3).  *order (optional) receives the largest h with |tau_h| >=
 * 1.96 / sqrt(rows), rows = n - pmax for OLS or the lag's c sampled rows
 * for the compressed estimator (Algorithm 3's order rule), 0 when no lag
 * passes.  d_series: device pointer, read on `stream`; pacf: host [pmax];
 * lag_status (optional): host [pmax], each lag's fit status (lags whose fit
 * failed do not count for the order; a stalled fit, TLS_ESTALL, holds its
 * best iterate and counts).  Returns TLS_OK when every lag's fit is TLS_OK,
 * else the first other status; TLS_EINVAL for NULL pointers,
 * pmax < 1 or n < 2 pmax + 1, TLS_EUNSUPPORTED for pmax > 1024. */
tls_status tls_pacf_device(tls_ctx* ctx, const double* d_series, int64_t n, int32_t pmax,
                           double tol, const tls_options* opt, void* stream, double* pacf,
                           int32_t* order, tls_status* lag_status);

/* ---- LSAR: PACF through approximate leverage scores carried across lags ------
 * Section 3.1 (the LSAR algorithm), the approximate leverage scores
 * definition, eqs. (FALS), (FAR), (FASD), and Algorithm 3.  Lag h (1..pmax)
 * fits AR(h) on the series prefix of n - pmax + h samples (every lag has
 * R = n - pmax rows) by the compressed estimator of eq. (OLSc) on c rows drawn
 * with replacement from pi_h = l_h / h and rescaled 1/sqrt(c pi_h), where
 * l_1(i) = y[i]^2 / sum_{t<R} y[t]^2 and l_h = l_{h-1} + r_{h-1}^2 / ||r_{h-1}||^2
 * with r_{h-1} = X_{h-1} phi_{h-1} - b_{h-1} over all R rows and phi_{h-1} the
 * previous lag's compressed solution.  tau_h = phi_h[h-1].  The block spectra
 * of the series are computed once and every lag's residual is one FFT pass
 * over them.  Lag h draws Philox stream 3 uniforms (h-1) c .. h c - 1 of
 * (opt.seed, opt.request_id); opt.block_lg may fix the FFT block length.
 * d_series: device, n doubles, read on `stream`.  pacf: host [pmax] out.
 * order (optional, host): the largest h whose fit succeeded with
 * |tau_h| >= 1.96 / sqrt(c), 0 when none.  phi_packed (optional, host,
 * pmax (pmax + 1) / 2 doubles): lag h's coefficients at h (h - 1) / 2.
 * rows (optional, host, pmax c int64): lag h's sampled rows at (h - 1) c.
 * lag_status (optional, host [pmax]): TLS_ERANK where lag h's compressed
 * problem was numerically rank deficient.  d_scores (optional, device,
 * n - pmax doubles): the scores l_pmax of the last lag.  Returns TLS_OK when
 * every lag succeeded, else the first failing status; TLS_EINVAL for NULL
 * pointers, pmax < 1, n < 2 pmax + 1 or c outside [pmax + 1, n - pmax];
 * TLS_EUNSUPPORTED for pmax > 1024. */
tls_status tls_lsar_device(tls_ctx* ctx, const double* d_series, int64_t n, int32_t pmax,
                           int32_t c, const tls_options* opt, void* stream, double* pacf,
                           int32_t* order, double* phi_packed, int64_t* rows,
                           tls_status* lag_status, double* d_scores);

/* ---- served continuous batching ----------------------------------------------
 * A server admits fit requests as they arrive and runs them to completion on
 * one device: each tick of its worker thread sets up the newly admitted fits
 * and runs tick_steps LSQR steps (an option, default 24) for every fit in
 * flight, all as batched launches, so
 * short and long, small-p and large-p requests share the device.  A request is
 * admitted first come, first served once its device footprint (series copy,
 * block spectra, sketch, factors, LSQR state: about 25 bytes per sample plus
 * O(c p + p^2) for the FP64 path) fits in the server's HBM budget and a slot is
 * free.  Each request gives the same result, bit for bit, as tls_fit_device
 * with the server's options and request_id, whatever else is in flight.
 * The worker spreads each tick's set-up, LSQR steps and finishing over four
 * streams of its own (work units of different fits; one host
 * synchronisation per tick) and hands finished results to their tickets as
 * soon as they reach the host.  Submit, poll and wait are thread-safe; the
 * context must outlive the server (the server uses only its read-only
 * tables, not its workspace or stream). */
typedef struct tls_server tls_server;
typedef uint64_t tls_ticket;

typedef struct tls_server_stats {
  uint64_t ticks;             /* worker ticks so far */
  uint64_t admitted;          /* requests admitted to the device */
  uint64_t completed;         /* requests finished */
  uint64_t queued;            /* waiting for admission */
  uint64_t in_flight;         /* admitted, not finished */
  uint64_t arena_bytes_in_use;
  uint64_t arena_bytes;       /* the HBM budget */
  tls_status status;          /* TLS_OK, or the device error that stopped the worker */
  int32_t reserved;
} tls_server_stats;

/* Create a server on ctx's device with `hbm_budget` bytes of device memory
 * (allocated now, at least 1 MiB) and at most `max_slots` fits in flight.
 * opt NULL = the context's options.  TLS_PREC_F64 and TLS_PREC_MIXED are served
 * (mixed: each fit's products FP32 or FP64 by its mixed_path, without the
 * refinement band: max_refine > 0 gives TLS_EUNSUPPORTED), not the
 * repeated-halving sketch (TLS_EUNSUPPORTED); other precisions TLS_EINVAL.
 * TLS_ENOMEM if the budget cannot be allocated. */
tls_status tls_server_create(tls_ctx* ctx, size_t hbm_budget, int32_t max_slots,
                             const tls_options* opt, tls_server** out);

/* Queue a fit of the host series (copied before return) of length n, order p,
 * LSQR tolerance tol; request_id selects its random streams (Philox fit id).
 * Validation as tls_fit_ex: TLS_EINVAL, TLS_EUNSUPPORTED (p > 623), TLS_ENOMEM
 * (footprint above the whole budget).  *ticket identifies the request. */
tls_status tls_submit(tls_server* server, const double* series, int64_t n, int32_t p, double tol,
                      uint64_t request_id, tls_ticket* ticket);

/* Same with the series in device memory on the server's device, borrowed (not
 * copied): it must stay valid and unmodified until the request is finished. */
tls_status tls_submit_device(tls_server* server, const double* d_series, int64_t n, int32_t p,
                             double tol, uint64_t request_id, tls_ticket* ticket);

/* Result of a finished request: coef (host, p doubles), out and fit_status
 * (the status tls_fit_device would return) may each be NULL; out->t_total_ms
 * is the request's latency from submission to completion.  Returns TLS_OK and
 * forgets the ticket, TLS_EAGAIN while the request is in flight (tls_poll),
 * or TLS_EINVAL for an unknown ticket.  tls_wait blocks until finished. */
tls_status tls_poll(tls_server* server, tls_ticket ticket, double* coef, tls_result* out,
                    tls_status* fit_status);
tls_status tls_wait(tls_server* server, tls_ticket ticket, double* coef, tls_result* out,
                    tls_status* fit_status);

tls_status tls_server_get_stats(tls_server* server, tls_server_stats* out);

/* Runs every queued and in-flight request to completion, then frees the
 * server; results not yet taken are discarded. */
void tls_server_destroy(tls_server* server);

/* ---- step-level entry points (device pointers; work enqueued on stream) ----
 * These run one step of the path on its own so that each step can be checked
 * against the CPU oracle.  prec: TLS_PREC_F64 or TLS_PREC_MIXED (FP32 data).
 * B: FFT block length (power of two, 128..16384, B >= 2p).  Block layout:
 * block k covers rows [kL, kL + L), L = B - p + 1, nblocks = ceil((n-p)/L). */

/* Number of FFT blocks for (n, p, B), or -1 if B is invalid. */
int64_t tls_num_blocks(int64_t n, int32_t p, int32_t B);

/* Packed block spectra of the series (the length-B real DFT of each window
 * y[kL .. kL+B), zero past the end): d_spec receives nblocks * B/2 complex
 * values (FP64 pairs for F64, FP32 pairs for MIXED); word 0 of a block holds
 * (X[0], X[B/2]), word j the bin X[j]. */
tls_status tls_op_spectra(tls_ctx* ctx, int32_t prec, const double* d_y, int64_t n, int32_t p,
                          int32_t B, void* d_spec, void* stream);

/* One pass of the lag matrix over a vector (eq. (xphi)):
 *   e = s1 * X v + s2 * w     (v: host, p doubles; w: device, n-p values or NULL)
 *   d_e (device, n-p values, may alias d_w; NULL = not stored)
 *   d_out (device, p+1 doubles): X^T e in [0, p) when want_rmv, ||e||^2 in [p].
 * If v is NULL, e = d_u_in (device, n-p values) and only X^T e, ||e||^2 are
 * formed.  Vectors of n-p values are FP64 (F64) or FP32 (MIXED). */
tls_status tls_op_toeplitz(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n, int32_t p,
                           int32_t B, const double* v, double s1, double s2, const void* d_w,
                           void* d_e, const void* d_u_in, int32_t want_rmv, double* d_out,
                           void* stream);

/* tls_op_toeplitz without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results, bit for bit, as
 * tls_op_toeplitz; its scratch lives in a fixed 16 MiB device array per
 * device, held until the process ends, instead of the context workspace.
 * The scratch is v, (s1, s2), v's spectrum (B/2 complex doubles) and the
 * partial sums, (p + 1) x ceil(nblocks / g) doubles with g = 4 for
 * B <= 1024, 2 for B <= 4096, else 1 (each slice rounded up to 256 bytes);
 * sizes needing more than 16 MiB return TLS_EUNSUPPORTED before any work is
 * queued (for p = 100, B = 1024: up to about 80 million series samples).
 * Every call on one device shares that device's array: calls that overlap
 * on one device (any contexts, streams or threads) race, so the caller must
 * order them.  The array is not cleared between calls (every byte it uses is
 * written before it is read).  The host copy of v is from pageable memory,
 * so the call synchronises `stream` before returning. */
tls_status tls_op_toeplitz_noalloc(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n,
                                   int32_t p, int32_t B, const double* v, double s1, double s2,
                                   const void* d_w, void* d_e, const void* d_u_in,
                                   int32_t want_rmv, double* d_out, void* stream);

/* Approximate generalised leverage scores in product form (eq. (glev)):
 * d_scores[i] = sum_q ((X omega_q)[i])^2 for the p x k matrix d_omega
 * (device FP64, column-major, columns contiguous).  d_scores: n-p values,
 * FP64 or FP32 by prec. */
tls_status tls_op_scores(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n, int32_t p,
                         int32_t B, const double* d_omega, int32_t k, void* d_scores, void* stream);

/* Leverage-score sampling (Algorithm 2, eq. (ldist)): c draws with
 * replacement from pi_i = s_i / sum s, by the inverse CDF of the running
 * total in row order; row i is rescaled by 1/sqrt(c pi_i).  d_u: device, c
 * uniforms in [0,1) (NULL: Philox stream 3 of (seed, fit)).  d_idx: c int64;
 * d_scale: c doubles.  d_scores FP64 or FP32 by prec. */
tls_status tls_op_sample(tls_ctx* ctx, int32_t prec, const void* d_scores, int64_t m,
                         const double* d_u, int32_t c, uint64_t seed, uint32_t fit,
                         int64_t* d_idx, double* d_scale, void* stream);

/* Repeated halving (Algorithm 4): zero the entries r of d_scores (m values,
 * FP64 or FP32 by prec, device) whose row is outside level `level` >= 0,
 * i.e. whose Philox stream-5 draw u_r of (seed, fit) is not below 2^-level
 * (level 0 keeps every row). */
tls_status tls_op_rh_mask(tls_ctx* ctx, int32_t prec, void* d_scores, int64_t m, int32_t level,
                          uint64_t seed, uint32_t fit, void* stream);

/* Sketch rows scale_t * [X(idx_t, :), b(idx_t)] into d_A (device FP64,
 * row-major, crows x ldq; rows >= c and columns >= p+1 zeroed).
 * mode 0: d_idx/d_scale given; 1: uniform trials from Philox stream 0 of
 * (seed, fit) with scale sqrt(m/c) (Algorithm 1), idx/scale written out if
 * non-NULL; 2: every row (c = n - p, scale 1). */
tls_status tls_op_gather(tls_ctx* ctx, const double* d_y, int64_t n, int32_t p, int32_t mode,
                         int64_t* d_idx, double* d_scale, int32_t c, int32_t crows, int32_t ldq,
                         double* d_A, uint64_t seed, uint32_t fit, void* stream);

/* QR of the sketch (Section 2.1: QR of the compressed matrix): upper
 * triangular d_R (q x q, row-major, non-negative diagonal) with
 * A^T A = R^T R for the crows x ldq row-major d_A (crows % 16 == 0,
 * ldq % 16 == 0, q <= ldq; d_A is overwritten).  *status_out (host) gets the
 * breakdown bits: 1 = the shifted first sweep broke down, 2 = a later sweep
 * broke down, 4 = min|R_ii| <= q u max|R_ii|; 2 or 4 mean numerically rank
 * deficient; 8 (informational) = the third refining sweep ran.  Synchronises
 * the stream. */
tls_status tls_op_qr(tls_ctx* ctx, double* d_A, int32_t crows, int32_t q, int32_t ldq,
                     double* d_R, int32_t* status_out, void* stream);

/* d_M = R[:p,:p]^{-1} (row-major, upper) and d_phi0 = R[:p,:p]^{-1} R[:p,p]
 * (the compressed problem's solution) from the q x q row-major d_R (q = p+1,
 * or q = p with d_phi0 NULL). */
tls_status tls_op_triinv(tls_ctx* ctx, const double* d_R, int32_t q, int32_t p, double* d_M,
                         double* d_phi0, void* stream);

/* The k x p JL map Pi (kind TLS_JL_*) from Philox streams of (seed, fit) and
 * Omega = R[:p,:p]^{-1} Pi^T (p x k column-major; eq. (glev): the scores are
 * the squared row norms of X Omega) for the upper-triangular q x q row-major
 * d_R (q >= p; entries below the diagonal are not read), by back
 * substitution.  d_Pi may be NULL.  TLS_EUNSUPPORTED for p > 1024. */
tls_status tls_op_jl(tls_ctx* ctx, const double* d_R, int32_t q, int32_t p, int32_t k,
                     int32_t kind, uint64_t seed, uint32_t fit, double* d_Pi, double* d_omega,
                     void* stream);

/* count Philox4x32-10 uniforms of stream `rng_stream`, fit `fit`, seed
 * `seed`, draws start .. start+count-1, into d_out (device FP64). */
tls_status tls_op_philox(tls_ctx* ctx, uint64_t seed, uint32_t rng_stream, uint32_t fit,
                         uint64_t start, int64_t count, double* d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TLS_H_ */
