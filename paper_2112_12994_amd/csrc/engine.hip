// Host engine and C-ABI of the Toeplitz least-squares library: contexts,
// device workspace, the per-fit plan (FFT block length, sketch size) and the
// orchestration of the kernels for one fit.
#include "engine.h"

tls_status run_fit(tls_ctx* ctx, const Plan& pl, const tls_options& o, const double* d_y_in,
                   const double* host_y, double tol, hipStream_t s, double* coef, tls_result* res) {
  const auto t0 = std::chrono::steady_clock::now();
  FitBufs b{};
  const size_t need = carve(pl, host_y != nullptr, &b, nullptr);
  TLS_CHECK(ensure_ws(ctx, need));
  carve(pl, host_y != nullptr, &b, static_cast<char*>(ctx->ws));
  TLS_CHECK(ensure_pinned(ctx, sizeof(HostOut) + pl.p * sizeof(double) + 64));
  HostOut* ho = static_cast<HostOut*>(ctx->pinned);
  double* hphi = reinterpret_cast<double*>(ho + 1);

  const double* d_y = d_y_in;
  if (host_y) {
    TLS_CHECK(hipMemcpyAsync(b.y, host_y, pl.n * sizeof(double), hipMemcpyHostToDevice, s));
    d_y = b.y;
  }
  const int prec = pl.prec;
  const int p = pl.p, q = pl.q;
  const double invB = 1.0 / pl.B;
  const uint64_t seed = o.seed;
  const uint32_t fit = static_cast<uint32_t>(o.request_id);
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;

  hipLaunchKernelGGL(fill_state_kernel, dim3(1), dim3(64), 0, s, b.st, tol, max_iter, b.status);
  TLS_CHECK(hipGetLastError());

  // Spectra of the series blocks.
  if (prec == TLS_PREC_MIXED) {
    TLS_CHECK(launch_spectra(PREC_F32, pl.lgn, d_y, pl.n, pl.L, pl.nblocks, b.Yhat, ctx->tw, s));
    TLS_CHECK(launch_spectra(PREC_F64, pl.lgn, d_y, pl.n, pl.L, pl.nblocks, b.Yhat64, ctx->tw, s));
  } else {
    TLS_CHECK(launch_spectra(PREC_F64, pl.lgn, d_y, pl.n, pl.L, pl.nblocks, b.Yhat, ctx->tw, s));
  }

  // Sketch -> R.
  if (pl.all_rows) {
    TLS_CHECK(launch_gather(d_y, pl.m, p, 2, nullptr, nullptr, pl.c, pl.crows, pl.ldq, b.A,
                            nullptr, nullptr, seed, fit, s));
  } else {
    TLS_CHECK(launch_gather(d_y, pl.m, p, 1, nullptr, nullptr, pl.c, pl.crows, pl.ldq, b.A, b.idx,
                            b.scale, seed, fit, s));
    if (o.sketch == TLS_SKETCH_LEVERAGE || o.sketch == TLS_SKETCH_RH) {
      // Leverage sketch: one level (scores of all rows w.r.t. the uniform
      // sketch).  Repeated halving: the uniform sketch stands for the
      // smallest of the nested halvings; going up, each level's rows are
      // scored w.r.t. the sketch of the level below and sampled into the
      // next sketch, the last level being all rows.
      const int levels = o.sketch == TLS_SKETCH_RH ? rh_levels(pl.m, pl.c) : 1;
      for (int lev = levels - 1; lev >= 0; --lev) {
        TLS_CHECK(launch_qr(b.A, pl.crows, q, pl.ldq, p, 1, b.R, b.G, b.R1, b.R2, b.status + 2, s));
        TLS_CHECK(launch_jl_solve(b.R, q, p, pl.k, o.jl_kind, b.Pi, b.Om, seed, fit, s));
        // scores and draws in FP64 in every precision (mixed: from the FP64 spectra)
        TLS_CHECK(launch_small_rfft(PREC_F64, pl.lgn, b.Om, p, p, pl.k, invB, b.Omhat, ctx->tw,
                                    nullptr, s));
        TLS_CHECK(launch_scores(PREC_F64, pl.lgn, b.Yhat64, b.Omhat, pl.k, b.u, ctx->tw, pl.m, p,
                                pl.L, pl.nblocks, s));
        if (lev > 0) TLS_CHECK(launch_rh_mask(PREC_F64, b.u, pl.m, lev, seed, fit, s));
        TLS_CHECK(launch_sample(PREC_F64, b.u, pl.m, nullptr, pl.c, b.idx, b.scale, b.swork, seed,
                                fit, s, static_cast<uint64_t>(lev) * pl.c));
        TLS_CHECK(launch_gather(d_y, pl.m, p, 0, b.idx, b.scale, pl.c, pl.crows, pl.ldq, b.A,
                                nullptr, nullptr, seed, fit, s));
      }
    }
  }
  TLS_CHECK(launch_qr(b.A, pl.crows, q, pl.ldq, p, 3, b.R, b.G, b.R1, b.R2, b.status, s));
  TLS_CHECK(launch_triinv(b.R, q, p, b.M, b.Mt, b.phi0, b.status + 1, s, b.dminmax));
  const bool compressed = o.estimator == TLS_EST_SKETCH;
  if (!o.warm_start && !compressed) {
    hipLaunchKernelGGL(zero_kernel, dim3((p + 255) / 256), dim3(256), 0, s, b.phi0, p);
  }
  TLS_CHECK(hipGetLastError());

  int total_iters = 0, istop = 0, refine = 0, pass_count = 0, pass_worked = 0, pass_kind = 0;
  double pass_ms = 0.0, lsqr_rnorm = 0.0, lsqr_arnorm = 0.0;

  // LSQR on A = X M from phi0 with products of precision `pp` over the
  // spectra `spec` (FP64: the FP64 spectra; FP32: the FP32 spectra, u and v's
  // spectrum in FP32, recurrences in FP64); `timed`: event pairs around every
  // fused pass.
  auto lsqr_run = [&](int pp, const void* spec, bool timed) -> tls_status {
    const int* flag = &b.st->done;
    void* vh = pp == PREC_F64 ? b.Vhat : b.Vhat32;
    size_t npass = 0;
    hipEvent_t ea = nullptr, eb = nullptr;
    // snap: NULL, or the host ring slot that receives the state after this
    // step (written by the step kernel itself)
    auto pass = [&](const void* w_in, LsqrState* snap) -> tls_status {
      if (timed) {
        TLS_CHECK(pass_events(ctx, npass, &ea, &eb));
        TLS_CHECK(hipEventRecord(ea, s));
      }
      TLS_CHECK(launch_toep(pp, pl.lgn, MODE_FUSED, spec, vh, w_in, b.u, nullptr, b.partial,
                            b.st->coef, flag, ctx->tw, pl.m, p, pl.L, pl.nblocks, s));
      if (timed) {
        TLS_CHECK(hipEventRecord(eb, s));
        ++npass;
      }
      TLS_CHECK(launch_colsum(b.partial, pl.ngroups, p + 1, b.g, flag, s));
      TLS_CHECK(launch_lsqr_step(pp, pl.lgn, p, b.st, b.g, b.M, b.Mt, b.v, b.w, b.z, b.phi0,
                                 b.phi, vh, b.q, snap, ctx->tw, s));
      return TLS_OK;
    };
    TLS_CHECK(launch_small_rfft(pp, pl.lgn, b.phi0, p, p, 1, invB, vh, ctx->tw, nullptr, s));
    if (pp != PREC_F64) {
      // the first pass's w term is b = y[p:], held in u in FP32
      hipLaunchKernelGGL(to_f32_kernel, dim3(static_cast<int>(std::min<int64_t>((pl.m + 255) / 256, 4096))),
                         dim3(256), 0, s, d_y + p, static_cast<float*>(b.u), pl.m);
      TLS_CHECK(hipGetLastError());
    }
    tls_status e = pass(pp == PREC_F64 ? static_cast<const void*>(d_y + p) : b.u, nullptr);
    if (e != TLS_OK) return e;
    // Chunks of iterations with one chunk always queued behind the one the
    // host waits for, so the device never idles on the host's convergence
    // check; iterations queued after convergence exit at once.  The first
    // check comes after CHUNK_ITERS iterations with half as many queued
    // behind it.  Later chunks run to where the convergence test is
    // expected to pass: the stopping ratio ||A^T r|| / (||A|| ||r||)
    // falls about geometrically, so its rate between two checks predicts
    // the iterations left; a chunk stops one short of that (the next check
    // then sees the last ones queued) and takes 2 to 8 iterations.
    int launched = 0;
    int prev_iter = -1;
    double prev_ratio = 0.0;
    auto next_chunk = [&](const LsqrState& st) -> int {
      const double an = sqrt(st.anorm2);
      const double ratio = an > 0.0 && st.rnorm > 0.0 ? st.arnorm / (an * st.rnorm) : 0.0;
      int n = 2;
      if (prev_iter >= 0 && st.iter > prev_iter && ratio > 0.0 && prev_ratio > ratio) {
        const double rate = pow(ratio / prev_ratio, 1.0 / (st.iter - prev_iter));
        if (ratio > st.tol && rate < 1.0) {
          const double left = ceil(log(st.tol / ratio) / log(rate));
          const int queued = launched - st.iter - 1;  // launched after this snapshot
          n = static_cast<int>(std::min(8.0, std::max(2.0, left - queued - 1)));
        }
      }
      prev_iter = st.iter;
      prev_ratio = ratio;
      return n;
    };
    // a chunk's last step writes the state into its ring slot in pinned
    // host memory (no copy launch on the stream)
    int last_slot = 0;
    auto chunk = [&](int iters, int slot) -> tls_status {
      for (int it = 0; it < iters; ++it) {
        const tls_status ec = pass(b.u, it + 1 == iters ? &ho->ring[slot] : nullptr);
        if (ec != TLS_OK) return ec;
      }
      launched += iters;
      last_slot = slot;
      TLS_CHECK(hipEventRecord(ctx->chunk_ev[slot], s));
      return TLS_OK;
    };
    e = chunk(CHUNK_ITERS, 0);
    if (e == TLS_OK) e = chunk(CHUNK_ITERS / 2, 1);
    if (e != TLS_OK) return e;
    for (int k = 0;; ++k) {
      const int slot = k & 1;
      TLS_CHECK(hipEventSynchronize(ctx->chunk_ev[slot]));
      if (ho->ring[slot].done || launched > max_iter + 2 * CHUNK_ITERS) break;
      e = chunk(next_chunk(ho->ring[slot]), slot);
      if (e != TLS_OK) return e;
    }
    // the last chunk launched ends the iteration: its snapshot is the final state
    TLS_CHECK(hipStreamSynchronize(s));
    ho->st = ho->ring[last_slot];
    if (timed) {
      // passes 0 .. iter did work; later launches in the last chunk exit at once
      double ms = 0.0;
      for (size_t i = 0; i < npass; ++i) {
        float t = 0.f;
        TLS_CHECK(hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]));
        ms += t;
      }
      pass_ms = ms;
      pass_count = static_cast<int>(npass);
      pass_worked = static_cast<int>(std::min(npass, static_cast<size_t>(ho->st.iter) + 1));
    }
    return TLS_OK;
  };

  // mixed precision: the path from kappa_F of the sketch factor
  int mixed_path = MP_NONE;
  if (!compressed && prec == TLS_PREC_MIXED) {
    hipLaunchKernelGGL(kappa_f_kernel, dim3(1), dim3(256), 0, s, b.R, q, b.M, p, b.dminmax + 2);
    TLS_CHECK(hipGetLastError());
    TLS_CHECK(hipMemcpyAsync(ho->dminmax, b.dminmax, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    TLS_CHECK(hipStreamSynchronize(s));
    const double kf = ho->dminmax[2];
    mixed_path = mixed_path_of(kf == kf ? kf : INFINITY, o.max_refine);
  }
  if (compressed) {
    // the compressed problem's solution (eq. (OLSc)), no iterations
    hipLaunchKernelGGL(copy_vec_kernel, dim3((p + 255) / 256), dim3(256), 0, s, b.phi0, p, b.phi);
    TLS_CHECK(hipGetLastError());
  } else if (prec == TLS_PREC_F64 || mixed_path == MP_F32 || mixed_path == MP_F64) {
    if (mixed_path == MP_F32) {
      hipLaunchKernelGGL(set_tol_kernel, dim3(1), dim3(64), 0, s, b.st, fmax(tol, MIXED_TOL_F32));
      TLS_CHECK(hipGetLastError());
    }
    const tls_status e = mixed_path == MP_F32 ? lsqr_run(PREC_F32, b.Yhat, o.profile != 0)
                                         : lsqr_run(PREC_F64, prec == TLS_PREC_F64 ? b.Yhat : b.Yhat64,
                                                    o.profile != 0);
    if (e != TLS_OK) return e;
    total_iters = ho->st.iter;
    istop = ho->st.istop;
    lsqr_rnorm = ho->st.rnorm;
    lsqr_arnorm = ho->st.arnorm;
    if (mixed_path == MP_F32) pass_kind = 2;
  } else {
    // Mixed precision: FP64 residual and gradient of the current phi, then a
    // CG solve of the preconditioned normal equations for the correction,
    // whose X^T X products are single FP32 passes over the FP32 spectra.
    // When the FP32 products stop contracting (conditioning beyond their
    // resolution) or the step limit is reached, FP64 LSQR over the FP64
    // spectra finishes from the best iterate.
    const int max_refine = o.max_refine;
    const int inner_max = std::min(max_iter, 25);
    constexpr int INNER_CHUNK = 6;
    hipLaunchKernelGGL(fill_refine_kernel, dim3(1), dim3(64), 0, s, b.rst, tol, max_refine,
                       inner_max, 1e-5);
    hipLaunchKernelGGL(copy_vec_kernel, dim3((p + 255) / 256), dim3(256), 0, s, b.phi0, p, b.phi);
    TLS_CHECK(hipGetLastError());
    size_t npass = 0;
    hipEvent_t ea = nullptr, eb = nullptr;
    RefineState* hr = &ho->rs;
    double all_ms = 0.0;
    int worked_passes = 0;
    for (int outer = 0; outer <= max_refine; ++outer) {
      const size_t first_pass = npass;
      TLS_CHECK(launch_small_rfft(PREC_F64, pl.lgn, b.phi, p, p, 1, invB, b.Vhat, ctx->tw, nullptr, s));
      TLS_CHECK(launch_toep(PREC_F64, pl.lgn, MODE_FUSED, b.Yhat64, b.Vhat, d_y + p, nullptr, nullptr,
                            b.partial, ctx->consts, &b.rst->done, ctx->tw, pl.m, p, pl.L, pl.nblocks, s));
      TLS_CHECK(launch_colsum(b.partial, pl.ngroups, p + 1, b.g, &b.rst->done, s));
      TLS_CHECK(launch_refine_outer(pl.lgn, p, b.rst, b.g, b.M, b.Mt, b.phi, b.phib, b.cw, b.cres,
                                    b.cd, b.Vhat32, ctx->tw, s));
      for (int it = 0; it < inner_max; it += INNER_CHUNK) {
        for (int k = it; k < std::min(inner_max, it + INNER_CHUNK); ++k) {
          if (o.profile) {
            TLS_CHECK(pass_events(ctx, npass, &ea, &eb));
            TLS_CHECK(hipEventRecord(ea, s));
          }
          TLS_CHECK(launch_toep(PREC_F32, pl.lgn, MODE_FUSED, b.Yhat, b.Vhat32, nullptr, nullptr,
                                nullptr, b.partial, ctx->consts + 2, &b.rst->inner_done, ctx->tw,
                                pl.m, p, pl.L, pl.nblocks, s));
          if (o.profile) {
            TLS_CHECK(hipEventRecord(eb, s));
            ++npass;
          }
          TLS_CHECK(launch_colsum(b.partial, pl.ngroups, p + 1, b.g, &b.rst->inner_done, s));
          TLS_CHECK(launch_refine_cg(pl.lgn, p, b.rst, b.g, b.M, b.Mt, b.cw, b.cres, b.cd, b.phi,
                                     b.Vhat32, ctx->tw, s));
        }
        TLS_CHECK(hipMemcpyAsync(hr, b.rst, sizeof(RefineState), hipMemcpyDeviceToHost, s));
        TLS_CHECK(hipStreamSynchronize(s));
        if (hr->inner_done) break;
      }
      if (o.profile) {
        // the first `inner` passes of this outer step did work; later ones exited at once
        for (size_t i = first_pass; i < npass; ++i) {
          float t = 0.f;
          TLS_CHECK(hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]));
          all_ms += t;
        }
        worked_passes += static_cast<int>(std::min(npass - first_pass, static_cast<size_t>(hr->inner)));
      }
      if (hr->done) break;
    }
    TLS_CHECK(hipMemcpyAsync(hr, b.rst, sizeof(RefineState), hipMemcpyDeviceToHost, s));
    TLS_CHECK(hipStreamSynchronize(s));
    const RefineState rs = *hr;
    total_iters = rs.total_inner;
    refine = rs.outer;
    lsqr_rnorm = rs.rnorm;
    lsqr_arnorm = rs.hnorm;
    istop = rs.stop == 1 ? 2 : 0;
    bool finish_timed = false;
    if (rs.stop == 5 || rs.stop == 7) {
      hipLaunchKernelGGL(copy_vec_kernel, dim3((p + 255) / 256), dim3(256), 0, s, b.phib, p, b.phi0);
      TLS_CHECK(hipGetLastError());
      // profile: times the FP64 passes into pass_ms / pass_count / pass_worked
      const tls_status e = lsqr_run(PREC_F64, b.Yhat64, o.profile != 0);
      if (e != TLS_OK) return e;
      finish_timed = o.profile != 0;
      total_iters += ho->st.iter;
      istop = ho->st.istop;
      lsqr_rnorm = ho->st.rnorm;
      lsqr_arnorm = ho->st.arnorm;
    }
    if (o.profile && (!finish_timed || all_ms >= pass_ms)) {
      // the FP32 passes took more device time than the FP64 finish (or it did not run)
      pass_ms = all_ms;
      pass_count = static_cast<int>(npass);
      pass_worked = worked_passes;
      pass_kind = 1;
    }
  }

  // FP64 residual of the returned coefficients, row by row.
  TLS_CHECK(launch_resid_direct(d_y, pl.m, p, b.phi, b.rpart, s));
  TLS_CHECK(launch_colsum(b.rpart, resid_direct_blocks(pl.m), 1, b.rr, nullptr, s));
  // the results packed straight into pinned host memory (one kernel, no copy)
  hipLaunchKernelGGL(pack_results_kernel, dim3(1), dim3(256), 0, s, b.phi, p, b.rr, b.dminmax,
                     b.status, hphi);
  TLS_CHECK(hipGetLastError());
  TLS_CHECK(hipStreamSynchronize(s));

  memcpy(coef, hphi, p * sizeof(double));
  ho->rr[0] = hphi[p];
  ho->dminmax[0] = hphi[p + 1];
  ho->dminmax[1] = hphi[p + 2];
  for (int k = 0; k < 4; ++k) ho->status[k] = static_cast<int>(hphi[p + 3 + k]);
  const auto t1 = std::chrono::steady_clock::now();
  if (res) {
    memset(res, 0, sizeof(*res));
    res->resid_norm = sqrt(ho->rr[0]);
    res->kappa_est = ho->dminmax[1] > 0 ? ho->dminmax[0] / ho->dminmax[1] : INFINITY;
    res->lsqr_rnorm = lsqr_rnorm;
    res->lsqr_arnorm = lsqr_arnorm;
    res->iters = total_iters;
    res->istop = istop;
    res->refine_steps = refine;
    res->sketch_rows = pl.c;
    res->block_len = pl.B;
    res->n_blocks = pl.nblocks;
    res->pass_ms = pass_ms;
    res->pass_count = pass_count;
    res->pass_worked = pass_worked;
    res->pass_kind = pass_kind;
    res->mixed_path = mixed_path;
    res->t_total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  // a non-finite coefficient from finite data is a numerical breakdown
  for (int i = 0; i < p; ++i)
    if (!isfinite(coef[i])) return TLS_ERANK;
  if ((ho->status[0] & 6) || (ho->status[1] & 4) || istop == 4) return TLS_ERANK;
  if (istop == 7) return TLS_ENOCONV;
  if (istop == 5) return TLS_ESTALL;
  return TLS_OK;
}

namespace {

// Fixed scratch memory of the allocation-free pass (tls_op_toeplitz_noalloc):
// one copy per device, held until the process ends and shared by every such
// call on that device.  Host code never uses this name as an address: the
// device address of each device's copy is looked up once (scratch_init) and
// kept in g_scratch.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t{16} << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// With `device` current: the device address of its scratch copy.
hipError_t scratch_init(int device, void** out) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = ptr;
  }
  *out = g_scratch[device];
  return hipSuccess;
}

// Scratch of one tls_op_toeplitz call: v, (s1, s2), v's packed spectrum and
// the (p + 1) x groups block partials, 256-byte aligned slices from `base`.
struct ToepScratch {
  double* v;
  double* coef;
  void* Vh;
  double* part;
};
size_t toep_scratch(int p, int B, int groups, char* base, ToepScratch* t) {
  Arena a;
  a.base = base;
  t->v = a.take<double>(p);
  t->coef = a.take<double>(2);
  t->Vh = a.take<char>(static_cast<size_t>(B / 2) * 16);
  t->part = a.take<double>(static_cast<size_t>(p + 1) * groups);
  return a.need;
}

// The pass of tls_op_toeplitz with its scratch at `base`.
tls_status toep_op(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n, int32_t p, int32_t B,
                   const double* v, double s1, double s2, const void* d_w, void* d_e,
                   const void* d_u_in, int32_t want_rmv, double* d_out, hipStream_t s,
                   const ToepScratch& t, int nb, int ng) {
  const int pr = prec == TLS_PREC_F64 ? PREC_F64 : PREC_F32;
  const int lgn = ilog2(B) - 1;
  int mode = MODE_RMV;
  if (v) {
    const double cf[2] = {s1, s2};
    TLS_CHECK(hipMemcpyAsync(t.v, v, p * sizeof(double), hipMemcpyHostToDevice, s));
    TLS_CHECK(hipMemcpyAsync(t.coef, cf, sizeof(cf), hipMemcpyHostToDevice, s));
    TLS_CHECK(launch_small_rfft(pr, lgn, t.v, p, p, 1, 1.0 / B, t.Vh, ctx->tw, nullptr, s));
    mode = want_rmv ? MODE_FUSED : MODE_MV;
  }
  TLS_CHECK(launch_toep(pr, lgn, mode, d_spec, t.Vh, d_w, d_e, d_u_in, t.part, t.coef, nullptr,
                        ctx->tw, n - p, p, B - p + 1, nb, s));
  if (mode & PM_RMV) {
    TLS_CHECK(launch_colsum(t.part, ng, p + 1, d_out, nullptr, s));
  } else {
    TLS_CHECK(launch_colsum(t.part + static_cast<size_t>(p) * ng, ng, 1, d_out + p, nullptr, s));
  }
  // the host copies above read pageable memory; finish before returning
  TLS_CHECK(hipStreamSynchronize(s));
  return TLS_OK;
}

tls_ctx* g_default = nullptr;
std::mutex g_default_mu;

const tls_options& eff_opt(tls_ctx* c, const tls_options* o) { return o ? *o : c->opt; }

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char* tls_status_string(tls_status s) {
  switch (s) {
    case TLS_OK: return "ok";
    case TLS_EINVAL: return "invalid argument";
    case TLS_ERANK: return "numerically rank-deficient lag matrix";
    case TLS_ENOCONV: return "iteration limit reached";
    case TLS_ENOMEM: return "device allocation failed";
    case TLS_EDEVICE: return "HIP runtime error";
    case TLS_EUNSUPPORTED: return "size outside the supported range";
    case TLS_EAGAIN: return "request not finished yet";
    case TLS_ESTALL: return "iteration stalled at the working precision before tol";
    default: return "unknown status";
  }
}

void tls_options_default(tls_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = TLS_PREC_F64;
  o->sketch = TLS_SKETCH_LEVERAGE;
  o->jl_kind = TLS_JL_SRHT;
  o->gamma = 8;
  o->jl_k = 8;
  o->max_iter = 1000;
  o->block_lg = 0;
  o->warm_start = 1;
  o->max_refine = 0;
  o->seed = 0;
  o->request_id = 0;
}

tls_status tls_create(tls_ctx** out, int device, const tls_options* opt) {
  if (!out) return TLS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TLS_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TLS_EDEVICE;
  tls_ctx* c = new tls_ctx();
  c->device = device;
  if (opt)
    c->opt = *opt;
  else
    tls_options_default(&c->opt);
  hipError_t e = hipStreamCreate(&c->stream);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&c->chunk_ev[k], hipEventDisableTiming);
  if (e == hipSuccess) e = build_twiddles(c);
  if (e == hipSuccess) e = scratch_init(device, &c->scratch);
  if (e != hipSuccess) {
    tls_destroy(c);
    return hip_status(e);
  }
  *out = c;
  return TLS_OK;
}

void tls_destroy(tls_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  for (int w = 0; w < BATCH_STREAMS; ++w) {
    if (c->bstream[w]) {
      hipStreamSynchronize(c->bstream[w]);
      hipStreamDestroy(c->bstream[w]);
    }
    if (c->bdone[w]) hipEventDestroy(c->bdone[w]);
    for (hipEvent_t e : c->bevents[w]) hipEventDestroy(e);
  }
  if (c->bready) hipEventDestroy(c->bready);
  if (c->ws) hipFree(c->ws);
  if (c->pinned) hipHostFree(c->pinned);
  if (c->tw64) hipFree(c->tw64);
  if (c->tw32) hipFree(c->tw32);
  if (c->consts) hipFree(c->consts);
  for (hipEvent_t e : c->events) hipEventDestroy(e);
  for (hipEvent_t e : c->chunk_ev)
    if (e) hipEventDestroy(e);
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
}

tls_status tls_fit_ex(tls_ctx* ctx, const double* series, int64_t n, int32_t p, double tol,
                      const tls_options* opt, double* coef, tls_result* out) {
  if (!ctx || !series || !coef) return TLS_EINVAL;
  const tls_options& o = eff_opt(ctx, opt);
  tls_status st = validate(n, p, tol, o);
  if (st != TLS_OK) return st;
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(series[i])) return TLS_EINVAL;
  Plan pl;
  st = make_plan(n, p, o, &pl, ctx);
  if (st != TLS_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return TLS_EDEVICE;
  return run_fit(ctx, pl, o, nullptr, series, tol, ctx->stream, coef, out);
}

tls_status tls_fit_device(tls_ctx* ctx, const double* d_series, int64_t n, int32_t p, double tol,
                          const tls_options* opt, void* stream, double* coef, tls_result* out) {
  if (!ctx || !d_series || !coef) return TLS_EINVAL;
  const tls_options& o = eff_opt(ctx, opt);
  tls_status st = validate(n, p, tol, o);
  if (st != TLS_OK) return st;
  Plan pl;
  st = make_plan(n, p, o, &pl, ctx);
  if (st != TLS_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return TLS_EDEVICE;
  return run_fit(ctx, pl, o, d_series, nullptr, tol, pick_stream(ctx, stream), coef, out);
}

tls_status tls_fit(const double* series, int64_t n, int32_t p, double tol, double* coef,
                   double* resid_norm, int32_t* iters) {
  if (!series || !coef) return TLS_EINVAL;
  {
    tls_options d;
    tls_options_default(&d);
    const tls_status v = validate(n, p, tol, d);
    if (v != TLS_OK) return v;
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(series[i])) return TLS_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default) {
      tls_status st = tls_create(&g_default, 0, nullptr);
      if (st != TLS_OK) return st;
    }
  }
  tls_result r;
  tls_status st = tls_fit_ex(g_default, series, n, p, tol, nullptr, coef, &r);
  if (st == TLS_OK || st == TLS_ENOCONV || st == TLS_ESTALL || st == TLS_ERANK) {
    if (resid_norm) *resid_norm = r.resid_norm;
    if (iters) *iters = r.iters;
  }
  return st;
}

tls_status tls_fit_batch(tls_ctx* ctx, int32_t count, const double* const* series, const int64_t* n,
                         const int32_t* p, double tol, const tls_options* opt, double* coef_packed,
                         const int64_t* coef_offset, double* resid_norm, int32_t* iters,
                         tls_status* per_fit_status) {
  if (!ctx || count < 0 || (count > 0 && (!series || !n || !p || !coef_packed || !coef_offset)))
    return TLS_EINVAL;
  hipSetDevice(ctx->device);
  std::vector<tls_result> r(static_cast<size_t>(count));
  std::vector<tls_status> fs(static_cast<size_t>(count), TLS_OK);
  const tls_status first = run_batch(ctx, count, series, nullptr, n, p, tol, eff_opt(ctx, opt),
                                     ctx->stream, coef_packed, coef_offset, r.data(), fs.data());
  for (int32_t i = 0; i < count; ++i) {
    if (per_fit_status) per_fit_status[i] = fs[i];
    if (fs[i] == TLS_OK || fs[i] == TLS_ENOCONV || fs[i] == TLS_ESTALL || fs[i] == TLS_ERANK) {
      if (resid_norm) resid_norm[i] = r[i].resid_norm;
      if (iters) iters[i] = r[i].iters;
    }
  }
  return first;
}

tls_status tls_fit_batch_device(tls_ctx* ctx, int32_t count, const double* const* d_series,
                                const int64_t* n, const int32_t* p, double tol,
                                const tls_options* opt, void* stream, double* coef_packed,
                                const int64_t* coef_offset, tls_result* out,
                                tls_status* per_fit_status) {
  if (!ctx || count < 0 || (count > 0 && (!d_series || !n || !p || !coef_packed || !coef_offset)))
    return TLS_EINVAL;
  hipSetDevice(ctx->device);
  std::vector<tls_status> fs(static_cast<size_t>(count), TLS_OK);
  const tls_status first = run_batch(ctx, count, nullptr, d_series, n, p, tol, eff_opt(ctx, opt),
                                     pick_stream(ctx, stream), coef_packed, coef_offset, out,
                                     fs.data());
  if (per_fit_status)
    for (int32_t i = 0; i < count; ++i) per_fit_status[i] = fs[i];
  return first;
}

tls_status tls_pacf_device(tls_ctx* ctx, const double* d_series, int64_t n, int32_t pmax,
                           double tol, const tls_options* opt, void* stream, double* pacf,
                           int32_t* order, tls_status* lag_status) {
  if (!ctx || !d_series || !pacf || pmax < 1) return TLS_EINVAL;
  if (n < 2 * static_cast<int64_t>(pmax) + 1) return TLS_EINVAL;
  if (pmax > P_MAX) return TLS_EUNSUPPORTED;
  hipSetDevice(ctx->device);
  // lag h: the AR(h) fit on the prefix of n - pmax + h samples (n - pmax rows each)
  std::vector<const double*> ptr(pmax, d_series);
  std::vector<int64_t> nh(pmax), off(pmax);
  std::vector<int32_t> ph(pmax);
  int64_t total = 0;
  for (int32_t h = 1; h <= pmax; ++h) {
    nh[h - 1] = n - pmax + h;
    ph[h - 1] = h;
    off[h - 1] = total;
    total += h;
  }
  std::vector<double> coef(static_cast<size_t>(total));
  std::vector<tls_result> res(pmax);
  std::vector<tls_status> fs(pmax, TLS_OK);
  const tls_options& o = eff_opt(ctx, opt);
  const tls_status first = run_batch(ctx, pmax, nullptr, ptr.data(), nh.data(), ph.data(), tol, o,
                                     pick_stream(ctx, stream), coef.data(), off.data(), res.data(),
                                     fs.data());
  const bool compressed = o.estimator == TLS_EST_SKETCH;
  int32_t best = 0;
  for (int32_t h = 1; h <= pmax; ++h) {
    const double tau = coef[static_cast<size_t>(off[h - 1] + h - 1)];
    pacf[h - 1] = tau;
    if (lag_status) lag_status[h - 1] = fs[h - 1];
    // 95% band of a zero PACF over the rows the lag-h estimate used
    const double rows = compressed ? res[h - 1].sketch_rows : static_cast<double>(n - pmax);
    // a stalled fit (TLS_ESTALL) holds the best iterate at working precision
    const bool usable = fs[h - 1] == TLS_OK || fs[h - 1] == TLS_ESTALL;
    if (usable && rows > 0 && fabs(tau) >= 1.96 / sqrt(rows)) best = h;
  }
  if (order) *order = best;
  return first;
}

// ---- step-level entry points -----------------------------------------------

int64_t tls_num_blocks(int64_t n, int32_t p, int32_t B) {
  if (p < 1 || B < 128 || B > BMAX || (B & (B - 1)) || B < 2 * p || n <= p) return -1;
  const int64_t L = B - p + 1;
  return (n - p + L - 1) / L;
}

tls_status tls_op_spectra(tls_ctx* ctx, int32_t prec, const double* d_y, int64_t n, int32_t p,
                          int32_t B, void* d_spec, void* stream) {
  if (!ctx || !d_y || !d_spec) return TLS_EINVAL;
  const int64_t nb = tls_num_blocks(n, p, B);
  if (nb < 1) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  TLS_CHECK(launch_spectra(prec == TLS_PREC_F64 ? PREC_F64 : PREC_F32, ilog2(B) - 1, d_y, n,
                           B - p + 1, static_cast<int>(nb), d_spec, ctx->tw, pick_stream(ctx, stream)));
  return TLS_OK;
}

tls_status tls_op_toeplitz(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n, int32_t p,
                           int32_t B, const double* v, double s1, double s2, const void* d_w,
                           void* d_e, const void* d_u_in, int32_t want_rmv, double* d_out,
                           void* stream) {
  if (!ctx || !d_spec || !d_out) return TLS_EINVAL;
  if (!v && (!d_u_in || !want_rmv)) return TLS_EINVAL;
  const int64_t nb64 = tls_num_blocks(n, p, B);
  if (nb64 < 1) return TLS_EINVAL;
  const int nb = static_cast<int>(nb64);
  const int ng = pass_groups(ilog2(B) - 1, nb);
  hipSetDevice(ctx->device);
  ToepScratch t{};
  TLS_CHECK(ensure_ws(ctx, toep_scratch(p, B, ng, nullptr, &t) + 256));
  toep_scratch(p, B, ng, static_cast<char*>(ctx->ws), &t);
  return toep_op(ctx, prec, d_spec, n, p, B, v, s1, s2, d_w, d_e, d_u_in, want_rmv, d_out,
                 pick_stream(ctx, stream), t, nb, ng);
}

tls_status tls_op_toeplitz_noalloc(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n,
                                   int32_t p, int32_t B, const double* v, double s1, double s2,
                                   const void* d_w, void* d_e, const void* d_u_in,
                                   int32_t want_rmv, double* d_out, void* stream) {
  if (!ctx || !d_spec || !d_out) return TLS_EINVAL;
  if (!v && (!d_u_in || !want_rmv)) return TLS_EINVAL;
  const int64_t nb64 = tls_num_blocks(n, p, B);
  if (nb64 < 1) return TLS_EINVAL;
  if (nb64 > (int64_t{1} << 30)) return TLS_EUNSUPPORTED;
  const int nb = static_cast<int>(nb64);
  const int ng = pass_groups(ilog2(B) - 1, nb);
  ToepScratch t{};
  if (toep_scratch(p, B, ng, nullptr, &t) > NOALLOC_SCRATCH_BYTES) return TLS_EUNSUPPORTED;
  if (!ctx->scratch) return TLS_EDEVICE;
  hipSetDevice(ctx->device);
  // every slice is written before it is read: nothing needs clearing
  toep_scratch(p, B, ng, static_cast<char*>(ctx->scratch), &t);
  return toep_op(ctx, prec, d_spec, n, p, B, v, s1, s2, d_w, d_e, d_u_in, want_rmv, d_out,
                 pick_stream(ctx, stream), t, nb, ng);
}

tls_status tls_op_scores(tls_ctx* ctx, int32_t prec, const void* d_spec, int64_t n, int32_t p,
                         int32_t B, const double* d_omega, int32_t k, void* d_scores, void* stream) {
  if (!ctx || !d_spec || !d_omega || !d_scores || k < 1) return TLS_EINVAL;
  const int64_t nb = tls_num_blocks(n, p, B);
  if (nb < 1) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  hipStream_t s = pick_stream(ctx, stream);
  const int pr = prec == TLS_PREC_F64 ? PREC_F64 : PREC_F32;
  const int lgn = ilog2(B) - 1;
  const size_t bytes = static_cast<size_t>(k) * (B / 2) * 16 + 256;
  TLS_CHECK(ensure_ws(ctx, bytes));
  TLS_CHECK(launch_small_rfft(pr, lgn, d_omega, p, p, k, 1.0 / B, ctx->ws, ctx->tw, nullptr, s));
  TLS_CHECK(launch_scores(pr, lgn, d_spec, ctx->ws, k, d_scores, ctx->tw, n - p, p, B - p + 1,
                          static_cast<int>(nb), s));
  return TLS_OK;
}

tls_status tls_op_rh_mask(tls_ctx* ctx, int32_t prec, void* d_scores, int64_t m, int32_t level,
                          uint64_t seed, uint32_t fit, void* stream) {
  if (!ctx || !d_scores || m < 1 || level < 0) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  TLS_CHECK(launch_rh_mask(prec == TLS_PREC_F64 ? PREC_F64 : PREC_F32, d_scores, m, level, seed,
                           fit, pick_stream(ctx, stream)));
  return TLS_OK;
}

tls_status tls_op_sample(tls_ctx* ctx, int32_t prec, const void* d_scores, int64_t m,
                         const double* d_u, int32_t c, uint64_t seed, uint32_t fit,
                         int64_t* d_idx, double* d_scale, void* stream) {
  if (!ctx || !d_scores || !d_idx || !d_scale || m < 1 || c < 1) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  TLS_CHECK(ensure_ws(ctx, sample_work_doubles(m) * sizeof(double) + 256));
  TLS_CHECK(launch_sample(prec == TLS_PREC_F64 ? PREC_F64 : PREC_F32, d_scores, m, d_u, c, d_idx,
                          d_scale, static_cast<double*>(ctx->ws), seed, fit,
                          pick_stream(ctx, stream)));
  return TLS_OK;
}

tls_status tls_op_gather(tls_ctx* ctx, const double* d_y, int64_t n, int32_t p, int32_t mode,
                         int64_t* d_idx, double* d_scale, int32_t c, int32_t crows, int32_t ldq,
                         double* d_A, uint64_t seed, uint32_t fit, void* stream) {
  if (!ctx || !d_y || !d_A || p < 1 || n < 2 * static_cast<int64_t>(p) + 1) return TLS_EINVAL;
  if (mode < 0 || mode > 2 || c < 1 || crows < c || ldq < p + 1) return TLS_EINVAL;
  if (mode == 0 && (!d_idx || !d_scale)) return TLS_EINVAL;
  if (mode == 2 && c != n - p) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  TLS_CHECK(launch_gather(d_y, n - p, p, mode, d_idx, d_scale, c, crows, ldq, d_A,
                          mode == 1 ? d_idx : nullptr, mode == 1 ? d_scale : nullptr, seed, fit,
                          pick_stream(ctx, stream)));
  return TLS_OK;
}

tls_status tls_op_qr(tls_ctx* ctx, double* d_A, int32_t crows, int32_t q, int32_t ldq, double* d_R,
                     int32_t* status_out, void* stream) {
  if (!ctx || !d_A || !d_R || q < 1 || crows % 16 || ldq % 16 || q > ldq || crows < 16)
    return TLS_EINVAL;
  hipSetDevice(ctx->device);
  hipStream_t s = pick_stream(ctx, stream);
  Arena a;
  a.take<double>(qr_scratch_doubles(crows, q, ldq));
  a.take<double>(static_cast<size_t>(q) * q);
  a.take<double>(static_cast<size_t>(q) * q);
  a.take<int>(4);
  TLS_CHECK(ensure_ws(ctx, a.need + 256));
  a.need = 0;
  a.base = static_cast<char*>(ctx->ws);
  double* G = a.take<double>(qr_scratch_doubles(crows, q, ldq));
  double* R1 = a.take<double>(static_cast<size_t>(q) * q);
  double* R2 = a.take<double>(static_cast<size_t>(q) * q);
  int* dst = a.take<int>(4);
  TLS_CHECK(hipMemsetAsync(dst, 0, 4 * sizeof(int), s));
  TLS_CHECK(launch_qr(d_A, crows, q, ldq, q, 3, d_R, G, R1, R2, dst, s));
  int hst[4];
  TLS_CHECK(hipMemcpyAsync(hst, dst, sizeof(hst), hipMemcpyDeviceToHost, s));
  TLS_CHECK(hipStreamSynchronize(s));
  if (status_out) *status_out = hst[0];
  return TLS_OK;
}

tls_status tls_op_triinv(tls_ctx* ctx, const double* d_R, int32_t q, int32_t p, double* d_M,
                         double* d_phi0, void* stream) {
  if (!ctx || !d_R || !d_M || p < 1 || q < p || (d_phi0 && q < p + 1)) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  hipStream_t s = pick_stream(ctx, stream);
  TLS_CHECK(ensure_ws(ctx, static_cast<size_t>(p) * p * sizeof(double) + 512));
  double* Mt = static_cast<double*>(ctx->ws);
  int* dst = reinterpret_cast<int*>(Mt + static_cast<size_t>(p) * p);
  TLS_CHECK(hipMemsetAsync(dst, 0, sizeof(int), s));
  TLS_CHECK(launch_triinv(d_R, q, p, d_M, Mt, d_phi0, dst, s));
  return TLS_OK;
}

tls_status tls_op_jl(tls_ctx* ctx, const double* d_R, int32_t q, int32_t p, int32_t k,
                     int32_t kind, uint64_t seed, uint32_t fit, double* d_Pi, double* d_omega,
                     void* stream) {
  if (!ctx || !d_R || !d_omega || p < 1 || q < p || k < 1 || (kind != 0 && kind != 1))
    return TLS_EINVAL;
  if (p > P_MAX) return TLS_EUNSUPPORTED;
  hipSetDevice(ctx->device);
  TLS_CHECK(launch_jl_solve(d_R, q, p, k, kind, d_Pi, d_omega, seed, fit, pick_stream(ctx, stream)));
  return TLS_OK;
}

tls_status tls_op_philox(tls_ctx* ctx, uint64_t seed, uint32_t rng_stream, uint32_t fit,
                         uint64_t start, int64_t count, double* d_out, void* stream) {
  if (!ctx || !d_out || count < 0) return TLS_EINVAL;
  hipSetDevice(ctx->device);
  TLS_CHECK(launch_philox_uniform(d_out, count, rng_stream, fit, seed, start,
                                  pick_stream(ctx, stream)));
  return TLS_OK;
}

}  // extern "C"
