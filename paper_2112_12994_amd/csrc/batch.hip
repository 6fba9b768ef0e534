// Batched execution: many independent AR(p) fits of different lengths and
// orders in one pass over the device.
//
// Every kernel of the single-fit path has a batched twin that maps its
// workgroup index through a table of work items {fit, local index} to a
// per-fit descriptor (FitDesc), so one launch serves the blocks, rows, tiles
// or columns of all fits of a launch class.  A launch class groups the fits
// that share every compile-time choice the single-fit path makes for them
// (ClassKey); within a class each fit runs exactly the arithmetic of its
// single fit, so the result of fit i equals tls_fit_ex with request_id + i
// bit for bit.  Fits that finish early leave their later workgroups with
// nothing to do (each checks its fit's done flag first); device counters tell
// the host when a whole class has finished.
//
// The first part is the execution core shared with the server (server.hip);
// the second the batched driver behind tls_fit_batch*.
#include "engine.h"

#include <atomic>
#include <functional>
#include <map>
#include <thread>

namespace {

constexpr int B_CHUNK_ITERS = 8;
constexpr int B_INNER_CHUNK = 6;

__global__ void init_b_kernel(const Item* fits, int nfits, FitDesc* D, int max_iter,
                              int max_refine, int inner_max, double inner_tol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nfits) return;
  const FitDesc& d = D[fits[k].fit];
  LsqrState s{};
  s.tol = d.tol;
  s.max_iter = max_iter;
  s.coef[0] = -1.0;
  s.coef[1] = 1.0;
  *d.st = s;
  RefineState r{};
  r.tol = d.tol;
  r.max_refine = max_refine;
  r.inner_max = inner_max;
  r.inner_tol = inner_tol;
  *d.rst = r;
  d.status[0] = d.status[1] = d.status[2] = d.status[3] = 0;
}

// After the final QR: zero phi0 for a cold start; the mixed refinement starts
// from phi = phi0.
__global__ void post_qr_b_kernel(const Item* fits, const FitDesc* D, int warm, int mixed) {
  const FitDesc& d = D[fits[blockIdx.x].fit];
  for (int i = threadIdx.x; i < d.p; i += blockDim.x) {
    const double v = warm ? d.phi0[i] : 0.0;
    if (!warm) d.phi0[i] = 0.0;
    if (mixed) d.phi[i] = v;
  }
}

// Mixed precision: fits whose refinement stopped without converging (stop 5
// or 7), and the fits set to FP64 LSQR by the dispatch (stop 5, phib = phi0),
// run FP64 LSQR from their best iterate; the others are marked done and
// counted.
__global__ void fallback_prep_b_kernel(const Item* fits, const FitDesc* D, int* counts) {
  const FitDesc& d = D[fits[blockIdx.x].fit];
  const int stop = d.rst->stop;
  if (stop == 5 || stop == 7) {
    for (int i = threadIdx.x; i < d.p; i += blockDim.x) d.phi0[i] = d.phib[i];
    if (threadIdx.x == 0) d.st->done = 0;
  } else if (threadIdx.x == 0) {
    d.st->done = 1;
    atomicAdd(counts, 1);
  }
}

__global__ void zero_ints_kernel(int* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

// The compressed estimator (eq. (OLSc)): phi = phi0 from the final QR, no
// LSQR iterations; the fit is counted as finished (and appended to
// done_list when given).
__global__ void compressed_b_kernel(const Item* __restrict__ fits, const FitDesc* __restrict__ D,
                                    int* __restrict__ counts, int* __restrict__ done_list) {
  const int f = fits[blockIdx.x].fit;
  const FitDesc& d = D[f];
  for (int i = threadIdx.x; i < d.p; i += blockDim.x) d.phi[i] = d.phi0[i];
  if (threadIdx.x == 0) {
    d.st->done = 1;
    atomicAdd(counts, 1);
    if (done_list) done_list[atomicAdd(counts + 2, 1)] = f;
  }
}

// flags[k] = 1 when the k-th listed fit has finished (which 0: its LSQR,
// 1: its mixed-precision refinement).
__global__ void done_flags_b_kernel(const Item* __restrict__ fits, int nfits,
                                    const FitDesc* __restrict__ D, int which,
                                    int* __restrict__ flags) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nfits) return;
  const FitDesc& d = D[fits[k].fit];
  flags[k] = (which == 0 ? d.st->done : (which == 1 ? d.rst->done : d.st->f32)) ? 1 : 0;
}

__global__ void collect_b_kernel(const Item* __restrict__ items, const FitDesc* __restrict__ D,
                                 int mixed, double* __restrict__ coef, FitRec* __restrict__ rec) {
  const Item it = items[blockIdx.x];
  const FitDesc& d = D[it.fit];
  for (int i = threadIdx.x; i < d.p; i += blockDim.x) coef[it.idx + i] = d.phi[i];
  if (threadIdx.x == 0) {
    FitRec r{};
    r.rr = d.rr[0];
    r.dmax = d.dminmax[0];
    r.dmin = d.dminmax[1];
    for (int k = 0; k < 4; ++k) r.status[k] = d.status[k];
    r.path = mixed ? d.rst->path : 0;
    if (mixed && d.rst->path == MP_REFINE) {
      const RefineState& s = *d.rst;
      r.rnorm = s.rnorm;
      r.arnorm = s.hnorm;
      r.iters = s.total_inner;
      r.refine = s.outer;
      r.istop = s.stop == 1 ? 2 : 0;
      if (s.stop == 5 || s.stop == 7) {  // finished by FP64 LSQR
        r.rnorm = d.st->rnorm;
        r.arnorm = d.st->arnorm;
        r.iters += d.st->iter;
        r.istop = d.st->istop;
      }
    } else {
      const LsqrState& s = *d.st;
      r.rnorm = s.rnorm;
      r.arnorm = s.arnorm;
      r.iters = s.iter;
      r.istop = s.istop;
    }
    rec[blockIdx.x] = r;
  }
}

template <typename F>
List add_items(std::vector<Item>& all, const std::vector<int>& desc,
               const std::vector<const Plan*>& plans, F&& per_fit) {
  List l;
  l.off = static_cast<int>(all.size());
  for (size_t j = 0; j < desc.size(); ++j) {
    const int cnt = per_fit(*plans[j]);
    for (int i = 0; i < cnt; ++i) all.push_back({desc[j], i});
  }
  l.n = static_cast<int>(all.size()) - l.off;
  return l;
}

}  // namespace

// ---- execution core -----------------------------------------------------------

// Register-tile counts of a launch class, rounded up to 4 or 8 tiles of 16
// (orders up to 64 and 128) and to 7 tiles of 32 (up to 224), so that a
// batch or a served tick holds few set-up classes: each class is a chain of
// small dependent kernels, and at 5000 requests/s of orders 2..200 the
// served latency went from p50 21 / p99 55 ms with exact counts to 13 / 35
// ms rounded to even counts and 9.3 / 25 ms with these.  A factorisation or
// inverse with more tiles than its order needs runs the same operations in
// the same order (the extra tiles hold zeros), so a fit's result does not
// depend on the class it lands in.
int class_tiles(int t) {
  if (t >= 1 && t <= 8) return t <= 4 ? 4 : 8;
  return t >= 105 ? 107 : t;
}

ClassKey class_key(const Plan& pl) {
  ClassKey k;
  k.lgn = pl.lgn;
  k.qt = class_tiles(reg_tiles(pl.q));
  k.pt = class_tiles(reg_tiles(pl.p));
  k.mlds = lsqr_step_lds(pl.lgn, pl.p) ? 1 : 0;
  return k;
}

ClassLists build_lists(std::vector<Item>& items, const std::vector<int>& desc,
                       const std::vector<const Plan*>& plans, bool lev) {
  ClassLists c;
  auto sampled = [lev](const Plan& q) { return lev && !q.all_rows; };
  c.blocks = add_items(items, desc, plans, [](const Plan& q) { return q.nblocks; });
  c.groups = add_items(items, desc, plans, [](const Plan& q) { return q.ngroups; });
  c.blocks1 = add_items(items, desc, plans, [&](const Plan& q) { return sampled(q) ? q.nblocks : 0; });
  c.rows1 = add_items(items, desc, plans, [](const Plan& q) { return q.crows; });
  c.rows2 = add_items(items, desc, plans, [&](const Plan& q) { return sampled(q) ? q.crows : 0; });
  c.tiles1 = add_items(items, desc, plans, [&](const Plan& q) {
    return sampled(q) ? (q.ldq / 16) * (q.ldq / 16) : 0;
  });
  c.tiles2 = add_items(items, desc, plans, [](const Plan& q) { return (q.ldq / 16) * (q.ldq / 16); });
  c.rowtiles2 = add_items(items, desc, plans, [](const Plan& q) { return q.crows / 16; });
  c.trmm2 = add_items(items, desc, plans, [](const Plan& q) { return q.q; });
  c.fits = add_items(items, desc, plans, [](const Plan&) { return 1; });
  c.fits1 = add_items(items, desc, plans, [&](const Plan& q) { return sampled(q) ? 1 : 0; });
  c.jl = add_items(items, desc, plans, [&](const Plan& q) { return sampled(q) ? q.k : 0; });
  int pmax = 0;
  for (const Plan* q : plans) pmax = std::max(pmax, q->p);
  const int kc = jl_cols(pmax);  // as launch_jl_b picks for the class
  c.jlg = add_items(items, desc, plans, [&](const Plan& q) {
    return sampled(q) ? (q.k + kc - 1) / kc : 0;
  });
  c.chunks = add_items(items, desc, plans, [&](const Plan& q) {
    return sampled(q) ? static_cast<int>((sample_work_doubles(q.m) - 1) / 2) : 0;
  });
  c.draws = add_items(items, desc, plans, [&](const Plan& q) { return sampled(q) ? q.c : 0; });
  c.cols = add_items(items, desc, plans, [](const Plan& q) { return q.p + 1; });
  c.rblocks = add_items(items, desc, plans, [](const Plan& q) { return resid_direct_blocks(q.m); });
  return c;
}

void fill_desc(const Plan& pl, const FitBufs& b, const double* y, uint32_t fit, double tol,
               FitDesc* d) {
  *d = FitDesc{};
  d->y = y;
  d->n = pl.n;
  d->m = pl.m;
  d->tol = tol;
  d->p = pl.p;
  d->q = pl.q;
  d->ldq = pl.ldq;
  d->c = pl.c;
  d->crows = pl.crows;
  d->k = pl.k;
  d->L = pl.L;
  d->nblocks = pl.nblocks;
  d->ngroups = pl.ngroups;
  d->nchunks = static_cast<int>((sample_work_doubles(pl.m) - 1) / 2);
  d->all_rows = pl.all_rows;
  d->fit = fit;
  d->Yhat = b.Yhat;
  d->Yhat64 = b.Yhat64;
  d->u = b.u;
  d->partial = b.partial;
  d->g = b.g;
  d->A = b.A;
  d->G = b.G;
  d->R1 = b.R1;
  d->R2 = b.R2;
  d->R = b.R;
  d->M = b.M;
  d->Mt = b.Mt;
  d->Pi = b.Pi;
  d->Om = b.Om;
  d->Omhat = b.Omhat;
  d->Vhat = b.Vhat;
  d->Vhat32 = b.Vhat32;
  d->v = b.v;
  d->w = b.w;
  d->z = b.z;
  d->phi0 = b.phi0;
  d->phi = b.phi;
  d->phib = b.phib;
  d->idx = b.idx;
  d->scale = b.scale;
  d->swork = b.swork;
  d->st = b.st;
  d->rst = b.rst;
  d->status = b.status;
  d->rpart = b.rpart;
  d->rr = b.rr;
  d->dminmax = b.dminmax;
  d->cw = b.cw;
  d->cres = b.cres;
  d->cd = b.cd;
}

hipError_t batch_init(const Item* fits, int nfits, FitDesc* D, int max_iter, int max_refine,
                      int inner_max, double inner_tol, hipStream_t s) {
  if (nfits < 1) return hipSuccess;
  hipLaunchKernelGGL(init_b_kernel, dim3((nfits + 63) / 64), dim3(64), 0, s, fits, nfits, D,
                     max_iter, max_refine, inner_max, inner_tol);
  return hipGetLastError();
}

hipError_t batch_zero_ints(int* x, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 63) / 64), dim3(64), 0, s, x, n);
  return hipGetLastError();
}

hipError_t PassTimer::begin(hipStream_t s) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = pool_events(*pool, n, &a, &b);
  return e == hipSuccess ? hipEventRecord(a, s) : e;
}

hipError_t PassTimer::end(hipStream_t s) {
  hipEvent_t b = (*pool)[2 * n + 1];
  ++n;
  return hipEventRecord(b, s);
}

hipError_t PassTimer::total_ms(double* ms) const {
  double t = 0.0;
  for (size_t k = 0; k < n; ++k) {
    float x = 0.f;
    hipError_t e = hipEventElapsedTime(&x, (*pool)[2 * k], (*pool)[2 * k + 1]);
    if (e != hipSuccess) return e;
    t += x;
  }
  *ms = t;
  return hipSuccess;
}

#define L_(lst) I + l.lst.off, l.lst.n

namespace {

// A fixed sequence of launches on one stream, captured as a HIP graph on
// first use and replayed afterwards (or launched directly when use = false).
// The sequences captured here hold kernel launches only.
struct GraphSlot {
  hipGraphExec_t exec = nullptr;
};

tls_status run_graph(GraphSlot& g, bool use, hipStream_t s,
                     const std::function<tls_status()>& body) {
  if (!use) return body();
  if (!g.exec) {
    TLS_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const tls_status e = body();
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (e != TLS_OK || ec != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return e != TLS_OK ? e : hip_status(ec);
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      return hip_status(ei);
    }
  }
  TLS_CHECK(hipGraphLaunch(g.exec, s));
  return TLS_OK;
}

}  // namespace

tls_status setup_class(tls_ctx* ctx, const ClassKey& k, int pmax, int ldqmax, const Item* I,
                       const ClassLists& l, FitDesc* D, const tls_options& o, hipStream_t s) {
  const bool mixed = o.precision == TLS_PREC_MIXED;
  const int cprec = mixed ? PREC_F32 : PREC_F64;
  const uint64_t seed = o.seed;
  // spectra of the series blocks (mixed: FP32 for the products of the fits
  // that take them, FP64 for the scores, the residuals and the others)
  TLS_CHECK(launch_spectra_b(cprec, k.lgn, L_(blocks), D, 0, ctx->tw, s));
  if (mixed) TLS_CHECK(launch_spectra_b(PREC_F64, k.lgn, L_(blocks), D, 1, ctx->tw, s));
  // sketch -> R
  TLS_CHECK(launch_gather_b(1, L_(rows1), D, seed, s));
  if (l.fits1.n > 0) {
    TLS_CHECK(launch_qr_b(1, k.qt, L_(tiles1), nullptr, 0, nullptr, 0, L_(fits1), ldqmax, D, s));
    TLS_CHECK(launch_jl_b(L_(jlg), D, o.jl_kind, pmax, seed, s));
    // the scores and the draw in FP64 in every precision
    TLS_CHECK(launch_small_rfft_b(PREC_F64, k.lgn, 0, L_(jl), D, ctx->tw, s));
    TLS_CHECK(launch_scores_b(PREC_F64, k.lgn, L_(blocks1), D, ctx->tw, s));
    TLS_CHECK(launch_sample_b(PREC_F64, L_(chunks), L_(draws), L_(fits1), D, seed, s));
    TLS_CHECK(launch_gather_b(2, L_(rows2), D, seed, s));
  }
  TLS_CHECK(launch_qr_b(2, k.qt, L_(tiles2), L_(rowtiles2), L_(trmm2), L_(fits), ldqmax, D, s));
  TLS_CHECK(launch_triinv_b(k.pt, L_(fits), pmax, D, s));
  if (l.fits.n > 0) {
    hipLaunchKernelGGL(post_qr_b_kernel, dim3(l.fits.n), dim3(64), 0, s, I + l.fits.off, D,
                       o.warm_start || o.estimator == TLS_EST_SKETCH ? 1 : 0, mixed ? 1 : 0);
    TLS_CHECK(hipGetLastError());
  }
  return TLS_OK;
}

tls_status lsqr_step_class(tls_ctx* ctx, int lgn, int pmax, bool mlds, bool first,
                           int precs, const Item* groups, int ngroups, const Item* cols, int ncols,
                           const Item* fits, int nfits, FitDesc* D, int* counts, int* done_list,
                           PassTimer* tm, hipStream_t s, const Item* groups32, int ngroups32,
                           const Item* fits32, int nfits32) {
  // FP32 products: FP32 spectra, u and v's spectrum in FP32 (LsqrState::f32)
  const bool p64 = (precs & 1) != 0, p32 = (precs & 2) != 0;
  if (!groups32) {
    groups32 = groups;
    ngroups32 = ngroups;
    fits32 = fits;
    nfits32 = nfits;
  }
  if (first && p64) TLS_CHECK(launch_small_rfft_b(PREC_F64, lgn, 1, fits, nfits, D, ctx->tw, s));
  if (first && p32)
    TLS_CHECK(launch_small_rfft_b(PREC_F32, lgn, 1, fits32, nfits32, D, ctx->tw, s));
  if (tm) TLS_CHECK(tm->begin(s));
  if (p64 && ngroups > 0)
    TLS_CHECK(launch_toep_b(PREC_F64, lgn, first ? BP_LSQR_FIRST : BP_LSQR, groups, ngroups, D,
                            ctx->consts, ctx->tw, s));
  if (p32 && ngroups32 > 0)
    TLS_CHECK(launch_toep_b(PREC_F32, lgn, BP_LSQR32, groups32, ngroups32, D, ctx->consts, ctx->tw,
                            s));
  if (tm) TLS_CHECK(tm->end(s));
  TLS_CHECK(launch_colsum_b(0, cols, ncols, D, s));
  if (p64)
    TLS_CHECK(launch_lsqr_step_b(PREC_F64, lgn, fits, nfits, pmax, mlds, D, counts, done_list,
                                 ctx->tw, s));
  if (p32)
    TLS_CHECK(launch_lsqr_step_b(PREC_F32, lgn, fits32, nfits32, pmax, mlds, D, counts, done_list,
                                 ctx->tw, s));
  return TLS_OK;
}

tls_status residual_class(const Item* rblocks, int nrblocks, const Item* fits, int nfits, int pmax,
                          FitDesc* D, hipStream_t s) {
  TLS_CHECK(launch_resid_b(rblocks, nrblocks, D, pmax, s));
  TLS_CHECK(launch_colsum_b(3, fits, nfits, D, s));
  return TLS_OK;
}

hipError_t launch_compressed_b(const Item* fits, int nfits, const FitDesc* D, int* counts,
                               int* done_list, hipStream_t s) {
  if (nfits < 1) return hipSuccess;
  hipLaunchKernelGGL(compressed_b_kernel, dim3(nfits), dim3(64), 0, s, fits, D, counts, done_list);
  return hipGetLastError();
}

hipError_t launch_done_flags_b(const Item* fits, int nfits, const FitDesc* D, int which,
                               int* flags, hipStream_t s) {
  if (nfits < 1) return hipSuccess;
  hipLaunchKernelGGL(done_flags_b_kernel, dim3((nfits + 255) / 256), dim3(256), 0, s, fits, nfits, D,
                     which, flags);
  return hipGetLastError();
}

hipError_t collect_b(const Item* fits, int nfits, const FitDesc* D, int mixed, double* coef,
                     FitRec* rec, hipStream_t s) {
  if (nfits < 1) return hipSuccess;
  hipLaunchKernelGGL(collect_b_kernel, dim3(nfits), dim3(64), 0, s, fits, D, mixed, coef, rec);
  return hipGetLastError();
}

tls_status record_status(const FitRec& r, const double* coef, int p) {
  for (int k = 0; k < p; ++k)
    if (!isfinite(coef[k])) return TLS_ERANK;
  if ((r.status[0] & 6) || (r.status[1] & 4) || r.istop == 4) return TLS_ERANK;
  if (r.istop == 7) return TLS_ENOCONV;
  if (r.istop == 5) return TLS_ESTALL;
  return TLS_OK;
}

void record_result(const FitRec& r, const Plan& pl, double ms, tls_result* o) {
  memset(o, 0, sizeof(*o));
  o->resid_norm = sqrt(r.rr);
  o->kappa_est = r.dmin > 0 ? r.dmax / r.dmin : INFINITY;
  o->lsqr_rnorm = r.rnorm;
  o->lsqr_arnorm = r.arnorm;
  o->iters = r.iters;
  o->istop = r.istop;
  o->refine_steps = r.refine;
  o->mixed_path = r.path;
  o->sketch_rows = pl.c;
  o->block_len = pl.B;
  o->n_blocks = pl.nblocks;
  o->t_total_ms = ms;
}

// ---- batched driver -------------------------------------------------------------

tls_status run_batch(tls_ctx* ctx, int count, const double* const* host_series,
                     const double* const* dev_series, const int64_t* n, const int32_t* p,
                     double tol, const tls_options& o, hipStream_t s, double* coef_packed,
                     const int64_t* coef_offset, tls_result* res, tls_status* fit_status) {
  const auto t0 = std::chrono::steady_clock::now();
  const bool mixed = o.precision == TLS_PREC_MIXED;
  const bool copy_y = host_series != nullptr;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  const int max_refine = o.max_refine > 0 ? o.max_refine : 0;
  const int inner_max = std::min(max_iter, 25);

  std::vector<Plan> plans(count);
  std::vector<tls_status> st(count, TLS_OK);
  std::vector<int> singles;  // fits outside the batched kernels' limits
  std::map<ClassKey, std::vector<int>> groups;
  for (int i = 0; i < count; ++i) {
    if (copy_y ? !host_series[i] : !dev_series[i]) {
      st[i] = TLS_EINVAL;
      continue;
    }
    st[i] = validate(n[i], p[i], tol, o);
    if (st[i] == TLS_OK && copy_y)
      for (int64_t t = 0; t < n[i]; ++t)
        if (!isfinite(host_series[i][t])) {
          st[i] = TLS_EINVAL;
          break;
        }
    if (st[i] == TLS_OK) st[i] = make_plan(n[i], p[i], o, &plans[i], ctx);
    if (st[i] != TLS_OK) continue;
    // beyond the batched kernels' limits, or a repeated-halving sketch (its
    // level loop is in the single-fit driver): one fit at a time
    if (plans[i].ldq > BATCH_LDQ_MAX || o.sketch == TLS_SKETCH_RH) {
      singles.push_back(i);
      continue;
    }
    groups[class_key(plans[i])].push_back(i);
  }

  // Order the batched fits by class (descriptor j = position in `order`) and
  // build each class's item lists.
  struct Cls {
    ClassKey key;
    int first, count, pmax, ldqmax;
    ClassLists l;
  };
  std::vector<int> order;
  std::vector<Cls> classes;
  std::vector<Item> items;
  for (auto& kv : groups) {
    Cls c{kv.first, static_cast<int>(order.size()), static_cast<int>(kv.second.size()), 0, 0, {}};
    std::vector<int> desc;
    std::vector<const Plan*> pls;
    for (int i : kv.second) {
      desc.push_back(static_cast<int>(order.size()));
      pls.push_back(&plans[i]);
      order.push_back(i);
      c.pmax = std::max(c.pmax, plans[i].p);
      c.ldqmax = std::max(c.ldqmax, plans[i].ldq);
    }
    c.l = build_lists(items, desc, pls, o.sketch == TLS_SKETCH_LEVERAGE);
    classes.push_back(c);
  }
  const int nb = static_cast<int>(order.size());
  // collect list: every batched fit, idx = offset of its packed coefficients
  const int collect_off = static_cast<int>(items.size());
  int64_t coef_total = 0;
  for (int j = 0; j < nb; ++j) {
    items.push_back({j, static_cast<int>(coef_total)});
    coef_total += plans[order[j]].p;
  }
  if (coef_total > (int64_t{1} << 30)) return TLS_EUNSUPPORTED;

  // Workspace: per-fit buffers, then the descriptors, items, counters and outputs.
  size_t total = 0;
  auto reserve = [&total](size_t bytes) {
    const size_t at = (total + 255) & ~size_t{255};
    total = at + bytes;
    return at;
  };
  std::vector<size_t> fit_off(nb);
  for (int j = 0; j < nb; ++j) {
    FitBufs tmp{};
    fit_off[j] = reserve(carve(plans[order[j]], copy_y, &tmp, nullptr));
  }
  const size_t ncounts = 4 * std::max<size_t>(classes.size(), 1);
  const size_t off_D = reserve(sizeof(FitDesc) * std::max(nb, 1));
  const size_t off_items = reserve(sizeof(Item) * std::max<size_t>(items.size(), 1));
  const size_t off_items2 = reserve(sizeof(Item) * std::max<size_t>(items.size(), 1));
  const size_t off_flags = reserve(sizeof(int) * std::max(nb, 1));
  const size_t off_counts = reserve(sizeof(int) * ncounts);
  const size_t off_coef = reserve(sizeof(double) * std::max<int64_t>(coef_total, 1));
  const size_t off_rec = reserve(sizeof(FitRec) * std::max(nb, 1));
  if (nb > 0) TLS_CHECK(ensure_ws(ctx, total + 256));
  char* base = static_cast<char*>(ctx->ws);

  std::vector<FitDesc> desc(nb);
  std::vector<FitBufs> bufs(nb);
  for (int j = 0; j < nb; ++j) {
    const int i = order[j];
    carve(plans[i], copy_y, &bufs[j], base + fit_off[j]);
    const double* y = copy_y ? bufs[j].y : dev_series[i];
    if (copy_y)
      TLS_CHECK(hipMemcpyAsync(bufs[j].y, host_series[i], plans[i].n * sizeof(double),
                               hipMemcpyHostToDevice, s));
    fill_desc(plans[i], bufs[j], y, static_cast<uint32_t>(o.request_id + static_cast<uint64_t>(i)),
              tol, &desc[j]);
  }
  FitDesc* D = reinterpret_cast<FitDesc*>(base + off_D);
  Item* items2 = reinterpret_cast<Item*>(base + off_items2);  // compacted step lists
  int* dflags = reinterpret_cast<int*>(base + off_flags);
  const Item* I = reinterpret_cast<const Item*>(base + off_items);
  int* counts = reinterpret_cast<int*>(base + off_counts);
  double* dcoef = reinterpret_cast<double*>(base + off_coef);
  FitRec* drec = reinterpret_cast<FitRec*>(base + off_rec);
  // pinned: counters, the fit records, the packed coefficients
  const size_t host_bytes = 256 + sizeof(FitRec) * std::max(nb, 1) +
                            sizeof(double) * std::max<int64_t>(coef_total, 1);
  TLS_CHECK(ensure_pinned(ctx, host_bytes));
  int* hcounts = static_cast<int*>(ctx->pinned);
  FitRec* hrec = reinterpret_cast<FitRec*>(static_cast<char*>(ctx->pinned) + 256);
  double* hcoef = reinterpret_cast<double*>(hrec + std::max(nb, 1));

  if (nb > 0) {
    TLS_CHECK(hipMemcpyAsync(D, desc.data(), sizeof(FitDesc) * nb, hipMemcpyHostToDevice, s));
    TLS_CHECK(hipMemcpyAsync(base + off_items, items.data(), sizeof(Item) * items.size(),
                             hipMemcpyHostToDevice, s));
    TLS_CHECK(batch_init(I + collect_off, nb, D, max_iter, max_refine, inner_max, 1e-5, s));
    TLS_CHECK(batch_zero_ints(counts, static_cast<int>(ncounts), s));
  }
  // profile = 1: event pairs around every launch of the fused LSQR pass (in
  // mixed batches both product precisions' launches), one pool per class
  // stream; the classes then run one at a time, so that each launch's
  // duration is its own and not shared with another class's kernels
  const bool graphs = !o.no_graph && !o.profile;

  // One class from setup to residual on stream cs; hc: 4 pinned ints.
  auto run_class = [&](const Cls& c, hipStream_t cs, int* hc, PassTimer* tm) -> tls_status {
    const ClassLists& l = c.l;
    int* cnt = counts + 4 * (&c - classes.data());
    const hipStream_t s = cs;
    const tls_status e0 = setup_class(ctx, c.key, c.pmax, c.ldqmax, I, l, D, o, s);
    if (e0 != TLS_OK) return e0;
    if (o.estimator == TLS_EST_SKETCH) {
      TLS_CHECK(launch_compressed_b(L_(fits), D, cnt, nullptr, s));
      return residual_class(L_(rblocks), L_(fits), c.pmax, D, s);
    }
    GraphSlot g_lsqr, g_inner, g_inner_tail;
    auto drop_graphs = [&]() {
      for (GraphSlot* g : {&g_lsqr, &g_inner, &g_inner_tail})
        if (g->exec) {
          hipGraphExecDestroy(g->exec);
          g->exec = nullptr;
        }
    };
    auto done = [&](tls_status e) {
      // the graphs' last launches finished at the host's final check
      drop_graphs();
      return e;
    };

    // The step lists (pass block groups, columns, fits) of the fits still iterating.
    // When at least half of a list's fits have finished, the lists are
    // rebuilt without them (in this class's region of the second item
    // buffer), so that the stragglers do not pay for launches over every
    // finished fit's blocks; the graphs are captured again.
    // With split set (mixed batches), groups / fits hold the FP64-product
    // fits and groups32 / fits32 the FP32-product ones (one list each per
    // launch, none of whose workgroups then exits for the other precision);
    // cols covers all of them.
    struct Lists {
      const Item *groups, *cols, *fits;
      int ngroups, ncols, nfits;
      std::vector<int> desc;  // descriptor index of each fit item, in list order
      const Item *groups32 = nullptr, *fits32 = nullptr;
      int ngroups32 = 0, nfits32 = 0;
    };
    auto full_lists = [&]() {
      Lists sl{I + l.groups.off, I + l.cols.off, I + l.fits.off, l.groups.n, l.cols.n, l.fits.n, {}};
      for (int j = 0; j < c.count; ++j) sl.desc.push_back(c.first + j);
      return sl;
    };
    std::vector<int> hflags;
    std::vector<char> is32;  // per fit of the class (index j - c.first) when split
    // which: 0 = LSQR finished (st->done), 1 = refinement finished (rst->done)
    auto compact = [&](Lists& sl, int which) -> tls_status {
      int* dfl = dflags + c.first;
      const int nlisted = static_cast<int>(sl.desc.size());
      // the listed fits in desc order (the split lists hold them FP64 first)
      TLS_CHECK(launch_done_flags_b(sl.fits, sl.nfits, D, which, dfl, s));
      if (sl.fits32 && sl.nfits32 > 0)
        TLS_CHECK(launch_done_flags_b(sl.fits32, sl.nfits32, D, which, dfl + sl.nfits, s));
      hflags.resize(nlisted);
      TLS_CHECK(hipMemcpyAsync(hflags.data(), dfl, nlisted * sizeof(int), hipMemcpyDeviceToHost, s));
      TLS_CHECK(hipStreamSynchronize(s));
      std::vector<Item> b2, c2, f2, b32, f32;
      std::vector<int> keep, keep32;
      for (int k = 0; k < nlisted; ++k) {
        if (hflags[k]) continue;
        const int j = sl.desc[k];
        const Plan& pl = plans[order[j]];
        const bool to32 = !is32.empty() && is32[j - c.first];
        for (int t = 0; t < pl.ngroups; ++t) (to32 ? b32 : b2).push_back({j, t});
        for (int t = 0; t <= pl.p; ++t) c2.push_back({j, t});
        (to32 ? f32 : f2).push_back({j, 0});
        (to32 ? keep32 : keep).push_back(j);
      }
      if (keep.empty() && keep32.empty()) return TLS_OK;
      const int n64g = static_cast<int>(b2.size()), n64f = static_cast<int>(f2.size());
      b2.insert(b2.end(), b32.begin(), b32.end());
      f2.insert(f2.end(), f32.begin(), f32.end());
      keep.insert(keep.end(), keep32.begin(), keep32.end());
      Item* base2 = items2;
      TLS_CHECK(hipMemcpyAsync(base2 + l.groups.off, b2.data(), b2.size() * sizeof(Item),
                               hipMemcpyHostToDevice, s));
      TLS_CHECK(hipMemcpyAsync(base2 + l.cols.off, c2.data(), c2.size() * sizeof(Item),
                               hipMemcpyHostToDevice, s));
      TLS_CHECK(hipMemcpyAsync(base2 + l.fits.off, f2.data(), f2.size() * sizeof(Item),
                               hipMemcpyHostToDevice, s));
      // the host vectors must outlive the copies
      TLS_CHECK(hipStreamSynchronize(s));
      const bool split = !is32.empty();
      sl = Lists{base2 + l.groups.off, base2 + l.cols.off, base2 + l.fits.off,
                 split ? n64g : static_cast<int>(b2.size()), static_cast<int>(c2.size()),
                 split ? n64f : static_cast<int>(f2.size()), keep};
      if (split) {
        sl.groups32 = base2 + l.groups.off + n64g;
        sl.ngroups32 = static_cast<int>(b2.size()) - n64g;
        sl.fits32 = base2 + l.fits.off + n64f;
        sl.nfits32 = static_cast<int>(f2.size()) - n64f;
      }
      drop_graphs();
      return TLS_OK;
    };
    auto worth_compacting = [](int remaining, int listed) {
      return listed >= 8 && remaining * 2 <= listed;
    };
#define SL_(lst) sl.lst, sl.n##lst

    // LSQR over the class (fits already done skip every step); cnt[0] holds
    // the number of finished fits, cnt[1] those with FP32 products.  precs:
    // bit 0 FP64 products, bit 1 FP32 products, both when the class holds
    // n32 FP32-product fits among others (each launch skips the fits of the
    // other precision); a precision whose fits have all finished is dropped
    // from the steps.  Every chunk after the first is the same sequence of
    // launches: a graph when enabled (captured again when precs changes).
    auto lsqr_any = [&](PassTimer* t, int precs, int n32) -> tls_status {
      Lists sl = full_lists();
      if (precs == 3) {
        // the lists split by product precision before the first step
        is32.assign(c.count, 0);
        TLS_CHECK(launch_done_flags_b(sl.fits, sl.nfits, D, 2, dflags + c.first, s));
        std::vector<int> f(sl.nfits);
        TLS_CHECK(hipMemcpyAsync(f.data(), dflags + c.first, sl.nfits * sizeof(int),
                                 hipMemcpyDeviceToHost, s));
        TLS_CHECK(hipStreamSynchronize(s));
        for (int k = 0; k < sl.nfits; ++k) is32[sl.desc[k] - c.first] = static_cast<char>(f[k]);
        const tls_status ec = compact(sl, 0);
        if (ec != TLS_OK) return ec;
      }
      for (int launched = 0;; launched += B_CHUNK_ITERS) {
        auto chunk = [&, launched]() -> tls_status {
          for (int it = 0; it < B_CHUNK_ITERS; ++it) {
            const tls_status e = lsqr_step_class(ctx, c.key.lgn, c.pmax, c.key.mlds != 0,
                                                 launched == 0 && it == 0, precs,
                                                 SL_(groups),
                                                 SL_(cols), SL_(fits), D, cnt, nullptr, t, s,
                                                 SL_(groups32), SL_(fits32));
            if (e != TLS_OK) return e;
          }
          return TLS_OK;
        };
        const tls_status e = run_graph(g_lsqr, graphs && launched > 0, s, chunk);
        if (e != TLS_OK) return e;
        TLS_CHECK(hipMemcpyAsync(hc, cnt, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
        TLS_CHECK(hipStreamSynchronize(s));
        if (hc[0] >= c.count || launched > max_iter) break;
        if (precs == 3) {
          const int left = (hc[1] >= n32 ? 2 : 0) | (hc[0] - hc[1] >= c.count - n32 ? 1 : 0);
          if (left) {
            precs &= ~left;
            drop_graphs();
          }
        }
        if (!t && worth_compacting(c.count - hc[0], sl.nfits + sl.nfits32)) {
          const tls_status ec = compact(sl, 0);
          if (ec != TLS_OK) return ec;
        }
      }
      return TLS_OK;
    };
    if (!mixed) {
      const tls_status e = lsqr_any(tm, 1, 0);
      if (e != TLS_OK) return done(e);
    } else if (max_refine == 0) {
      // each fit's path (mixed_path_of): FP32- and FP64-product LSQR in the
      // same steps
      if (hipError_t he = batch_zero_ints(cnt, 4, s)) return done(hip_status(he));
      hipLaunchKernelGGL(mixed_dispatch_b_kernel, dim3(l.fits.n), dim3(256), 0, s, I + l.fits.off,
                         D, 0, MIXED_TOL_F32, cnt, 0);
      if (hipError_t he = hipGetLastError()) return done(hip_status(he));
      hipLaunchKernelGGL(to_f32_b_kernel, dim3(l.blocks.n), dim3(256), 0, s, I + l.blocks.off, D);
      if (hipError_t he = hipGetLastError()) return done(hip_status(he));
      if (hipError_t he = hipMemcpyAsync(hc, cnt, 4 * sizeof(int), hipMemcpyDeviceToHost, s))
        return done(hip_status(he));
      if (hipError_t he = hipStreamSynchronize(s)) return done(hip_status(he));
      const int n32 = hc[3];
      if (hipError_t he = batch_zero_ints(cnt, 4, s)) return done(hip_status(he));
      const tls_status e =
          lsqr_any(tm, (n32 > 0 ? 2 : 0) | (n32 < c.count ? 1 : 0), n32);
      if (e != TLS_OK) return done(e);
    } else {
      // each fit's path (mixed_path_of): FP32-product LSQR first, then the
      // refinement fits, then FP64 LSQR for the rest and for refinements
      // that stopped short
      if (hipError_t he = batch_zero_ints(cnt, 4, s)) return done(hip_status(he));
      hipLaunchKernelGGL(mixed_dispatch_b_kernel, dim3(l.fits.n), dim3(256), 0, s, I + l.fits.off,
                         D, max_refine, MIXED_TOL_F32, cnt, 1);
      if (hipError_t he = hipGetLastError()) return done(hip_status(he));
      if (hipError_t he = hipMemcpyAsync(hc, cnt, 4 * sizeof(int), hipMemcpyDeviceToHost, s))
        return done(hip_status(he));
      if (hipError_t he = hipStreamSynchronize(s)) return done(hip_status(he));
      const int n_refine = hc[1];
      if (hc[0] < c.count) {
        hipLaunchKernelGGL(to_f32_b_kernel, dim3(l.blocks.n), dim3(256), 0, s, I + l.blocks.off, D);
        if (hipError_t he = hipGetLastError()) return done(hip_status(he));
        const tls_status e = lsqr_any(tm, 2, c.count - hc[0]);
        if (e != TLS_OK) return done(e);
        drop_graphs();
      }
      Lists sl = full_lists();
      for (int outer = 0; n_refine > 0 && outer <= max_refine; ++outer) {
        if (hipError_t he = batch_zero_ints(cnt, 2, s)) return done(hip_status(he));
        auto outer_step = [&]() -> hipError_t {
          hipError_t he = launch_small_rfft_b(PREC_F64, c.key.lgn, 2, SL_(fits), D, ctx->tw, s);
          if (!he) he = launch_toep_b(PREC_F64, c.key.lgn, BP_OUTER64, SL_(groups), D, ctx->consts,
                                      ctx->tw, s);
          if (!he) he = launch_colsum_b(1, SL_(cols), D, s);
          if (!he) he = launch_refine_outer_b(c.key.lgn, SL_(fits), c.pmax, D, cnt, ctx->tw, s);
          return he;
        };
        if (hipError_t he = outer_step()) return done(hip_status(he));
        for (int it = 0; it < inner_max; it += B_INNER_CHUNK) {
          const int kend = std::min(inner_max, it + B_INNER_CHUNK);
          auto inner = [&, it, kend]() -> tls_status {
            for (int k = it; k < kend; ++k) {
              if (tm) TLS_CHECK(tm->begin(s));
              TLS_CHECK(launch_toep_b(PREC_F32, c.key.lgn, BP_INNER32, SL_(groups), D, ctx->consts,
                                      ctx->tw, s));
              if (tm) TLS_CHECK(tm->end(s));
              TLS_CHECK(launch_colsum_b(2, SL_(cols), D, s));
              TLS_CHECK(launch_refine_cg_b(c.key.lgn, SL_(fits), c.pmax, D, cnt, ctx->tw, s));
            }
            return TLS_OK;
          };
          const tls_status e = run_graph(kend - it == B_INNER_CHUNK ? g_inner : g_inner_tail,
                                         graphs, s, inner);
          if (e != TLS_OK) return done(e);
          if (hipError_t he = hipMemcpyAsync(hc, cnt, 4 * sizeof(int), hipMemcpyDeviceToHost, s))
            return done(hip_status(he));
          if (hipError_t he = hipStreamSynchronize(s)) return done(hip_status(he));
          if (hc[1] >= sl.nfits) break;
        }
        // counts[0]: fits of the current lists whose refinement has finished
        if (hc[0] >= sl.nfits) break;
        if (!tm && worth_compacting(sl.nfits - hc[0], sl.nfits)) {
          const tls_status ec = compact(sl, 1);
          if (ec != TLS_OK) return done(ec);
        }
      }
      // FP64 finish for the fits whose refinement stopped short
      if (hipError_t he = batch_zero_ints(cnt, 4, s)) return done(hip_status(he));
      hipLaunchKernelGGL(fallback_prep_b_kernel, dim3(l.fits.n), dim3(64), 0, s, I + l.fits.off,
                         D, cnt);
      if (hipError_t he = hipGetLastError()) return done(hip_status(he));
      if (hipError_t he = hipMemcpyAsync(hc, cnt, 4 * sizeof(int), hipMemcpyDeviceToHost, s))
        return done(hip_status(he));
      if (hipError_t he = hipStreamSynchronize(s)) return done(hip_status(he));
      if (hc[0] < c.count) {
        drop_graphs();
        const tls_status e = lsqr_any(nullptr, 1, 0);
        if (e != TLS_OK) return done(e);
      }
    }
#undef SL_
    return done(residual_class(L_(rblocks), L_(fits), c.pmax, D, s));
  };

  // The classes are independent: up to BATCH_STREAMS of them run at once
  // (one while profiling), each on a stream of its own driven by a host
  // thread; the caller's stream orders them after the uploads above and
  // waits for all of them.
  const int nw = std::min<int>(static_cast<int>(classes.size()), o.profile ? 1 : BATCH_STREAMS);
  std::vector<PassTimer> timers(BATCH_STREAMS);
  if (nw > 0) {
    TLS_CHECK(ensure_batch_streams(ctx));
    TLS_CHECK(hipEventRecord(ctx->bready, s));
    std::atomic<int> next{0};
    std::vector<tls_status> wst(nw, TLS_OK);
    auto worker = [&](int w) {
      hipStream_t cs = ctx->bstream[w];
      timers[w].pool = &ctx->bevents[w];
      if (hipSetDevice(ctx->device) != hipSuccess || hipStreamWaitEvent(cs, ctx->bready, 0)) {
        wst[w] = TLS_EDEVICE;
      } else {
        for (int k; (k = next.fetch_add(1)) < static_cast<int>(classes.size());) {
          const tls_status e = run_class(classes[k], cs, hcounts + 8 * w,
                                         o.profile ? &timers[w] : nullptr);
          if (e != TLS_OK) {
            wst[w] = e;
            break;
          }
        }
      }
      if (hipEventRecord(ctx->bdone[w], cs) != hipSuccess && wst[w] == TLS_OK) wst[w] = TLS_EDEVICE;
    };
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(worker, w);
    worker(0);
    for (auto& t : th) t.join();
    for (int w = 0; w < nw; ++w) TLS_CHECK(hipStreamWaitEvent(s, ctx->bdone[w], 0));
    for (int w = 0; w < nw; ++w)
      if (wst[w] != TLS_OK) return wst[w];
  }
  if (nb > 0) {
    TLS_CHECK(collect_b(I + collect_off, nb, D, mixed ? 1 : 0, dcoef, drec, s));
    TLS_CHECK(hipMemcpyAsync(hrec, drec, sizeof(FitRec) * nb, hipMemcpyDeviceToHost, s));
    TLS_CHECK(hipMemcpyAsync(hcoef, dcoef, sizeof(double) * coef_total, hipMemcpyDeviceToHost, s));
    TLS_CHECK(hipStreamSynchronize(s));
  }
  const auto t1 = std::chrono::steady_clock::now();
  const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  double pass_ms = 0.0;
  int pass_count = 0;
  for (int w = 0; w < nw; ++w) {
    double x = 0.0;
    TLS_CHECK(timers[w].total_ms(&x));
    pass_ms += x;
    pass_count += static_cast<int>(timers[w].n);
  }

  int64_t off = 0;
  for (int j = 0; j < nb; ++j) {
    const int i = order[j];
    const Plan& pl = plans[i];
    double* coef = coef_packed + coef_offset[i];
    memcpy(coef, hcoef + off, pl.p * sizeof(double));
    off += pl.p;
    if (res) {
      record_result(hrec[j], pl, ms, &res[i]);
      res[i].pass_ms = pass_ms;  // the whole batch's launches of the dominant pass
      res[i].pass_count = pass_count;
      res[i].pass_kind = mixed ? 2 : 0;  // mixed: the FP32-product LSQR passes are timed
    }
    st[i] = record_status(hrec[j], coef, pl.p);
  }
  // Fits beyond the batched kernels' limits run one at a time.
  for (int i : singles) {
    tls_options oi = o;
    oi.request_id = o.request_id + static_cast<uint64_t>(i);
    tls_result r{};
    st[i] = run_fit(ctx, plans[i], oi, copy_y ? nullptr : dev_series[i],
                    copy_y ? host_series[i] : nullptr, tol, s, coef_packed + coef_offset[i], &r);
    if (res) res[i] = r;
  }
  tls_status first = TLS_OK;
  for (int i = 0; i < count; ++i) {
    if (fit_status) fit_status[i] = st[i];
    if (st[i] != TLS_OK && first == TLS_OK) first = st[i];
  }
  return first;
}
