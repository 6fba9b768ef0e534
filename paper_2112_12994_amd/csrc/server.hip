// Served continuous batching.
//
// Requests arrive at any time from any thread.  A worker thread owns one
// device arena of a fixed HBM budget and a table of fit slots; a request is
// admitted (first come, first served) as soon as its device footprint fits in
// the arena and a slot is free.  Every tick of the worker:
//   1. sets up the newly admitted fits (spectra, two-stage sketch, QR,
//      inverse, warm start, first LSQR steps), batched by launch class;
//   2. runs tick_steps (default 24) LSQR steps for every fit already
//      iterating, batched by FFT length and step variant, whatever its age
//      (a fit that converges on the way skips the remaining steps);
//   3. computes the FP64 residual and collects coefficients and results of
//      the fits that finished in the previous tick;
// then synchronises once, hands finished results to their tickets and
// releases their arena space and slots.  The work units of a tick (one
// launch class's set-up, one iteration group's steps, the finishing lists)
// touch disjoint fits, so they are spread over the server's streams by an
// estimate of their device time: most of these kernels fill a few compute
// units only, and concurrent units overlap their latency chains.  Series,
// spectra, the sketch factor and the LSQR state stay resident in the arena
// for a fit's whole life.
//
// Each fit runs the arithmetic of its single fit (the batched kernels share
// the single-fit kernels' bodies and launch-class choices), so its result is
// the same, bit for bit, whatever else is being served.
#include "engine.h"

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

namespace {

struct Request {
  tls_ticket ticket = 0;
  uint64_t request_id = 0;
  double tol = 0.0;
  const double* dev_y = nullptr;  // borrowed device series
  std::vector<double> host_y;     // or a copy of the host series
  Plan pl{};
  size_t bytes = 0, off = 0;
  int slot = -1;
  FitBufs b{};
  tls_status status = TLS_OK;
  tls_result res{};
  std::vector<double> coef;
  std::chrono::steady_clock::time_point t_submit;
  bool lsqr_done = false;  // worker only: LSQR finished, residual pending
  bool done = false;       // under the server mutex: result ready
};

// First-fit allocator over byte offsets [0, size), 256-byte granules.
class RangeAlloc {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size & ~size_t{255};
  }
  bool alloc(size_t len, size_t* off) {
    len = (len + 255) & ~size_t{255};
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const size_t rest = it->second - len, at = it->first;
      free_.erase(it);
      if (rest) free_[at + len] = rest;
      in_use_ += len;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t len) {
    len = (len + 255) & ~size_t{255};
    in_use_ -= len;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t in_use() const { return in_use_; }

 private:
  std::map<size_t, size_t> free_;
  size_t in_use_ = 0;
};

// Device buffer that grows (never shrinks) between ticks.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t count, hipStream_t s) {
    if (count <= cap) return hipSuccess;
    if (p) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      hipFree(p);
      p = nullptr;
    }
    const size_t c = std::max<size_t>(count + count / 2, 1024);
    hipError_t e = hipMalloc(&p, c * sizeof(T));
    if (e != hipSuccess) {
      cap = 0;
      return e;
    }
    cap = c;
    return hipSuccess;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Pinned host buffer that grows between ticks (each tick ends synchronised).
template <typename T>
struct HostBuf {
  T* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t count) {
    if (count <= cap) return hipSuccess;
    if (p) hipHostFree(p);
    p = nullptr;
    const size_t c = std::max<size_t>(count + count / 2, 1024);
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p), c * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) {
      cap = 0;
      return e;
    }
    cap = c;
    return hipSuccess;
  }
  void release() {
    if (p) hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Streams of a server: the worker's own plus SERVER_AUX more (the device
// runs four hardware queues per process).
constexpr int SERVER_AUX = 3;
// LSQR steps per tick by default: at 5000 requests/s of AR(2..200) series
// of 2^10..2^20 samples, 4, 8, 12 and 24 steps per tick gave median
// latencies of 33, 25, 23 and 22 ms and 99th percentiles of 111, 77, 67 and
// 57 ms (a request needs about 20 steps; shorter ticks cost more of them)
constexpr int SERVER_TICK_STEPS = 24;

}  // namespace

struct tls_server {
  tls_ctx* ctx = nullptr;
  tls_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t aux[SERVER_AUX] = {};
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_fin = nullptr;
  hipEvent_t ev_aux[SERVER_AUX] = {};
  char* arena = nullptr;
  size_t budget = 0;
  RangeAlloc alloc;
  int max_slots = 0;
  std::vector<int> free_slots;
  std::vector<Request*> slot_req;  // worker only
  FitDesc* dD = nullptr;       // max_slots descriptors
  int* dCounts = nullptr;      // [0] finished, [2] done-list length
  int* dDone = nullptr;        // done list (slots)
  DevBuf<Item> dItems;
  DevBuf<double> dCoef;
  DevBuf<FitRec> dRec;
  HostBuf<Item> hItems;
  HostBuf<FitDesc> hDesc;
  HostBuf<double> hCoef;
  HostBuf<FitRec> hRec;
  HostBuf<int> hDone;          // counters (4) then the done list

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<tls_ticket, Request*> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  tls_status failed = TLS_OK;  // a device error stops the worker
  uint64_t ticks = 0, admitted = 0, completed = 0;
  std::thread worker;
};

namespace {

using Clock = std::chrono::steady_clock;

// Fails every request not yet finished (the worker met a device error).
void fail_all(tls_server* S, std::vector<Request*>& lists, tls_status st) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->failed = st;
  for (Request* r : lists) {
    r->status = st;
    r->done = true;
  }
  for (Request* r : S->queue) {
    r->status = st;
    r->done = true;
  }
  S->queue.clear();
  S->cv_done.notify_all();
}

// Hands the finished requests to their tickets and frees their space.
void deliver(tls_server* S, const std::vector<Request*>& finishing) {
  std::lock_guard<std::mutex> lk(S->mu);
  for (Request* r : finishing) {
    S->alloc.release(r->off, r->bytes);
    S->free_slots.push_back(r->slot);
    S->slot_req[r->slot] = nullptr;
    r->done = true;
  }
  S->completed += finishing.size();
  if (!finishing.empty()) S->cv_done.notify_all();
}

// One tick of device work; returns a HIP error or success.  `admitted` are
// new fits (slots and arena space assigned); `active` iterate; `finishing`
// finished in the previous tick: their residual and results go first on the
// worker's stream, and they are delivered as soon as those are on the host,
// while the rest of the tick still runs.
hipError_t tick(tls_server* S, std::vector<Request*>& admitted, std::vector<Request*>& active,
                std::vector<Request*>& finishing, std::vector<Request*>* newly_done) {
  tls_ctx* ctx = S->ctx;
  hipStream_t s = S->stream;
  const tls_options& o = S->opt;
  const bool mixed = o.precision == TLS_PREC_MIXED;
  // LSQR variants per step: FP64 products, plus FP32 ones for mixed servers
  const int precs = mixed ? 3 : 1;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  const int steps = o.tick_steps > 0 ? o.tick_steps : SERVER_TICK_STEPS;
  hipError_t e;

  // descriptors of the new fits, series copies
  e = S->hDesc.ensure(admitted.size() + 1);
  if (e != hipSuccess) return e;
  for (size_t k = 0; k < admitted.size(); ++k) {
    Request* r = admitted[k];
    const bool copy_y = r->dev_y == nullptr;
    carve(r->pl, copy_y, &r->b, S->arena + r->off);
    if (copy_y) {
      e = hipMemcpyAsync(r->b.y, r->host_y.data(), r->pl.n * sizeof(double), hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return e;
    }
    fill_desc(r->pl, r->b, copy_y ? r->b.y : r->dev_y, static_cast<uint32_t>(r->request_id), r->tol,
              &S->hDesc.p[k]);
  }
  for (size_t k = 0; k < admitted.size(); ++k) {
    e = hipMemcpyAsync(S->dD + admitted[k]->slot, &S->hDesc.p[k], sizeof(FitDesc),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }

  // item lists: setup classes of the new fits; iteration groups of the
  // active fits; residual and collect lists of the finishing fits
  std::vector<Item> items;
  struct Setup {
    ClassKey key;
    int pmax, ldqmax;
    ClassLists l;
  };
  std::vector<Setup> setups;
  {
    std::map<ClassKey, std::vector<Request*>> g;
    for (Request* r : admitted) g[class_key(r->pl)].push_back(r);
    for (auto& kv : g) {
      Setup su{kv.first, 0, 0, {}};
      std::vector<int> desc;
      std::vector<const Plan*> pls;
      for (Request* r : kv.second) {
        desc.push_back(r->slot);
        pls.push_back(&r->pl);
        su.pmax = std::max(su.pmax, r->pl.p);
        su.ldqmax = std::max(su.ldqmax, r->pl.ldq);
      }
      su.l = build_lists(items, desc, pls, o.sketch == TLS_SKETCH_LEVERAGE);
      setups.push_back(su);
    }
  }
  List init_fits{static_cast<int>(items.size()), static_cast<int>(admitted.size())};
  for (Request* r : admitted) items.push_back({r->slot, 0});
  struct Iter {
    int lgn, pmax;
    bool mlds;
    List groups, cols, fits;  // pass block groups, columns of the partials, fits
  };
  std::vector<Iter> iters;
  {
    std::map<std::pair<int, int>, std::vector<Request*>> g;
    for (Request* r : active) g[{r->pl.lgn, lsqr_step_lds(r->pl.lgn, r->pl.p) ? 1 : 0}].push_back(r);
    for (auto& kv : g) {
      Iter it{kv.first.first, 0, kv.first.second != 0, {}, {}, {}};
      it.groups.off = static_cast<int>(items.size());
      for (Request* r : kv.second)
        for (int j = 0; j < r->pl.ngroups; ++j) items.push_back({r->slot, j});
      it.groups.n = static_cast<int>(items.size()) - it.groups.off;
      it.cols.off = static_cast<int>(items.size());
      for (Request* r : kv.second)
        for (int j = 0; j <= r->pl.p; ++j) items.push_back({r->slot, j});
      it.cols.n = static_cast<int>(items.size()) - it.cols.off;
      it.fits.off = static_cast<int>(items.size());
      for (Request* r : kv.second) {
        items.push_back({r->slot, 0});
        it.pmax = std::max(it.pmax, r->pl.p);
      }
      it.fits.n = static_cast<int>(items.size()) - it.fits.off;
      iters.push_back(it);
    }
  }
  List fin_rblocks{static_cast<int>(items.size()), 0};
  int fin_pmax = 0;
  for (Request* r : finishing) {
    for (int j = 0; j < resid_direct_blocks(r->pl.m); ++j) items.push_back({r->slot, j});
    fin_pmax = std::max(fin_pmax, r->pl.p);
  }
  fin_rblocks.n = static_cast<int>(items.size()) - fin_rblocks.off;
  List fin_fits{static_cast<int>(items.size()), static_cast<int>(finishing.size())};
  for (Request* r : finishing) items.push_back({r->slot, 0});
  List fin_collect{static_cast<int>(items.size()), static_cast<int>(finishing.size())};
  int64_t coef_total = 0;
  for (Request* r : finishing) {
    items.push_back({r->slot, static_cast<int>(coef_total)});
    coef_total += r->pl.p;
  }

  if (!items.empty()) {
    e = S->hItems.ensure(items.size());
    if (e == hipSuccess) e = S->dItems.ensure(items.size(), s);
    if (e != hipSuccess) return e;
    memcpy(S->hItems.p, items.data(), items.size() * sizeof(Item));
    e = hipMemcpyAsync(S->dItems.p, S->hItems.p, items.size() * sizeof(Item), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  const Item* I = S->dItems.p;
  e = batch_zero_ints(S->dCounts, 4, s);
  if (e != hipSuccess) return e;
  if (!admitted.empty()) {
    e = batch_init(I + init_fits.off, init_fits.n, S->dD, max_iter, 0, 0, 0.0, s);
    if (e != hipSuccess) return e;
  }

  // Each unit to the stream with the least estimated device time so far
  // (microseconds; a set-up is a chain of small factorisation kernels whose
  // length grows with the order, an LSQR step costs a few launches plus
  // its blocks).  Stream 0 (the worker's) also takes the finishing lists.
  hipStream_t sv[SERVER_AUX + 1] = {s};
  for (int k = 0; k < SERVER_AUX; ++k) sv[k + 1] = S->aux[k];
  double load[SERVER_AUX + 1] = {};
  bool used[SERVER_AUX + 1] = {true};
  int64_t fin_samples = 0;
  for (Request* r : finishing) fin_samples += r->pl.n;
  load[0] = finishing.empty() ? 0.0 : 40.0 + 1e-4 * static_cast<double>(fin_samples);
  auto pick = [&](double cost) {
    int k = 0;
    for (int j = 1; j <= SERVER_AUX; ++j)
      if (load[j] < load[k]) k = j;
    load[k] += cost;
    if (!used[k]) {
      used[k] = true;
      // the stream starts after this tick's uploads and initialisation
      if (hipStreamWaitEvent(sv[k], S->ev_start, 0) != hipSuccess) return -1;
    }
    return k;
  };
  e = hipEventRecord(S->ev_start, s);
  if (e != hipSuccess) return e;

  // 1. residual and results of the fits that finished in the previous tick
  if (!finishing.empty()) {
    if (residual_class(I + fin_rblocks.off, fin_rblocks.n, I + fin_fits.off, fin_fits.n, fin_pmax,
                       S->dD, s) != TLS_OK)
      return hipErrorUnknown;
    e = S->dCoef.ensure(coef_total, s);
    if (e == hipSuccess) e = S->dRec.ensure(finishing.size(), s);
    if (e == hipSuccess) e = S->hCoef.ensure(coef_total);
    if (e == hipSuccess) e = S->hRec.ensure(finishing.size());
    if (e != hipSuccess) return e;
    e = collect_b(I + fin_collect.off, fin_collect.n, S->dD, mixed ? 1 : 0, S->dCoef.p, S->dRec.p,
                  s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S->hRec.p, S->dRec.p, finishing.size() * sizeof(FitRec), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S->hCoef.p, S->dCoef.p, coef_total * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(S->ev_fin, s);
    if (e != hipSuccess) return e;
  }

  // 2. set-up and first LSQR steps of the new fits
  for (const Setup& su : setups) {
    const ClassLists& l = su.l;
    const int si = pick(300.0 + 3.0 * su.pmax + steps * (15.0 + 0.02 * l.groups.n));
    if (si < 0) return hipErrorUnknown;
    const hipStream_t ss = sv[si];
    if (setup_class(ctx, su.key, su.pmax, su.ldqmax, I, su.l, S->dD, o, ss) != TLS_OK)
      return hipErrorUnknown;
    if (mixed && o.estimator != TLS_EST_SKETCH) {
      // each new fit's products: FP32 when its sketch factor allows it
      // (mixed_path_of), else FP64; both LSQR variants then run over the lists
      hipLaunchKernelGGL(mixed_dispatch_b_kernel, dim3(l.fits.n), dim3(256), 0, ss,
                         I + l.fits.off, S->dD, 0, MIXED_TOL_F32, S->dCounts, 0);
      hipLaunchKernelGGL(to_f32_b_kernel, dim3(l.blocks.n), dim3(256), 0, ss, I + l.blocks.off, S->dD);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (o.estimator == TLS_EST_SKETCH) {
      // the compressed estimator: finished at set-up
      e = launch_compressed_b(I + l.fits.off, l.fits.n, S->dD, S->dCounts, S->dDone, ss);
      if (e != hipSuccess) return e;
      continue;
    }
    for (int k = 0; k < steps; ++k)
      if (lsqr_step_class(ctx, su.key.lgn, su.pmax, su.key.mlds != 0, k == 0, precs, I + l.groups.off,
                          l.groups.n, I + l.cols.off, l.cols.n, I + l.fits.off, l.fits.n, S->dD,
                          S->dCounts, S->dDone, nullptr, ss) != TLS_OK)
        return hipErrorUnknown;
  }
  // 3. tick_steps LSQR steps of every iterating fit (fits that finish on
  // the way skip the remaining steps)
  for (const Iter& it : iters) {
    const int si = pick(steps * (15.0 + 0.02 * it.groups.n));
    if (si < 0) return hipErrorUnknown;
    for (int k = 0; k < steps; ++k)
      if (lsqr_step_class(ctx, it.lgn, it.pmax, it.mlds, false, precs, I + it.groups.off, it.groups.n,
                          I + it.cols.off, it.cols.n, I + it.fits.off, it.fits.n, S->dD,
                          S->dCounts, S->dDone, nullptr, sv[si]) != TLS_OK)
        return hipErrorUnknown;
  }
  // the worker's stream waits for the others before the counters are read
  for (int k = 1; k <= SERVER_AUX; ++k) {
    if (!used[k]) continue;
    e = hipEventRecord(S->ev_aux[k - 1], sv[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, S->ev_aux[k - 1], 0);
    if (e != hipSuccess) return e;
  }
  e = hipMemcpyAsync(S->hDone.p, S->dCounts, 4 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->hDone.p + 4, S->dDone, S->max_slots * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;

  // results of the finishing fits, delivered before the tick ends
  if (!finishing.empty()) {
    e = hipEventSynchronize(S->ev_fin);
    if (e != hipSuccess) return e;
    int64_t off = 0;
    const auto now = Clock::now();
    for (size_t k = 0; k < finishing.size(); ++k) {
      Request* r = finishing[k];
      r->coef.assign(S->hCoef.p + off, S->hCoef.p + off + r->pl.p);
      off += r->pl.p;
      record_result(S->hRec.p[k], r->pl,
                    std::chrono::duration<double, std::milli>(now - r->t_submit).count(), &r->res);
      r->status = record_status(S->hRec.p[k], r->coef.data(), r->pl.p);
    }
    deliver(S, finishing);
    finishing.clear();  // handed over: no longer the worker's
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  // fits that finished in this tick (setup's first step or an iteration)
  const int ndone = std::min(S->hDone.p[2], S->max_slots);
  for (int k = 0; k < ndone; ++k) {
    const int slot = S->hDone.p[4 + k];
    if (slot < 0 || slot >= S->max_slots || !S->slot_req[slot]) return hipErrorUnknown;
    Request* r = S->slot_req[slot];
    r->lsqr_done = true;
    newly_done->push_back(r);
  }
  return hipSuccess;
}

void worker_main(tls_server* S) {
  hipSetDevice(S->ctx->device);
  std::vector<Request*> active, finishing;
  for (;;) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (active.empty() && finishing.empty()) {
        S->cv_work.wait(lk, [&] { return S->stopping || !S->queue.empty(); });
        if (S->queue.empty()) break;  // stopping and nothing left
      }
      while (!S->queue.empty() && !S->free_slots.empty()) {
        Request* r = S->queue.front();
        size_t off = 0;
        if (!S->alloc.alloc(r->bytes, &off)) break;
        r->off = off;
        r->slot = S->free_slots.back();
        S->free_slots.pop_back();
        S->slot_req[r->slot] = r;
        S->queue.pop_front();
        admitted.push_back(r);
      }
      S->admitted += admitted.size();
    }
    std::vector<Request*> newly_done;
    const hipError_t e = tick(S, admitted, active, finishing, &newly_done);
    if (e != hipSuccess) {
      std::vector<Request*> all = admitted;
      all.insert(all.end(), active.begin(), active.end());
      all.insert(all.end(), finishing.begin(), finishing.end());
      fail_all(S, all, e == hipErrorOutOfMemory ? TLS_ENOMEM : TLS_EDEVICE);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->ticks += 1;
    }
    // new state: the fits done in this tick finish next tick
    std::vector<Request*> next_active;
    for (Request* r : active)
      if (!r->lsqr_done) next_active.push_back(r);
    for (Request* r : admitted)
      if (!r->lsqr_done) next_active.push_back(r);
    active.swap(next_active);
    finishing.swap(newly_done);
  }
}

tls_status submit(tls_server* S, const double* host_y, const double* dev_y, int64_t n, int32_t p,
                  double tol, uint64_t request_id, tls_ticket* ticket) {
  if (!S || !ticket || (!host_y && !dev_y)) return TLS_EINVAL;
  tls_status st = validate(n, p, tol, S->opt);
  if (st != TLS_OK) return st;
  if (host_y)
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(host_y[i])) return TLS_EINVAL;
  auto* r = new Request();
  st = make_plan(n, p, S->opt, &r->pl, S->ctx);
  if (st == TLS_OK && r->pl.ldq > BATCH_LDQ_MAX) st = TLS_EUNSUPPORTED;
  if (st == TLS_OK) {
    FitBufs tmp{};
    r->bytes = carve(r->pl, host_y != nullptr, &tmp, nullptr);
    if (((r->bytes + 255) & ~size_t{255}) > (S->budget & ~size_t{255})) st = TLS_ENOMEM;
  }
  if (st != TLS_OK) {
    delete r;
    return st;
  }
  r->request_id = request_id;
  r->tol = tol;
  r->dev_y = dev_y;
  if (host_y) r->host_y.assign(host_y, host_y + n);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping || S->failed != TLS_OK) {
      const tls_status f = S->failed != TLS_OK ? S->failed : TLS_EINVAL;
      delete r;
      return f;
    }
    r->ticket = S->next_ticket++;
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
  }
  S->cv_work.notify_one();
  return TLS_OK;
}

tls_status take(tls_server* S, tls_ticket t, bool block, double* coef, tls_result* out,
                tls_status* fit_status) {
  if (!S) return TLS_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(t);
  if (it == S->reqs.end()) return TLS_EINVAL;
  Request* r = it->second;
  if (!r->done) {
    if (!block) return TLS_EAGAIN;
    S->cv_done.wait(lk, [&] { return r->done; });
  }
  S->reqs.erase(t);
  lk.unlock();
  if (coef && !r->coef.empty()) memcpy(coef, r->coef.data(), r->coef.size() * sizeof(double));
  if (out) *out = r->res;
  if (fit_status) *fit_status = r->status;
  delete r;
  return TLS_OK;
}

}  // namespace

extern "C" {

tls_status tls_server_create(tls_ctx* ctx, size_t hbm_budget, int32_t max_slots,
                             const tls_options* opt, tls_server** out) {
  if (!ctx || !out || max_slots < 1 || hbm_budget < (size_t{1} << 20)) return TLS_EINVAL;
  const tls_options o = opt ? *opt : ctx->opt;
  // served fits take FP32 or FP64 products per fit (mixed_path_of); the FP64
  // refinement band and repeated halving are not served
  if (o.sketch == TLS_SKETCH_RH) return TLS_EUNSUPPORTED;
  if (o.precision == TLS_PREC_MIXED && o.max_refine > 0) return TLS_EUNSUPPORTED;
  if (o.precision != TLS_PREC_F64 && o.precision != TLS_PREC_MIXED) return TLS_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return TLS_EDEVICE;
  auto* S = new tls_server();
  S->ctx = ctx;
  S->opt = o;
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  for (int k = 0; k < SERVER_AUX && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&S->aux[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_aux[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_start, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_fin, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&S->arena, hbm_budget);
  if (e == hipSuccess) e = hipMalloc(&S->dD, sizeof(FitDesc) * max_slots);
  if (e == hipSuccess) e = hipMalloc(&S->dCounts, 4 * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&S->dDone, sizeof(int) * max_slots);
  if (e == hipSuccess) e = S->hDone.ensure(4 + static_cast<size_t>(max_slots));
  if (e != hipSuccess) {
    if (S->arena) hipFree(S->arena);
    if (S->dD) hipFree(S->dD);
    if (S->dCounts) hipFree(S->dCounts);
    if (S->dDone) hipFree(S->dDone);
    S->hDone.release();
    for (int k = 0; k < SERVER_AUX; ++k) {
      if (S->aux[k]) hipStreamDestroy(S->aux[k]);
      if (S->ev_aux[k]) hipEventDestroy(S->ev_aux[k]);
    }
    if (S->ev_start) hipEventDestroy(S->ev_start);
    if (S->ev_fin) hipEventDestroy(S->ev_fin);
    if (S->stream) hipStreamDestroy(S->stream);
    delete S;
    return e == hipErrorOutOfMemory ? TLS_ENOMEM : TLS_EDEVICE;
  }
  S->alloc.init(hbm_budget);
  for (int k = max_slots - 1; k >= 0; --k) S->free_slots.push_back(k);
  S->slot_req.assign(max_slots, nullptr);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return TLS_OK;
}

tls_status tls_submit(tls_server* S, const double* series, int64_t n, int32_t p, double tol,
                      uint64_t request_id, tls_ticket* ticket) {
  if (!series) return TLS_EINVAL;
  return submit(S, series, nullptr, n, p, tol, request_id, ticket);
}

tls_status tls_submit_device(tls_server* S, const double* d_series, int64_t n, int32_t p,
                             double tol, uint64_t request_id, tls_ticket* ticket) {
  if (!d_series) return TLS_EINVAL;
  return submit(S, nullptr, d_series, n, p, tol, request_id, ticket);
}

tls_status tls_poll(tls_server* S, tls_ticket ticket, double* coef, tls_result* out,
                    tls_status* fit_status) {
  return take(S, ticket, false, coef, out, fit_status);
}

tls_status tls_wait(tls_server* S, tls_ticket ticket, double* coef, tls_result* out,
                    tls_status* fit_status) {
  return take(S, ticket, true, coef, out, fit_status);
}

tls_status tls_server_get_stats(tls_server* S, tls_server_stats* out) {
  if (!S || !out) return TLS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out->ticks = S->ticks;
  out->admitted = S->admitted;
  out->completed = S->completed;
  out->queued = S->queue.size();
  out->in_flight = S->admitted - S->completed;
  out->arena_bytes_in_use = S->alloc.in_use();
  out->arena_bytes = S->budget;
  out->status = S->failed;
  return TLS_OK;
}

void tls_server_destroy(tls_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  hipSetDevice(S->ctx->device);
  hipStreamSynchronize(S->stream);
  for (int k = 0; k < SERVER_AUX; ++k) hipStreamSynchronize(S->aux[k]);
  for (auto& kv : S->reqs) delete kv.second;
  S->dItems.release();
  S->dCoef.release();
  S->dRec.release();
  S->hItems.release();
  S->hDesc.release();
  S->hCoef.release();
  S->hRec.release();
  S->hDone.release();
  hipFree(S->arena);
  hipFree(S->dD);
  hipFree(S->dCounts);
  hipFree(S->dDone);
  for (int k = 0; k < SERVER_AUX; ++k) {
    hipStreamDestroy(S->aux[k]);
    hipEventDestroy(S->ev_aux[k]);
  }
  hipEventDestroy(S->ev_start);
  hipEventDestroy(S->ev_fin);
  hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
