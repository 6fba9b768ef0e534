"""Throughput of the Toeplitz least-squares AR(p) fit on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ar100]

A step is one complete fit (block spectra, two-stage randomized sketch, QR,
R-preconditioned LSQR, FP64 residual) of one synthetic series already
resident in device memory, through the C-ABI (tls_fit_device).  W untimed
steps, then K timed steps between device synchronisations; value = K / time.

Besides the JSON fields of the bench contract, the line carries:
  roofline      the fused Toeplitz pass (X v, the u update and X^T u in one
                launch): algorithmic bytes per launch / its average device
                time, timed live with HIP events on the library stream during
                the timed steps, against the 8 TB/s HBM peak;
  cpu_baseline  the FP64 QR oracle timed on the host's cores on a bounded
                prefix of the same series, scaled to one full-size solve;
  accuracy      relative coefficient error, fitted-value error and residual
                difference against the stored oracle solution, with kappa(X).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AR(p) Toeplitz-LSQR solves/sec & FFT-matvec HBM GB/s at rel err 1e-6"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6  # MI355X dense FP64 matrix peak

WORKLOAD_TEXT = {
    "ar100": "AR(100) series, n=2^22, 50 pole pairs with moduli U[0.5,0.95] and angles "
             "U(0,pi), N(0,1) innovations, seed 0; sketch 8p rows, LSQR tol 1e-10, FP64",
    "ar3": "AR(3), phi=(0.5,-0.3,0.1), n=10000, N(0,1), burn-in 500, seed 0; sketch 20p, "
           "LSQR tol 1e-10, FP64",
    "ar500": "AR(500) series, n=2^25, 250 pole pairs with moduli U[0.5,0.95] and angles U(0,pi), "
             "N(0,1) innovations, seed 0; sketch 8p rows, tol 1e-10",
    "batch": "2048 independent series, n=round(2^U(12,18)), p~U{4..64}, pole moduli U[0.3,0.95], "
             "t5 innovations, seed 0; one batched call per step; sketch 8p rows, tol 1e-10",
    "sketch": "AR(100) series, n=2^22 (the ar100 series); compressed (sketch-and-solve) "
              "estimator of eq. (OLSc) for sketch sizes c = gamma p, gamma in 2..64, FP64; "
              "errors against the FP64 OLS fit of the same series",
    "pacf": "AR(150) series, n=2,000,000, 75 pole pairs with moduli U[0.5,0.95] and angles U(0,pi), "
            "N(0,1) innovations, seed 0; PACF at lags 1..250 (one AR(h) fit per lag on the prefix "
            "of n-250+h samples), exact (FP64 OLS) and compressed (sketch 8h rows), tol 1e-10",
    "rh": "AR(5), AR(20), AR(100) series, n=2,000,000, pole moduli U[0.5,0.95], N(0,1) innovations, "
          "seed 0, without and with 1000 outliers (+U[-3,3]+N(0,100), Section 4.2); lags 1..p on "
          "the prefix windows of the PACF study; compressed estimates from the leverage (LSAR) and "
          "repeated-halving (RH) sketches with c = 20h rows against the exact FP64 OLS fits",
    "serve": "Poisson arrivals at 5000 requests/s, each a series drawn with replacement from a pool "
             "of resident series with n=round(2^U(10,20)), p~U{2..200}, pole moduli U[0.5,0.95], "
             "N(0,1) innovations, seed 0; FP64, sketch 8p rows, tol 1e-10",
}


# Sources that define the fused Toeplitz pass: HBM counters taken from a
# profile are used only while these are unchanged.
PASS_SOURCES = ["paper_2112_12994_amd/csrc/toeplitz_impl.h", "paper_2112_12994_amd/csrc/fft.h",
                "paper_2112_12994_amd/csrc/common.h", "paper_2112_12994_amd/csrc/toeplitz.hip"]


def qr_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2112_12994_amd/csrc/qr.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def read_mfma_profile(workload: str):
    """FP64-MFMA figures of the QR kernels from the committed counter summary
    (profiles/qr_mfma_<workload>.txt) while qr.hip is unchanged since."""
    path = os.path.join(ROOT, "profiles", f"qr_mfma_{workload}.txt")
    if not os.path.exists(path):
        return None
    rows, hsh = [], None
    with open(path) as fh:
        for line in fh:
            if line.startswith("qr_source_hash:"):
                hsh = line.split(":", 1)[1].strip()
            elif line and not line.startswith(("#", "kernel", "qr_source_hash")):
                f = line.split()
                if len(f) >= 6:
                    rows.append({"kernel": " ".join(f[:-5]), "dispatches": int(f[-5]),
                                 "f64_mfma_flop_per_dispatch": float(f[-4]),
                                 "avg_us": float(f[-3]), "tflops": float(f[-2]),
                                 "util": float(f[-1])})
    if hsh != qr_source_hash() or not rows:
        return None
    flop = sum(r["f64_mfma_flop_per_dispatch"] * r["dispatches"] for r in rows)
    us = sum(r["avg_us"] * r["dispatches"] for r in rows)
    return {"source": os.path.relpath(path, ROOT), "kernels": rows,
            "util_over_mfma_kernels": flop / (us * 1e-6) / (FP64_MFMA_PEAK_TFS * 1e12)}


def pass_source_hash() -> str:
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hbm_profile_name(workload: str, precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"toep_pass_{precision}_{workload}_hbm_counters.txt")


def read_hbm_profile(workload: str, precision: str, kernel_prefix: str = "toep_pass_kernel<double"):
    """HBM bytes per launch of the dominant pass from the committed counter
    summary, or None when there is none, it covers another kernel, or the
    pass sources changed since."""
    path = hbm_profile_name(workload, precision)
    if not os.path.exists(path):
        return None, "no counter profile"
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if not kv.get("kernel", "").startswith(kernel_prefix):
        return None, f"the counter profile covers {kv.get('kernel')}, not the timed pass"
    if kv.get("source_hash") != pass_source_hash():
        return None, "pass sources changed since the counters were taken"
    return float(kv["hbm_bytes_per_dispatch"]), os.path.relpath(path, ROOT)


def _rows(pattern_dir: str, suffix: str):
    files = sorted(glob.glob(os.path.join(pattern_dir, "**", f"*{suffix}"), recursive=True))
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend({k.lower(): v for k, v in r.items()} for r in csv.DictReader(fh))
    return rows


def _short(name: str) -> str:
    s = name.replace("(anonymous namespace)::", "").replace("tls::", "")
    if s.startswith("void "):
        s = s[5:]
    return s.split("(")[0] if "(" in s and not s.startswith("(") else s


def prof_summary(kind: str, dirs: list, out: str, cmd: str, title: str):
    """Compact text summaries of rocprofv3 CSV output (kernel statistics, or
    per-dispatch HBM counters with the copy-kernel calibration)."""
    lines = [f"# {title}", f"# command: {cmd}", f"source_hash: {pass_source_hash()}"]
    if kind == "mfma":
        # dirs: counter run (SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES,
        # GRBM_GUI_ACTIVE), kernel-statistics run of the same command
        lines[2] = f"qr_source_hash: {qr_source_hash()}"
        per = {}
        for r in _rows(dirs[0], "counter_collection.csv"):
            k = _short(r["kernel_name"])
            d = per.setdefault(k, {}).setdefault(r["dispatch_id"], {})
            d[r["counter_name"]] = float(r["counter_value"])
        avg = {_short(r["name"]): float(r["averagens"]) for r in _rows(dirs[1], "kernel_stats.csv")}
        lines.append(f"{'kernel':60s} {'disp':>5s} {'f64_mfma_flop':>14s} {'avg_us':>9s} "
                     f"{'TFLOP/s':>8s} {'util_of_78.6':>12s}")
        for k, ds in sorted(per.items()):
            mops = [d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for d in ds.values()]
            if not any(mops):
                continue
            flop = 512.0 * sum(mops) / len(mops)
            us = avg.get(k, float("nan")) / 1e3
            tf = flop / (us * 1e-6) / 1e12 if us == us else float("nan")
            lines.append(f"{k[:60]:60s} {len(ds):5d} {flop:14.4e} {us:9.2f} {tf:8.3f} "
                         f"{tf / FP64_MFMA_PEAK_TFS:12.4f}")
    elif kind == "stats":
        rows = _rows(dirs[0], "kernel_stats.csv")
        tot = sum(float(r["totaldurationns"]) for r in rows) or 1.0
        lines.append(f"{'kernel':90s} {'calls':>7s} {'total_us':>11s} {'avg_us':>9s} {'pct':>6s}")
        for r in sorted(rows, key=lambda r: -float(r["totaldurationns"])):
            lines.append(f"{_short(r['name'])[:90]:90s} {int(r['calls']):7d} "
                         f"{float(r['totaldurationns']) / 1e3:11.1f} {float(r['averagens']) / 1e3:9.2f} "
                         f"{100 * float(r['totaldurationns']) / tot:6.2f}")
    else:
        # dirs: FETCH run, WRITE run, copy FETCH run, copy WRITE run; kernel filter
        kern, copy_bytes = kind.split("=", 1)[1].rsplit("@", 1)
        copy_bytes = float(copy_bytes)

        def mean_for(d, counter, match):
            vals = {}
            for r in _rows(d, "counter_collection.csv"):
                if r.get("counter_name") != counter:
                    continue
                vals.setdefault(_short(r["kernel_name"]), []).append(float(r["counter_value"]))
            if match is None:  # the copy run: the kernel that moved the most
                name = max(vals, key=lambda k: max(vals[k]))
            elif match.endswith("*"):  # every kernel with this prefix, pooled
                v = [x for k in vals if k.startswith(match[:-1]) for x in vals[k]]
                return match, sum(v) / len(v), len(v)
            else:
                name = next(k for k in vals if k.startswith(match))
            v = vals[name]
            return name, sum(v) / len(v), len(v)

        kname, fetch, nf = mean_for(dirs[0], "FETCH_SIZE", kern)
        _, write, nw = mean_for(dirs[1], "WRITE_SIZE", kern)
        if kern.endswith("*"):
            kname = kern + " (every instantiation)"
        cname, cfetch, _ = mean_for(dirs[2], "FETCH_SIZE", None)
        _, cwrite, _ = mean_for(dirs[3], "WRITE_SIZE", None)
        fs, ws = copy_bytes / (cfetch * 1024), copy_bytes / (cwrite * 1024)
        lines += [f"kernel: {kname}", f"dispatches_fetch: {nf}", f"dispatches_write: {nw}",
                  f"fetch_kib_per_dispatch: {fetch:.1f}", f"write_kib_per_dispatch: {write:.1f}",
                  f"copy_kernel: {cname}", f"copy_bytes_each_way: {copy_bytes:.0f}",
                  f"copy_fetch_kib_per_dispatch: {cfetch:.1f}",
                  f"copy_write_kib_per_dispatch: {cwrite:.1f}",
                  f"fetch_scale: {fs:.4f}", f"write_scale: {ws:.4f}",
                  f"hbm_bytes_per_dispatch: {fetch * 1024 * fs + write * 1024 * ws:.0f}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def pass_groups(B: int, nblocks: int) -> int:
    """Workgroups of the Toeplitz pass: up to B = 1024 a 256-thread
    workgroup takes 256 / (B / 16) blocks (B / 16 threads each, at least 8:
    32 blocks at B = 128, 4 at B = 1024), 2 at a time up to B = 4096, else
    singly (the library's pass_nw)."""
    lgn = B.bit_length() - 2
    nt = min(max((1 << lgn) // 8, 8), 256)
    nw = 256 // nt if lgn <= 9 else (2 if lgn <= 11 else 1)
    return -(-nblocks // nw)


def fused_pass_bytes(n: int, p: int, B: int, nblocks: int, elem: int) -> int:
    """Algorithmic bytes of one fused pass: read every block spectrum
    (B/2 complex words per block), read and write the m-vector u, read v's
    spectrum once, write the (p+1) partial sums of every block group."""
    m = n - p
    spec = nblocks * (B // 2) * 2 * elem
    return (spec + 2 * m * elem + (B // 2) * 2 * elem
            + (p + 1) * pass_groups(B, nblocks) * 8)


def cpu_baseline(y: np.ndarray, p: int, budget_s: float = 20.0) -> dict:
    """Oracle (dense LAPACK QR of [X | b]) on a prefix, scaled linearly in the
    row count (the QR of an m x (p+1) matrix costs O(m p^2))."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    m_full = y.size - p
    rows = min(m_full, 1 << 16)
    t = 0.0
    while True:
        t0 = time.perf_counter()
        oracle.fit_qr(y[: rows + p], p)
        t = time.perf_counter() - t0
        if rows >= m_full or t > budget_s / 4 or rows >= (1 << 20):
            break
        rows = min(m_full, rows * 4)
    per_solve = t * m_full / rows
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": int(cores),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"oracle.fit_qr (dense [X|b] + LAPACK Householder QR) on the first "
                      f"{rows + p} samples ({rows} rows) in {t:.2f} s, scaled by {m_full}/{rows} "
                      f"rows to one full-size solve"}


def accuracy(y, p, coef, resid, workload):
    """Errors against the stored oracle solution (AR(100) seed 0) or a fresh
    oracle solve (small workloads)."""
    import oracle
    if workload == "ar100" and y.size == (1 << 22):
        d = np.loadtxt(os.path.join(ROOT, "tests", "golden", "ar100_seed0_oracle.txt"))
        phi, rnorm, kappa = d[:-3], float(d[-3]), float(d[-2])
    else:
        ref = oracle.fit_qr(y, p)
        phi, rnorm, kappa = ref["phi"], ref["rnorm"], ref["kappa"]
    # fitted-value error ||X (coef - phi)|| / ||X phi|| in row chunks
    num = den = 0.0
    step = 1 << 18
    m = y.size - p
    for a in range(0, m, step):
        rows = min(step, m - a)
        seg = y[a: a + rows + p]
        num += float(np.sum(oracle.matvec(seg, p, coef - phi) ** 2))
        den += float(np.sum(oracle.matvec(seg, p, phi) ** 2))
    return {"kappa": kappa, "rel_err": oracle.rel_error(coef, phi),
            "fitted_rel_err": float(np.sqrt(num / den)),
            "resid_rel_diff": abs(resid - rnorm) / rnorm,
            "attainable": "coefficients beyond FP64 resolution (kappa*1e-16 > 1e-6)"
            if kappa * 1e-16 > 1e-6 else "coefficient gate attainable"}


def row_chunks(m: int, step: int = 1 << 16, max_chunks: int = 16):
    """Row ranges for the dense checks: all rows in chunks, or at most
    max_chunks chunks spread evenly over the rows."""
    starts = list(range(0, m, step))
    if len(starts) > max_chunks:
        pick = np.linspace(0, len(starts) - 1, max_chunks).round().astype(int)
        starts = [starts[i] for i in sorted(set(pick))]
    return [(a, min(step, m - a)) for a in starts]


def gpu_fp64_agreement(y, p, out, ref):
    """Full-size comparison of a fit against the GPU FP64 fit of the same
    series (the dense oracle does not fit in host memory at this size);
    fitted values on 16 row chunks of 2^16 spread over the series."""
    import oracle
    d = out["coef"] - ref["coef"]
    num = den = 0.0
    m = y.size - p
    for a, rows in row_chunks(m):
        seg = y[a: a + rows + p]
        num += float(np.sum(oracle.matvec(seg, p, d) ** 2))
        den += float(np.sum(oracle.matvec(seg, p, ref["coef"]) ** 2))
    return {"reference": "GPU FP64 fit at full size (fitted values on 16 row chunks of 2^16)",
            "kappa_est_R": ref["kappa_est"],
            "rel_err_vs_f64": float(np.linalg.norm(d) / np.linalg.norm(ref["coef"])),
            "fitted_rel_err": float(np.sqrt(num / den)),
            "resid_rel_diff": abs(out["resid_norm"] - ref["resid_norm"]) / ref["resid_norm"],
            "f64_status": ref["status"]}


def batch_bench(args, torch, synth, capi):
    """The batched workload: `steps` calls of tls_fit_batch_device over 2048
    resident series; value = fits per second.  Beside it: the same fits as
    one synchronous FP64 tls_fit_device call each (the plain per-series
    path), the oracle on a bounded subset, and agreement with the oracle on
    a sample of fits."""
    import oracle
    prec = 1 if args.precision == "mixed" else 0
    t0 = time.perf_counter()
    fits = synth.workload_batch(seed=0)
    print(f"[bench] batch of {len(fits)} generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    dys = [torch.from_numpy(f.y).to("cuda:0") for f in fits]
    ps = [f.p for f in fits]
    torch.cuda.synchronize()
    ctx = capi.Context(0, gamma=8, precision=prec, block_lg=args.block_lg)
    stream = torch.cuda.current_stream()
    tuned = {}
    if args.block_lg == 0:
        # block lengths from the autotuner (device measurements, before the timed region)
        t0 = time.perf_counter()
        pmin, pmax = min(ps), max(ps)
        nmin, nmax = min(f.y.size for f in fits), max(f.y.size for f in fits)
        ctx.autotune(prec, pmin, pmax, max(nmin, 2 * pmax + 1), nmax)
        table = ctx.tuning()
        for f in fits:
            lg = int(table[capi.tune_index(prec, f.p, f.y.size - f.p)])
            key = "p<=%d,m<=2^%d" % (1 << max(0, (f.p - 1).bit_length()),
                                     max(0, (f.y.size - f.p - 1).bit_length()))
            tuned[key] = 1 << lg if lg else None
        print(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        s, outs = ctx.fit_batch_device(dys, ps, 1e-10, stream=stream)
    torch.cuda.synchronize()
    print(f"[bench] warmup done: status {capi.status_string(s) if args.warmup else None}",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s, outs = ctx.fit_batch_device(dys, ps, 1e-10, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} batches in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # one more call with every launch of the dominant pass bracketed by HIP
    # events (graphs off while profiling): the pass's average launch time
    _, pouts = ctx.fit_batch_device(dys, ps, 1e-10, stream=stream, profile=1)
    torch.cuda.synchronize()
    pass_ms = pouts[0]["pass_ms"]
    pass_count = pouts[0]["pass_count"]
    # algorithmic bytes of the dominant pass over one batch: per fit, bytes of
    # one pass times the passes that did work for it
    tot_bytes = 0.0
    # (mixed: the fused pass with FP32 products for the fits on that path,
    # whose launches the same events bracket)
    for f, o in zip(fits, outs):
        B, nb = o["block_len"], o["n_blocks"]
        elem = 4 if prec and o["mixed_path"] == 1 else 8
        tot_bytes += fused_pass_bytes(f.y.size, f.p, B, nb, elem) * (o["iters"] + 1)
    avg_launch_s = pass_ms / max(pass_count, 1) / 1e3
    achieved = tot_bytes / (pass_ms / 1e3) / 1e9 if pass_ms else 0.0
    statuses = [o["status"] for o in outs]

    # plain path: one synchronous FP64 fit per series
    plain = None
    if not args.no_extras:
        ctx64 = capi.Context(0, gamma=8, precision=0)
        for i in range(8):
            ctx64.fit_device(dys[i], ps[i], 1e-10, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d, p in zip(dys, ps):
            ctx64.fit_device(d, p, 1e-10, stream=stream)
        torch.cuda.synchronize()
        plain = len(fits) / (time.perf_counter() - t0)
        ctx64.close()

    # agreement with the oracle on every 32nd fit
    errs = []
    for i in range(0, 0 if args.no_extras else len(fits), 32):
        ref = oracle.fit_qr(fits[i].y, fits[i].p)
        errs.append((ref["kappa"], oracle.rel_error(outs[i]["coef"], ref["phi"])))
    gate = 1e-4 if prec else 1e-6
    strata = {}
    for lo, hi, name in [(0, 1e6, "kappa<1e6"), (1e6, 1e12, "1e6<=kappa<1e12"),
                         (1e12, float("inf"), "kappa>=1e12")]:
        sel = [e for k, e in errs if lo <= k < hi]
        strata[name] = {"fits": len(sel), "within_gate": sum(e <= gate for e in sel),
                        "max_rel_err": max(sel) if sel else None}

    cpu = None
    if not args.no_cpu:
        cost = [(f.y.size - f.p) * (f.p + 1) ** 2 for f in fits]
        t0 = time.perf_counter()
        done = 0
        for f in fits:
            oracle.fit_qr(f.y, f.p)
            done += 1
            if time.perf_counter() - t0 > 15.0:
                break
        t = time.perf_counter() - t0
        total = t * sum(cost) / sum(cost[:done])
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
        except Exception:  # pragma: no cover
            cores = os.cpu_count() or 1
        cpu = {"value": len(fits) / total, "unit": "solves/s", "cores": int(cores),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": f"oracle.fit_qr on the first {done} of the {len(fits)} series in {t:.1f} s, "
                         f"scaled by the m (p+1)^2 cost of all series"}
    classes = sorted({(o["block_len"]) for o in outs})
    traffic, traffic_src = None, "non-default configuration"
    if not args.block_lg:
        traffic, traffic_src = read_hbm_profile(
            "batch", args.precision, "toep_b_kernel<double" if prec == 0 else "toep_b_kernel<float")
    mf = read_mfma_profile("batch")
    line = {
        "metric": METRIC, "value": args.steps * len(fits) / elapsed, "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == 0 else "f32 products, f64 recurrences",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["batch"], "fits_per_step": len(fits),
                   "samples_per_step": int(sum(f.y.size for f in fits)),
                   "precision": args.precision, "fft_blocks_used": classes,
                   "fft_block_source": "autotuner" if tuned else "block_lg=%d" % args.block_lg,
                   "autotuned_blocks": tuned or None,
                   "graphs": "each chunk of LSQR / inner steps of a class replayed as a HIP graph",
                   "status": capi.status_string(s),
                   "fit_statuses": {capi.status_string(k): statuses.count(k) for k in set(statuses)},
                   "median_iters": int(np.median([o["iters"] for o in outs])),
                   "mixed_paths": ({"fp32_products": sum(o["mixed_path"] == 1 for o in outs),
                                    "fp64_refinement": sum(o["mixed_path"] == 2 for o in outs),
                                    "fp64_products": sum(o["mixed_path"] == 3 for o in outs)}
                                   if prec else None)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": traffic_src,
                     "kernel": "toep_b_kernel (batched Toeplitz pass, "
                               + ("FP64 fused LSQR pass)" if prec == 0 else "FP32 normal-equation pass)"),
                     "bytes_per_launch": tot_bytes / max(pass_count, 1),
                     "avg_launch_us": avg_launch_s * 1e6, "launches_timed": pass_count,
                     "timed_in": "one extra batched call with profile=1 after the timed steps"},
        "plain_fp64_per_series": {"value": plain, "unit": "solves/s",
                                  "what": "one synchronous FP64 tls_fit_device per series"},
        "accuracy": {"oracle_sample": len(errs), "gate": gate, "by_kappa": strata},
    }
    if mf:
        line["qr_fp64_mfma"] = mf
    if cpu:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


def sketch_bench(args, torch, synth, capi):
    """The paper's compressed estimator (Section 2.1, eq. (OLSc)) on the AR(100)
    n=2^22 series for a sweep of sketch sizes (the error-versus-c study of
    Section 4.1, here on the synthetic series): per gamma, fits/s of the
    compressed estimator (estimator = TLS_EST_SKETCH, no LSQR), its relative
    coefficient error and residual ratio against the FP64 OLS fit.  value:
    fits/s at gamma = 8."""
    f = synth.WORKLOADS["ar100"](seed=0)
    y, p = f.y, f.p
    dy = torch.from_numpy(y).to("cuda:0")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ctx = capi.Context(0, precision=0)
    ctx.fit_device(dy, p, 1e-10, stream=stream)  # warm-up
    ols = ctx.fit_device(dy, p, 1e-10, stream=stream)
    rows = []
    value = None
    for gamma in (2, 4, 8, 16, 32, 64):
        for _ in range(args.warmup):
            out = ctx.fit_device(dy, p, 1e-10, stream=stream, gamma=gamma, estimator=capi.EST_SKETCH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = ctx.fit_device(dy, p, 1e-10, stream=stream, gamma=gamma, estimator=capi.EST_SKETCH)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        err = float(np.linalg.norm(out["coef"] - ols["coef"]) / np.linalg.norm(ols["coef"]))
        rows.append({"gamma": gamma, "c": gamma * p, "ms_per_fit": dt * 1e3, "fits_per_s": 1.0 / dt,
                     "rel_err_vs_ols": err, "resid_ratio": out["resid_norm"] / ols["resid_norm"],
                     "status": capi.status_string(out["status"])})
        print(f"[bench] gamma {gamma}: {dt * 1e3:.3f} ms, err {err:.3g}, "
              f"ratio {rows[-1]['resid_ratio']:.6f}", file=sys.stderr, flush=True)
        if gamma == 8:
            value = 1.0 / dt
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 / value, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["sketch"], "n": int(y.size), "p": p,
                   "estimator": "compressed (sketch-and-solve)", "value_at_gamma": 8},
        "sweep": rows,
        "ols_reference": {"iters": ols["iters"], "resid_norm": ols["resid_norm"],
                          "ms_per_fit": ols["t_total_ms"]},
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def pacf_bench(args, torch, synth, capi):
    """The PACF study of Section 4.1 on synthetic data: lags 1..250 of an
    AR(150) series with n = 2,000,000, every lag an AR(h) fit, all lags in
    one batched call; exact (OLS) and compressed (estimator SKETCH, 8h rows,
    2000 at the last lag) PACF; and LSAR (Algorithm 3, tls_lsar_device:
    the lags one after another, c = 2000 rows each, scores carried from lag
    to lag).  value: exact lag fits per second."""
    import oracle
    f = synth.WORKLOADS["pacf"](seed=0)
    y, pmax = f.y, f.p
    dy = torch.from_numpy(y).to("cuda:0")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ctx = capi.Context(0, precision=0)
    res = {}
    for name, opts in (("exact", {}), ("compressed", {"estimator": capi.EST_SKETCH})):
        for _ in range(args.warmup):
            ctx.pacf_device(dy, pmax, 1e-10, stream=stream, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s, tau, order, st = ctx.pacf_device(dy, pmax, 1e-10, stream=stream, **opts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = {"seconds": dt, "lag_fits_per_s": pmax / dt, "order": order,
                     "status": capi.status_string(s),
                     "lags_ok": int(np.sum(st == capi.TLS_OK)), "tau": tau}
        print(f"[bench] {name} PACF: {dt:.3f} s, order {order}", file=sys.stderr, flush=True)
    # LSAR (Algorithm 3): c = 2000 rows at every lag, as in the paper's study
    c_lsar = 2000
    for _ in range(args.warmup):
        ctx.lsar_device(dy, pmax, c_lsar, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        la = ctx.lsar_device(dy, pmax, c_lsar, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    res["lsar"] = {"seconds": dt, "lag_fits_per_s": pmax / dt, "order": la["order"],
                   "status": capi.status_string(la["status"]), "rows_per_lag": c_lsar,
                   "lags_ok": int(np.sum(la["lag_status"] == capi.TLS_OK)), "tau": la["pacf"]}
    print(f"[bench] LSAR PACF: {dt:.3f} s, order {la['order']}", file=sys.stderr, flush=True)
    diff = np.abs(res["exact"]["tau"] - res["compressed"]["tau"])
    # oracle on a bounded sample: the first lags on a prefix, timed on the host
    cpu = None
    if not args.no_cpu:
        nsub, lags = 1 << 18, 12
        t0 = time.perf_counter()
        ref = oracle.pacf(y[:nsub], lags)
        t = time.perf_counter() - t0
        sub = np.zeros(lags)
        for h in range(1, lags + 1):
            sub[h - 1] = ctx.fit(y[: nsub - lags + h], h, 1e-10)["coef"][h - 1]
        cost_sample = sum((nsub - lags) * (h + 1) ** 2 for h in range(1, lags + 1))
        cost_all = sum((y.size - pmax) * (h + 1) ** 2 for h in range(1, pmax + 1))
        cpu = {"value": pmax / (t * cost_all / cost_sample), "unit": "lag fits/s",
               "cores": lapack_threads(), "cpu_model": cpu_model(),
               "kind": "oracle",
               "sample": f"oracle.pacf of lags 1..{lags} on the first {nsub} samples in {t:.2f} s, "
                         f"scaled by the m (h+1)^2 cost of all {pmax} lags at full length",
               "max_abs_tau_diff_vs_gpu_on_sample": float(np.abs(ref - sub).max())}
        # the oracle's LSAR on the same kind of sample: its per-lag cost is a
        # residual over the rows (R h) and the compressed QR (c h^2)
        import oracle.lsar as olsar
        draws = [oracle.philox_uniform(c_lsar, capi.RNG_LEVERAGE, 0, 0, start=(h - 1) * c_lsar)
                 for h in range(1, lags + 1)]
        t0 = time.perf_counter()
        olsar.lsar_pacf(y[:nsub], lags, c_lsar, draws)
        t = time.perf_counter() - t0
        cost_sample = sum((nsub - lags) * h + c_lsar * h * h for h in range(1, lags + 1))
        cost_all = sum((y.size - pmax) * h + c_lsar * h * h for h in range(1, pmax + 1))
        cpu["lsar"] = {"value": pmax / (t * cost_all / cost_sample), "unit": "lag fits/s",
                       "sample": f"oracle.lsar.lsar_pacf of lags 1..{lags} on the first {nsub} "
                                 f"samples (c = {c_lsar}) in {t:.2f} s, scaled by the "
                                 f"R h + c h^2 cost of all {pmax} lags at full length"}
    line = {
        "metric": METRIC, "value": res["exact"]["lag_fits_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["exact"]["seconds"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["pacf"], "n": int(y.size), "lags": pmax,
                   "true_order": 150},
        "exact": {k: v for k, v in res["exact"].items() if k != "tau"},
        "compressed": {k: v for k, v in res["compressed"].items() if k != "tau"},
        "lsar": {k: v for k, v in res["lsar"].items() if k != "tau"},
        "max_abs_tau_diff_exact_vs_compressed": float(diff.max()),
        "max_abs_tau_diff_exact_vs_lsar": float(np.abs(res["exact"]["tau"]
                                                       - res["lsar"]["tau"]).max()),
        "paper_context": "the paper reports a ~700 s gap between exact and compressed PACF "
                         "for AR(150), n=2e6, 250 lags (MATLAB, 4-core laptop CPU)",
    }
    if cpu:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


def rh_bench(args, torch, synth, capi):
    """The LSAR-versus-RH comparison of Sections 4.1-4.2 on synthetic data:
    relative percentage coefficient error (100 ||phi_c - phi*|| / ||phi*||)
    of the compressed estimate at every lag 1..p against the exact fit of
    that lag, with and without outliers, and the time of each method's lags:
    LSAR (Algorithm 3: scores carried from lag to lag, c = 20p rows at every
    lag), repeated halving (Algorithm 4, 20h rows at lag h) and, for
    reference, the one-level generalised leverage sketch (eq. (glev) scores
    w.r.t. a uniform sketch, 20h rows).  value: LSAR lag fits/s on AR(100)."""
    models = (5, 20, 100)
    n = 2_000_000
    ctx = capi.Context(0, precision=0)
    stream = torch.cuda.current_stream()
    out, value = [], None
    for p in models:
        for outliers in (False, True):
            rng = np.random.default_rng(p)
            y = synth.ar_series(n, p, rng, 0.5, 0.95)
            if outliers:
                y = synth.add_outliers(y, np.random.default_rng(1000 + p), 1000)
            dy = torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0")
            lags = list(range(1, p + 1))
            ptrs = [dy[: n - p + h] for h in lags]  # prefix views, no copies
            res = {}
            for name, opts in (("exact", {}),
                               ("leverage1", {"estimator": capi.EST_SKETCH, "gamma": 20}),
                               ("rh", {"estimator": capi.EST_SKETCH, "gamma": 20,
                                       "sketch": capi.SKETCH_RH})):
                ctx.fit_batch_device(ptrs, lags, 1e-10, stream=stream, **opts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s, fits = ctx.fit_batch_device(ptrs, lags, 1e-10, stream=stream, **opts)
                torch.cuda.synchronize()
                res[name] = (time.perf_counter() - t0, fits, s)
            ctx.lsar_device(dy, p, 20 * p, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            la = ctx.lsar_device(dy, p, 20 * p, stream=stream)
            torch.cuda.synchronize()
            res["lsar"] = (time.perf_counter() - t0, [{"coef": ph} for ph in la["phi"]],
                           la["status"])
            ex = res["exact"][1]
            row = {"p": p, "outliers": outliers, "lags": len(lags)}
            for name in ("exact", "lsar", "rh", "leverage1"):
                t, fits, s = res[name]
                row[name + "_seconds"] = t
                row[name + "_status"] = capi.status_string(s)
                if name != "exact":
                    errs = [100 * np.linalg.norm(f["coef"] - e["coef"]) / np.linalg.norm(e["coef"])
                            for f, e in zip(fits, ex)]
                    row[name + "_mean_pct_err"] = float(np.mean(errs))
                    row[name + "_max_pct_err"] = float(np.max(errs))
            print(f"[bench] AR({p}) outliers={outliers}: exact {row['exact_seconds']:.3f} s, "
                  f"LSAR {row['lsar_seconds']:.3f} s err {row['lsar_mean_pct_err']:.2f}%, "
                  f"RH {row['rh_seconds']:.3f} s err {row['rh_mean_pct_err']:.2f}%, one-level "
                  f"{row['leverage1_seconds']:.3f} s err {row['leverage1_mean_pct_err']:.2f}%",
                  file=sys.stderr, flush=True)
            if p == models[-1] and not outliers:
                value = len(lags) / row["lsar_seconds"]
            out.append(row)
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": 1e3 / value, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["rh"], "value": "LSAR compressed lag fits/s, AR(100)"},
        "comparison": out,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def serve_bench(args, torch, synth, capi):
    """Open-loop served workload: one thread submits requests at their Poisson
    arrival times (series resident in device memory, borrowed by the server),
    another takes the results in order; value = completed requests per second
    over the timed window, with latency percentiles."""
    import threading

    import oracle
    duration = args.duration
    t0 = time.perf_counter()
    arrivals, which, pool = synth.workload_serve(seed=0, rate=args.rate, duration=duration + 2.0,
                                                 pool=args.pool)
    print(f"[bench] pool of {len(pool)} series ({sum(f.y.size for f in pool)} samples) generated in "
          f"{time.perf_counter() - t0:.1f} s; {arrivals.size} arrivals", file=sys.stderr, flush=True)
    dys = [torch.from_numpy(f.y).to("cuda:0") for f in pool]
    torch.cuda.synchronize()
    max_iter = args.max_iter or 200
    ctx = capi.Context(0, gamma=8, max_iter=max_iter)
    srv = capi.Server(ctx, args.serve_budget << 30, args.serve_slots, tick_steps=args.tick_steps)
    # warm-up: a burst of requests, all taken before the timed window
    warm = [srv.submit_device(dys[int(i)], pool[int(i)].p, 1e-10, request_id=10_000_000 + k)
            for k, i in enumerate(which[:args.warmup * 50])]
    for t in warm:
        srv.wait(t)
    print(f"[bench] warmup done ({len(warm)} requests)", file=sys.stderr, flush=True)

    results = [None] * arrivals.size
    tickets = [None] * arrivals.size
    ready = [threading.Event() for _ in range(arrivals.size)]
    sub_done = [0.0]

    def submitter(start):
        for k in range(arrivals.size):
            due = start + arrivals[k]
            while True:
                left = due - time.perf_counter()
                if left <= 0:
                    break
                if left > 5e-4:
                    time.sleep(left - 3e-4)
            i = int(which[k])
            tickets[k] = srv.submit_device(dys[i], pool[i].p, 1e-10, request_id=k)
            ready[k].set()
        sub_done[0] = time.perf_counter()

    def collector():
        for k in range(arrivals.size):
            ready[k].wait()
            results[k] = srv.wait(tickets[k])

    start = time.perf_counter() + 0.05
    ts = threading.Thread(target=submitter, args=(start,))
    tc = threading.Thread(target=collector)
    ts.start()
    tc.start()
    last_report = start
    while tc.is_alive():
        tc.join(timeout=5.0)
        now = time.perf_counter()
        if now - last_report >= 5.0 and tc.is_alive():
            st = srv.stats()
            print(f"[bench] t={now - start:.0f}s completed={st['completed']} in_flight={st['in_flight']} "
                  f"queued={st['queued']} ticks={st['ticks']}", file=sys.stderr, flush=True)
            last_report = now
    ts.join()
    end = time.perf_counter()
    stats = srv.stats()
    srv.close()
    lat = np.array([r["t_total_ms"] for r in results])
    statuses = [r["status"] for r in results]
    samples = int(sum(pool[int(i)].y.size for i in which))
    elapsed = end - start
    # agreement with the oracle on a sample of requests (series up to 2^17)
    errs = []
    for k in range(0, arrivals.size, max(1, arrivals.size // 40)):
        f = pool[int(which[k])]
        if f.y.size > (1 << 17):
            continue
        ref = oracle.fit_qr(f.y, f.p)
        errs.append((ref["kappa"], oracle.rel_error(results[k]["coef"], ref["phi"])))
    strata = {}
    for lo, hi, name in [(0, 1e6, "kappa<1e6"), (1e6, 1e12, "1e6<=kappa<1e12"),
                         (1e12, float("inf"), "kappa>=1e12")]:
        sel = [e for kk, e in errs if lo <= kk < hi]
        strata[name] = {"fits": len(sel), "within_1e-6": sum(e <= 1e-6 for e in sel),
                        "within_1e-4": sum(e <= 1e-4 for e in sel),
                        "max_rel_err": max(sel) if sel else None}
    cpu = None
    if not args.no_cpu:
        cost = [(f.y.size - f.p) * (f.p + 1) ** 2 for f in (pool[int(i)] for i in which)]
        tc0 = time.perf_counter()
        done = 0
        for i in which:
            f = pool[int(i)]
            oracle.fit_qr(f.y, f.p)
            done += 1
            if time.perf_counter() - tc0 > 15.0:
                break
        t = time.perf_counter() - tc0
        total = t * sum(cost) / sum(cost[:done])
        cpu = {"value": arrivals.size / total, "unit": "requests/s", "cores": lapack_threads(),
               "cpu_model": cpu_model(),
               "kind": "oracle",
               "sample": f"oracle.fit_qr on the first {done} of {arrivals.size} requests in {t:.1f} s, "
                         f"scaled by the m (p+1)^2 cost of all requests"}
    line = {
        "metric": METRIC, "value": arrivals.size / elapsed, "unit": "requests/s", "n_gpus": 1,
        "steps": int(arrivals.size), "warmup": len(warm), "ms_per_step": elapsed / arrivals.size * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["serve"], "offered_rate": args.rate,
                   "duration_s": duration, "pool_series": len(pool), "requests": int(arrivals.size),
                   "samples": samples, "hbm_budget_gib": args.serve_budget,
                   "max_slots": args.serve_slots, "max_iter": max_iter,
                   "tick_steps": args.tick_steps or 24,
                   "fit_statuses": {capi.status_string(k): statuses.count(k) for k in set(statuses)}},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                       "p99": float(np.percentile(lat, 99)), "mean": float(lat.mean()),
                       "max": float(lat.max())},
        "samples_per_s": samples / elapsed,
        "server": {"ticks": stats["ticks"], "ticks_per_s": stats["ticks"] / elapsed,
                   "submit_lag_s": sub_done[0] - (start + float(arrivals[-1]))},
        "accuracy": {"oracle_sample": len(errs), "by_kappa": strata},
    }
    if cpu:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


def time_fits(ctx, dy, p, tol, stream, torch, steps, warmup, **opts):
    """`warmup` untimed fits, then `steps` timed fits of the resident series.
    HIP events bracket every pass of the last tenth of the timed fits (at
    least one): they give the pass's launch durations, and since an event
    record between kernels adds a gap, the other fits run without them."""
    out = None
    for _ in range(warmup):
        out = ctx.fit_device(dy, p, tol, stream=stream, **opts)
    torch.cuda.synchronize()
    nprof = max(1, steps // 10)
    pass_ms, pass_count, pass_worked, iters = 0.0, 0, 0, []
    t0 = time.perf_counter()
    for i in range(steps):
        out = ctx.fit_device(dy, p, tol, stream=stream, profile=int(i >= steps - nprof), **opts)
        pass_ms += out["pass_ms"]
        pass_count += out["pass_count"]
        pass_worked += out["pass_worked"]
        iters.append(out["iters"])
    torch.cuda.synchronize()
    return {"out": out, "elapsed": time.perf_counter() - t0, "pass_ms": pass_ms,
            "pass_count": pass_count, "pass_worked": pass_worked, "iters": iters, "nprof": nprof}


def roofline_record(n, p, run, steps, prec, traffic, traffic_src):
    """Roofline of the dominant pass from the event-timed launches of `run`.
    Every launch is timed, including the few queued after a fit converged
    (they exit at once): bytes per launch is the algorithmic bytes of a
    working pass times the fraction of launches that worked."""
    out = run["out"]
    B, nb = out["block_len"], out["n_blocks"]
    if out["pass_kind"] == 0:
        bytes_pass = fused_pass_bytes(n, p, B, nb, 8)
        kernel_name = "toep_pass_kernel<double, fused>: e = X v - a u, X^T e, ||e||^2"
        if prec != 0:
            kernel_name += " (the FP64 LSQR of the mixed fit)"
    elif out["pass_kind"] == 2:
        bytes_pass = fused_pass_bytes(n, p, B, nb, 4)
        kernel_name = "toep_pass_kernel<float, fused>: e = X v - a u, X^T e, ||e||^2 (FP32 products)"
    else:
        # the CG pass reads only the FP32 spectra and writes the block partials
        bytes_pass = nb * (B // 2) * 8 + (B // 2) * 8 + (p + 1) * pass_groups(B, nb) * 8
        kernel_name = "toep_pass_kernel<float, fused>: X^T X v (CG normal-equation product)"
    cnt = max(run["pass_count"], 1)
    avg_pass_s = run["pass_ms"] / cnt / 1e3
    bytes_launch = bytes_pass * run["pass_worked"] / cnt
    achieved = bytes_launch / avg_pass_s / 1e9 if run["pass_count"] else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
            "kernel": kernel_name, "bytes_per_launch": bytes_launch,
            "bytes_per_working_launch": bytes_pass, "avg_launch_us": avg_pass_s * 1e6,
            "launches_timed": run["pass_count"], "launches_worked": run["pass_worked"],
            "timed_in": f"HIP events around every pass of the last {run['nprof']} of the "
                        f"{steps} timed fits"}


def hbm_resident_record(ctx, torch, synth, capi, stream, steps=3):
    """The fused FP64 pass on a working set far above the 256 MB Infinity
    Cache: the AR(500), n = 2^25 series (0.86 GB of spectra and u per pass),
    FP64 fits with every pass event-timed; counter traffic from the
    committed profile of that configuration."""
    t0 = time.perf_counter()
    f = synth.workload_ar500(seed=0)
    print(f"[bench] AR(500) n=2^25 series generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    dy = torch.from_numpy(f.y).to("cuda:0")
    run = time_fits(ctx, dy, f.p, f.tol, stream, torch, steps, 1, precision=0, gamma=f.gamma)
    traffic, src = read_hbm_profile("ar500", "f64")
    rec = roofline_record(f.y.size, f.p, run, steps, 0, traffic, src)
    rec["timed_in"] = f"HIP events around every pass of {steps} FP64 fits"
    mf = read_mfma_profile("ar500")
    if mf:
        rec["qr_fp64_mfma"] = mf
    rec.update({"workload": "AR(500), n=2^25, seed 0, FP64, sketch 8p rows, tol 1e-10",
                "iters": int(np.median(run["iters"])),
                "status": capi.status_string(run["out"]["status"]),
                "working_set_bytes": rec["bytes_per_working_launch"]})
    del dy
    torch.cuda.empty_cache()
    return rec


def lapack_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1]))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ar100", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="ar100: skip the 24p-sketch and HBM-resident AR(500) sub-records")
    ap.add_argument("--precision", default="f64", choices=["f64", "mixed"])
    ap.add_argument("--block-lg", type=int, default=0, help="log2 FFT block length (0 = automatic)")
    ap.add_argument("--n", type=int, default=0, help="override the series length")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=5000.0, help="serve: requests per second")
    ap.add_argument("--pool", type=int, default=512, help="serve: resident series in the pool")
    ap.add_argument("--serve-budget", type=int, default=64, help="serve: HBM budget in GiB")
    ap.add_argument("--serve-slots", type=int, default=8192, help="serve: fits in flight at most")
    ap.add_argument("--tick-steps", type=int, default=0,
                    help="serve: LSQR steps per tick (0: the library default, 24)")
    ap.add_argument("--max-iter", type=int, default=0,
                    help="LSQR iteration limit (0: the library default, 1000; serve default 200)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (calibrates the HBM "
                         "byte counters against a known size) and exit")
    ap.add_argument("--prof-summary", nargs="+", metavar="ARG",
                    help="KIND OUT TITLE CMD DIR...: summarise rocprofv3 CSV output and exit "
                         "(KIND 'stats', or 'hbm=<kernel prefix>@<copy bytes>' with the FETCH, "
                         "WRITE, copy-FETCH and copy-WRITE run directories)")
    args = ap.parse_args()
    if args.prof_summary:
        kind, out, title, cmd, *dirs = args.prof_summary
        prof_summary(kind, dirs, out, cmd, title)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); sharding a fit "
              "over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2112_12994_amd import capi

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batch":
        batch_bench(args, torch, synth, capi)
        return
    if args.workload == "serve":
        serve_bench(args, torch, synth, capi)
        return
    if args.workload == "sketch":
        sketch_bench(args, torch, synth, capi)
        return
    if args.workload == "pacf":
        pacf_bench(args, torch, synth, capi)
        return
    if args.workload == "rh":
        rh_bench(args, torch, synth, capi)
        return
    f = synth.WORKLOADS[args.workload](seed=0, **({"n": args.n} if args.n else {}))
    prec = 1 if args.precision == "mixed" else 0
    y, p = f.y, f.p
    print(f"[bench] workload {args.workload}: n={y.size} p={p}", file=sys.stderr, flush=True)
    dy = torch.from_numpy(y).to("cuda:0")
    torch.cuda.synchronize()
    ctx = capi.Context(0, gamma=f.gamma, precision=prec, block_lg=args.block_lg)
    stream = torch.cuda.current_stream()

    run = time_fits(ctx, dy, p, f.tol, stream, torch, args.steps, args.warmup)
    out = run["out"]
    print(f"[bench] timed {args.steps} steps in {run['elapsed']:.4f} s", file=sys.stderr, flush=True)
    B, nb = out["block_len"], out["n_blocks"]
    traffic, traffic_src = None, "non-default configuration"
    if not args.block_lg and not args.n:
        traffic, traffic_src = read_hbm_profile(
            args.workload, args.precision,
            "toep_pass_kernel<double" if out["pass_kind"] == 0 else "toep_pass_kernel<float")
    roof = roofline_record(y.size, p, run, args.steps, prec, traffic, traffic_src)
    elapsed = run["elapsed"]
    iters = run["iters"]
    if args.workload == "ar500":
        ref = ctx.fit_device(dy, p, f.tol, stream=stream, precision=0)
        acc = gpu_fp64_agreement(y, p, out, ref)
    else:
        acc = accuracy(y, p, out["coef"], out["resid_norm"], args.workload)

    line = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32 products, f64 recurrences",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "n": int(y.size), "p": p,
                   "sketch_rows": out["sketch_rows"], "sketch_gamma": f.gamma,
                   "fft_block": B, "fft_blocks": nb,
                   "precision": args.precision, "iters": int(np.median(iters)),
                   "refine_steps": out["refine_steps"], "kappa_est_R": out["kappa_est"],
                   "status": capi.status_string(out["status"])},
        "roofline": roof,
        "accuracy": acc,
    }
    mf = read_mfma_profile(args.workload) if not args.block_lg and not args.n else None
    if mf:
        line["qr_fp64_mfma"] = mf
    if args.workload == "ar100" and not args.n and not args.block_lg and not args.no_extras:
        # the same series on a 24p-row sketch: fewer LSQR iterations for a larger QR
        r24 = time_fits(ctx, dy, p, f.tol, stream, torch, args.steps, args.warmup, gamma=24)
        line["sketch_24p"] = {
            "what": "the same fit with a 24p-row sketch (not the configured 8p)",
            "value": args.steps / r24["elapsed"], "unit": "solves/s",
            "ms_per_step": r24["elapsed"] / args.steps * 1e3,
            "iters": int(np.median(r24["iters"])), "sketch_rows": r24["out"]["sketch_rows"],
            "roofline_frac": roofline_record(y.size, p, r24, args.steps, prec, None, "")["frac"]}
        del dy
        torch.cuda.empty_cache()
        line["hbm_resident"] = hbm_resident_record(ctx, torch, synth, capi, stream)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(y, p)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
