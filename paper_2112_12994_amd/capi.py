"""ctypes binding of libtls.so: the C-ABI of include/tls.h under the same names.

Argument marshalling only; every step of a fit runs in the HIP library.
Device buffers are torch tensors on a ROCm device (torch is used for device
memory and streams only); host buffers are NumPy arrays.  Importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtls.so")

(TLS_OK, TLS_EINVAL, TLS_ERANK, TLS_ENOCONV, TLS_ENOMEM, TLS_EDEVICE, TLS_EUNSUPPORTED,
 TLS_EAGAIN, TLS_ESTALL) = range(9)
PREC_F64, PREC_MIXED = 0, 1
SKETCH_LEVERAGE, SKETCH_UNIFORM, SKETCH_RH = 0, 1, 2
JL_SRHT, JL_GAUSS = 0, 1
EST_OLS, EST_SKETCH = 0, 1

# Philox stream numbers of one fit (include/tls.h, tls_op_* documentation)
RNG_UNIFORM_ROWS, RNG_SRHT_SIGNS, RNG_SRHT_ROWS, RNG_LEVERAGE, RNG_GAUSS, RNG_RH_LEVEL = range(6)
TUNE_PRECS, TUNE_PBUCKETS, TUNE_MBUCKETS = 2, 11, 41
TUNE_ENTRIES = TUNE_PRECS * TUNE_PBUCKETS * TUNE_MBUCKETS


def tune_index(precision: int, p: int, m: int) -> int:
    """Index of the table entry that a fit of order p and m = n - p rows uses."""
    pb = max(0, (int(p) - 1).bit_length())
    mb = min(max(0, (int(m) - 1).bit_length()), TUNE_MBUCKETS - 1)
    return ((1 if precision == PREC_MIXED else 0) * TUNE_PBUCKETS + pb) * TUNE_MBUCKETS + mb


class TlsOptions(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("sketch", ctypes.c_int32),
        ("jl_kind", ctypes.c_int32),
        ("gamma", ctypes.c_int32),
        ("jl_k", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("block_lg", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
        ("max_refine", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("request_id", ctypes.c_uint64),
        ("no_graph", ctypes.c_int32),
        ("tick_steps", ctypes.c_int32),
        ("estimator", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
        ("reserved", ctypes.c_int64 * 2),
    ]


class TlsServerStats(ctypes.Structure):
    _fields_ = [
        ("ticks", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("queued", ctypes.c_uint64),
        ("in_flight", ctypes.c_uint64),
        ("arena_bytes_in_use", ctypes.c_uint64),
        ("arena_bytes", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class TlsResult(ctypes.Structure):
    _fields_ = [
        ("resid_norm", ctypes.c_double),
        ("kappa_est", ctypes.c_double),
        ("lsqr_rnorm", ctypes.c_double),
        ("lsqr_arnorm", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("istop", ctypes.c_int32),
        ("refine_steps", ctypes.c_int32),
        ("sketch_rows", ctypes.c_int32),
        ("block_len", ctypes.c_int32),
        ("n_blocks", ctypes.c_int32),
        ("t_total_ms", ctypes.c_double),
        ("pass_ms", ctypes.c_double),
        ("pass_count", ctypes.c_int32),
        ("pass_worked", ctypes.c_int32),
        ("pass_kind", ctypes.c_int32),
        ("mixed_path", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("reserved")}


def _hip_runtimes():
    """Paths of every libamdhip64 mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2112_12994_amd.build)")
    # torch (device memory and streams) carries its own HIP runtime with the
    # same soname as the system one; loading torch first makes the library
    # bind to that runtime, so torch's device pointers and streams are valid
    # in library calls.  Two runtimes in one process would not share them.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    handle = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError(f"two HIP runtimes mapped into the process: {sorted(runtimes)}")
    return handle


lib = _load()

_c = ctypes
_vp = _c.c_void_p
_dp = _c.POINTER(_c.c_double)
_i32 = _c.c_int32
_i64 = _c.c_int64
_u32 = _c.c_uint32
_u64 = _c.c_uint64
_ctxp = _c.c_void_p

_SIGS = {
    "tls_status_string": (_c.c_char_p, [_i32]),
    "tls_options_default": (None, [_c.POINTER(TlsOptions)]),
    "tls_create": (_i32, [_c.POINTER(_ctxp), _c.c_int, _c.POINTER(TlsOptions)]),
    "tls_destroy": (None, [_ctxp]),
    "tls_fit": (_i32, [_dp, _i64, _i32, _c.c_double, _dp, _dp, _c.POINTER(_i32)]),
    "tls_fit_ex": (_i32, [_ctxp, _dp, _i64, _i32, _c.c_double, _c.POINTER(TlsOptions), _dp,
                          _c.POINTER(TlsResult)]),
    "tls_fit_device": (_i32, [_ctxp, _vp, _i64, _i32, _c.c_double, _c.POINTER(TlsOptions), _vp,
                              _dp, _c.POINTER(TlsResult)]),
    "tls_fit_batch": (_i32, [_ctxp, _i32, _c.POINTER(_dp), _c.POINTER(_i64), _c.POINTER(_i32),
                             _c.c_double, _c.POINTER(TlsOptions), _dp, _c.POINTER(_i64), _dp,
                             _c.POINTER(_i32), _c.POINTER(_i32)]),
    "tls_fit_batch_device": (_i32, [_ctxp, _i32, _c.POINTER(_vp), _c.POINTER(_i64),
                                    _c.POINTER(_i32), _c.c_double, _c.POINTER(TlsOptions), _vp,
                                    _dp, _c.POINTER(_i64), _c.POINTER(TlsResult),
                                    _c.POINTER(_i32)]),
    "tls_server_create": (_i32, [_ctxp, _c.c_size_t, _i32, _c.POINTER(TlsOptions),
                                 _c.POINTER(_vp)]),
    "tls_submit": (_i32, [_vp, _dp, _i64, _i32, _c.c_double, _u64, _c.POINTER(_u64)]),
    "tls_submit_device": (_i32, [_vp, _vp, _i64, _i32, _c.c_double, _u64, _c.POINTER(_u64)]),
    "tls_poll": (_i32, [_vp, _u64, _dp, _c.POINTER(TlsResult), _c.POINTER(_i32)]),
    "tls_wait": (_i32, [_vp, _u64, _dp, _c.POINTER(TlsResult), _c.POINTER(_i32)]),
    "tls_server_get_stats": (_i32, [_vp, _c.POINTER(TlsServerStats)]),
    "tls_server_destroy": (None, [_vp]),
    "tls_pacf_device": (_i32, [_ctxp, _vp, _i64, _i32, _c.c_double, _c.POINTER(TlsOptions), _vp,
                               _dp, _c.POINTER(_i32), _c.POINTER(_i32)]),
    "tls_lsar_device": (_i32, [_ctxp, _vp, _i64, _i32, _i32, _c.POINTER(TlsOptions), _vp, _dp,
                               _c.POINTER(_i32), _dp, _c.POINTER(_i64), _c.POINTER(_i32), _vp]),
    "tls_autotune": (_i32, [_ctxp, _i32, _i32, _i32, _i64, _i64, _c.POINTER(_i32)]),
    "tls_get_tuning": (_i32, [_ctxp, _c.POINTER(_c.c_int8)]),
    "tls_set_tuning": (_i32, [_ctxp, _c.POINTER(_c.c_int8)]),
    "tls_num_blocks": (_i64, [_i64, _i32, _i32]),
    "tls_op_spectra": (_i32, [_ctxp, _i32, _vp, _i64, _i32, _i32, _vp, _vp]),
    "tls_op_toeplitz": (_i32, [_ctxp, _i32, _vp, _i64, _i32, _i32, _dp, _c.c_double, _c.c_double,
                               _vp, _vp, _vp, _i32, _vp, _vp]),
    "tls_op_toeplitz_noalloc": (_i32, [_ctxp, _i32, _vp, _i64, _i32, _i32, _dp, _c.c_double,
                                       _c.c_double, _vp, _vp, _vp, _i32, _vp, _vp]),
    "tls_op_scores": (_i32, [_ctxp, _i32, _vp, _i64, _i32, _i32, _vp, _i32, _vp, _vp]),
    "tls_op_sample": (_i32, [_ctxp, _i32, _vp, _i64, _vp, _i32, _u64, _u32, _vp, _vp, _vp]),
    "tls_op_rh_mask": (_i32, [_ctxp, _i32, _vp, _i64, _i32, _u64, _u32, _vp]),
    "tls_op_gather": (_i32, [_ctxp, _vp, _i64, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _u64,
                             _u32, _vp]),
    "tls_op_qr": (_i32, [_ctxp, _vp, _i32, _i32, _i32, _vp, _c.POINTER(_i32), _vp]),
    "tls_op_triinv": (_i32, [_ctxp, _vp, _i32, _i32, _vp, _vp, _vp]),
    "tls_op_jl": (_i32, [_ctxp, _vp, _i32, _i32, _i32, _i32, _u64, _u32, _vp, _vp, _vp]),
    "tls_op_philox": (_i32, [_ctxp, _u64, _u32, _u32, _u64, _i64, _vp, _vp]),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class TlsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


def status_string(s: int) -> str:
    return lib.tls_status_string(int(s)).decode()


def _check(s: int, what: str):
    if s != TLS_OK:
        raise TlsError(s, what)


def options(**kw) -> TlsOptions:
    o = TlsOptions()
    lib.tls_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k!r}")
        setattr(o, k, v)
    return o


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _stream(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


# ---- plain calls ------------------------------------------------------------

def tls_fit(series, p: int, tol: float = 1e-10):
    """(status, coef, resid_norm, iters) with the default context."""
    y = np.ascontiguousarray(series, dtype=np.float64)
    coef = np.zeros(p)
    rn = ctypes.c_double(0.0)
    it = _i32(0)
    s = lib.tls_fit(_dptr(y), y.size, p, tol, _dptr(coef), ctypes.byref(rn), ctypes.byref(it))
    return s, coef, rn.value, it.value


class Context:
    """A tls_ctx: one device, its own stream and workspace."""

    def __init__(self, device: int = 0, **opts):
        self._h = ctypes.c_void_p()
        self.opts = options(**opts)
        _check(lib.tls_create(ctypes.byref(self._h), device, ctypes.byref(self.opts)), "tls_create")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib.tls_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _opt(self, kw):
        if not kw:
            return self.opts
        o = TlsOptions.from_buffer_copy(self.opts)
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k!r}")
            setattr(o, k, v)
        return o

    def fit(self, series, p: int, tol: float = 1e-10, **opts):
        """tls_fit_ex on a host series: dict(status, coef, result fields)."""
        y = np.ascontiguousarray(series, dtype=np.float64)
        coef = np.zeros(p)
        res = TlsResult()
        o = self._opt(opts)
        s = lib.tls_fit_ex(self._h, _dptr(y), y.size, p, tol, ctypes.byref(o), _dptr(coef),
                           ctypes.byref(res))
        out = res.as_dict()
        out.update(status=s, coef=coef)
        return out

    def fit_device(self, d_series, p: int, tol: float = 1e-10, stream=None, **opts):
        """tls_fit_device on a torch float64 device tensor."""
        coef = np.zeros(p)
        res = TlsResult()
        o = self._opt(opts)
        s = lib.tls_fit_device(self._h, _ptr(d_series), d_series.numel(), p, tol, ctypes.byref(o),
                               _stream(stream), _dptr(coef), ctypes.byref(res))
        out = res.as_dict()
        out.update(status=s, coef=coef)
        return out

    def fit_batch(self, series_list, p_list, tol: float = 1e-10, **opts):
        """tls_fit_batch: list of dicts (status, coef, resid_norm, iters)."""
        count = len(series_list)
        ys = [np.ascontiguousarray(y, dtype=np.float64) for y in series_list]
        ptrs = (_dp * count)(*[_dptr(y) for y in ys])
        ns = np.array([y.size for y in ys], dtype=np.int64)
        ps = np.array(p_list, dtype=np.int32)
        off = np.zeros(count, dtype=np.int64)
        if count:
            off[1:] = np.cumsum(ps[:-1])
        coef = np.zeros(int(ps.sum()) if count else 0)
        rn = np.zeros(count)
        its = np.zeros(count, dtype=np.int32)
        sts = np.zeros(count, dtype=np.int32)
        o = self._opt(opts)
        s = lib.tls_fit_batch(self._h, count, ptrs, ns.ctypes.data_as(_c.POINTER(_i64)),
                              ps.ctypes.data_as(_c.POINTER(_i32)), tol, ctypes.byref(o),
                              _dptr(coef), off.ctypes.data_as(_c.POINTER(_i64)), _dptr(rn),
                              its.ctypes.data_as(_c.POINTER(_i32)),
                              sts.ctypes.data_as(_c.POINTER(_i32)))
        outs = [{"status": int(sts[i]), "coef": coef[off[i]: off[i] + ps[i]].copy(),
                 "resid_norm": float(rn[i]), "iters": int(its[i])} for i in range(count)]
        return s, outs

    def fit_batch_device(self, d_series_list, p_list, tol: float = 1e-10, stream=None, **opts):
        """tls_fit_batch_device on torch float64 device tensors: (status,
        list of dicts with status, coef and the result fields)."""
        count = len(d_series_list)
        ptrs = (_vp * count)(*[_ptr(t) for t in d_series_list])
        ns = np.array([t.numel() for t in d_series_list], dtype=np.int64)
        ps = np.array(p_list, dtype=np.int32)
        off = np.zeros(count, dtype=np.int64)
        if count:
            off[1:] = np.cumsum(ps[:-1])
        coef = np.zeros(int(ps.sum()) if count else 0)
        res = (TlsResult * max(count, 1))()
        sts = np.zeros(count, dtype=np.int32)
        o = self._opt(opts)
        s = lib.tls_fit_batch_device(self._h, count, ptrs, ns.ctypes.data_as(_c.POINTER(_i64)),
                                     ps.ctypes.data_as(_c.POINTER(_i32)), tol, ctypes.byref(o),
                                     _stream(stream), _dptr(coef),
                                     off.ctypes.data_as(_c.POINTER(_i64)), res,
                                     sts.ctypes.data_as(_c.POINTER(_i32)))
        outs = []
        for i in range(count):
            d = res[i].as_dict()
            d.update(status=int(sts[i]), coef=coef[off[i]: off[i] + ps[i]].copy())
            outs.append(d)
        return s, outs

    # ---- step-level calls (torch device tensors) ----------------------------

    def op_spectra(self, prec, d_y, p, B, d_spec, stream=None):
        return lib.tls_op_spectra(self._h, prec, _ptr(d_y), d_y.numel(), p, B, _ptr(d_spec),
                                  _stream(stream))

    def op_toeplitz(self, prec, d_spec, n, p, B, v=None, s1=1.0, s2=0.0, d_w=None, d_e=None,
                    d_u_in=None, want_rmv=True, d_out=None, stream=None):
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        return lib.tls_op_toeplitz(self._h, prec, _ptr(d_spec), n, p, B,
                                   None if vv is None else _dptr(vv), s1, s2, _ptr(d_w), _ptr(d_e),
                                   _ptr(d_u_in), 1 if want_rmv else 0, _ptr(d_out), _stream(stream))

    def op_toeplitz_noalloc(self, prec, d_spec, n, p, B, v=None, s1=1.0, s2=0.0, d_w=None,
                            d_e=None, d_u_in=None, want_rmv=True, d_out=None, stream=None):
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        return lib.tls_op_toeplitz_noalloc(self._h, prec, _ptr(d_spec), n, p, B,
                                           None if vv is None else _dptr(vv), s1, s2, _ptr(d_w),
                                           _ptr(d_e), _ptr(d_u_in), 1 if want_rmv else 0,
                                           _ptr(d_out), _stream(stream))

    def op_scores(self, prec, d_spec, n, p, B, d_omega, k, d_scores, stream=None):
        return lib.tls_op_scores(self._h, prec, _ptr(d_spec), n, p, B, _ptr(d_omega), k,
                                 _ptr(d_scores), _stream(stream))

    def op_sample(self, prec, d_scores, m, d_u, c, seed, fit, d_idx, d_scale, stream=None):
        return lib.tls_op_sample(self._h, prec, _ptr(d_scores), m, _ptr(d_u), c, seed, fit,
                                 _ptr(d_idx), _ptr(d_scale), _stream(stream))

    def op_gather(self, d_y, p, mode, d_idx, d_scale, c, crows, ldq, d_A, seed=0, fit=0,
                  stream=None):
        return lib.tls_op_gather(self._h, _ptr(d_y), d_y.numel(), p, mode, _ptr(d_idx),
                                 _ptr(d_scale), c, crows, ldq, _ptr(d_A), seed, fit, _stream(stream))

    def pacf_device(self, d_series, pmax: int, tol: float = 1e-10, stream=None, **opts):
        """tls_pacf_device: (status, pacf[pmax], order, per-lag statuses)."""
        pacf = np.zeros(pmax)
        order = _i32(0)
        st = np.zeros(pmax, dtype=np.int32)
        o = self._opt(opts)
        s = lib.tls_pacf_device(self._h, _ptr(d_series), d_series.numel(), pmax, tol,
                                ctypes.byref(o), _stream(stream), _dptr(pacf), ctypes.byref(order),
                                st.ctypes.data_as(ctypes.POINTER(_i32)))
        return s, pacf, order.value, st

    def lsar_device(self, d_series, pmax: int, c: int, stream=None, d_scores=None, **opts):
        """tls_lsar_device: dict with status, pacf[pmax], order, phi (list: lag h's
        coefficients), rows (pmax x c sampled rows), lag_status[pmax]; the last
        lag's scores go to the device tensor d_scores when given."""
        pacf = np.zeros(pmax)
        order = _i32(0)
        phi = np.zeros(pmax * (pmax + 1) // 2)
        rows = np.zeros((pmax, c), dtype=np.int64)
        st = np.zeros(pmax, dtype=np.int32)
        o = self._opt(opts)
        s = lib.tls_lsar_device(self._h, _ptr(d_series), d_series.numel(), pmax, c,
                                ctypes.byref(o), _stream(stream), _dptr(pacf), ctypes.byref(order),
                                _dptr(phi), rows.ctypes.data_as(ctypes.POINTER(_i64)),
                                st.ctypes.data_as(ctypes.POINTER(_i32)), _ptr(d_scores))
        phis = [phi[h * (h - 1) // 2: h * (h - 1) // 2 + h].copy() for h in range(1, pmax + 1)]
        return {"status": s, "pacf": pacf, "order": order.value, "phi": phis, "rows": rows,
                "lag_status": st}

    def autotune(self, precision: int, p_min: int, p_max: int, n_min: int, n_max: int) -> int:
        """Measure block lengths on the device; returns the table entries written."""
        k = _i32(0)
        _check(lib.tls_autotune(self._h, precision, p_min, p_max, n_min, n_max, ctypes.byref(k)),
               "tls_autotune")
        return k.value

    def tuning(self):
        """The autotuned table, int8[TLS_TUNE_ENTRIES] (0 = not tuned)."""
        import numpy as np
        t = np.zeros(TUNE_ENTRIES, dtype=np.int8)
        _check(lib.tls_get_tuning(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))),
               "tls_get_tuning")
        return t

    def set_tuning(self, table) -> int:
        import numpy as np
        t = np.ascontiguousarray(table, dtype=np.int8)
        if t.size != TUNE_ENTRIES:
            raise ValueError("tuning table must have %d entries" % TUNE_ENTRIES)
        return lib.tls_set_tuning(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))

    def op_rh_mask(self, prec, d_scores, m, level, seed, fit, stream=None):
        return lib.tls_op_rh_mask(self._h, prec, _ptr(d_scores), m, level, seed, fit,
                                  _stream(stream))

    def op_qr(self, d_A, crows, q, ldq, d_R, stream=None):
        st = _i32(0)
        s = lib.tls_op_qr(self._h, _ptr(d_A), crows, q, ldq, _ptr(d_R), ctypes.byref(st),
                          _stream(stream))
        return s, st.value

    def op_triinv(self, d_R, q, p, d_M, d_phi0=None, stream=None):
        return lib.tls_op_triinv(self._h, _ptr(d_R), q, p, _ptr(d_M), _ptr(d_phi0), _stream(stream))

    def op_jl(self, d_R, q, p, k, kind, seed, fit, d_Pi, d_omega, stream=None):
        return lib.tls_op_jl(self._h, _ptr(d_R), q, p, k, kind, seed, fit, _ptr(d_Pi),
                             _ptr(d_omega), _stream(stream))

    def op_philox(self, seed, rng_stream, fit, start, count, d_out, stream=None):
        return lib.tls_op_philox(self._h, seed, rng_stream, fit, start, count, _ptr(d_out),
                                 _stream(stream))


class Server:
    """A tls_server on a Context: submit fits at any time, take results by
    ticket.  Device series are borrowed: the tensor is kept referenced here
    until its result is taken."""

    def __init__(self, ctx: "Context", hbm_budget: int, max_slots: int = 4096, **opts):
        self._h = ctypes.c_void_p()
        self.ctx = ctx
        o = ctx._opt(opts)
        _check(lib.tls_server_create(ctx.handle, hbm_budget, max_slots, ctypes.byref(o),
                                     ctypes.byref(self._h)), "tls_server_create")
        self._p = {}
        self._keep = {}

    def submit(self, series, p: int, tol: float = 1e-10, request_id: int = 0) -> int:
        """Host series (copied); returns the ticket, raises TlsError on rejection."""
        y = np.ascontiguousarray(series, dtype=np.float64)
        t = _u64(0)
        _check(lib.tls_submit(self._h, _dptr(y), y.size, p, tol, request_id, ctypes.byref(t)),
               "tls_submit")
        self._p[t.value] = p
        return t.value

    def submit_device(self, d_series, p: int, tol: float = 1e-10, request_id: int = 0) -> int:
        """torch float64 device tensor (borrowed until the result is taken)."""
        t = _u64(0)
        _check(lib.tls_submit_device(self._h, _ptr(d_series), d_series.numel(), p, tol, request_id,
                                     ctypes.byref(t)), "tls_submit_device")
        self._p[t.value] = p
        self._keep[t.value] = d_series
        return t.value

    def _take(self, fn, ticket: int):
        p = self._p.get(ticket, 0)
        coef = np.zeros(max(p, 1))
        res = TlsResult()
        st = _i32(0)
        s = fn(self._h, ticket, _dptr(coef), ctypes.byref(res), ctypes.byref(st))
        if s == TLS_EAGAIN:
            return None
        _check(s, "tls_wait/poll")
        self._p.pop(ticket, None)
        self._keep.pop(ticket, None)
        out = res.as_dict()
        out.update(status=st.value, coef=coef[:p])
        return out

    def poll(self, ticket: int):
        """Result dict, or None while in flight."""
        return self._take(lib.tls_poll, ticket)

    def wait(self, ticket: int):
        return self._take(lib.tls_wait, ticket)

    def stats(self) -> dict:
        s = TlsServerStats()
        _check(lib.tls_server_get_stats(self._h, ctypes.byref(s)), "tls_server_get_stats")
        return {f: getattr(s, f) for f, _ in s._fields_ if f != "reserved"}

    def close(self):
        if self._h:
            lib.tls_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def num_blocks(n: int, p: int, B: int) -> int:
    return int(lib.tls_num_blocks(n, p, B))
