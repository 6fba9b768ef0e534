"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/tls.h declares, and validates arguments before touching a device."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tls.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tls_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def capi():
    from paper_2112_12994_amd import capi as c
    return c


def test_every_declared_symbol_is_exported(capi):
    names = _declared()
    assert "tls_fit" in names and "tls_op_toeplitz" in names
    for name in names:
        assert hasattr(capi.lib, name), name
    # and the binding covers every declared entry point with a signature
    assert set(names) <= set(capi.EXPORTED)


def test_status_strings(capi):
    assert capi.status_string(capi.TLS_OK) == "ok"
    assert "rank" in capi.status_string(capi.TLS_ERANK)
    assert capi.status_string(99) == "unknown status"


def test_option_and_tuning_layout(capi):
    """The binding's option struct has the header's size, and its table index
    uses the library's buckets: ceil(log2 p), ceil(log2 m) clamped to 40."""
    import ctypes
    assert ctypes.sizeof(capi.TlsOptions) == 10 * 4 + 2 * 8 + 2 * 4 + 3 * 8
    assert capi.TUNE_ENTRIES == 2 * 11 * 41
    assert capi.tune_index(capi.PREC_F64, 1, 1) == 0
    assert capi.tune_index(capi.PREC_F64, 100, 4194204) == 7 * 41 + 22
    assert capi.tune_index(capi.PREC_F64, 64, 1 << 12) == 6 * 41 + 12
    assert capi.tune_index(capi.PREC_MIXED, 65, (1 << 12) + 1) == (11 + 7) * 41 + 13
    assert capi.tune_index(capi.PREC_F64, 1024, 1 << 50) == 10 * 41 + 40


def test_default_options(capi):
    o = capi.options()
    assert (o.precision, o.sketch, o.jl_kind, o.gamma, o.jl_k, o.max_iter, o.warm_start,
            o.no_graph) == (0, 0, 0, 8, 8, 1000, 1, 0)
    with pytest.raises(TypeError):
        capi.options(bogus=1)


@pytest.mark.parametrize("n,p,B,expect", [
    (10000, 3, 256, -(-9997 // 254)),
    (200, 3, 128, 2),
    (1000, 100, 128, -1),   # B < 2p
    (1000, 3, 100, -1),     # not a power of two
    (1000, 3, 1 << 15, -1), # above the largest block
    (3, 3, 128, -1),        # no rows
])
def test_num_blocks(capi, n, p, B, expect):
    assert capi.num_blocks(n, p, B) == expect


def test_fit_validates_before_device(capi):
    y = np.random.default_rng(0).standard_normal(100)
    assert capi.tls_fit(y, 0, 1e-10)[0] == capi.TLS_EINVAL
    assert capi.tls_fit(y, 50, 1e-10)[0] == capi.TLS_EINVAL          # n < 2p + 1
    assert capi.tls_fit(y, 3, 0.0)[0] == capi.TLS_EINVAL
    assert capi.tls_fit(y, 3, 1.5)[0] == capi.TLS_EINVAL
    assert capi.tls_fit(y, 3, float("nan"))[0] == capi.TLS_EINVAL
    yb = y.copy()
    yb[5] = np.inf
    assert capi.tls_fit(yb, 3, 1e-10)[0] == capi.TLS_EINVAL
    big = np.zeros(5000)
    assert capi.tls_fit(big, 2000, 1e-10)[0] == capi.TLS_EUNSUPPORTED  # p above the limit


def test_library_path_is_in_tree(capi):
    assert os.path.dirname(capi.LIB_PATH) == os.path.join(ROOT, "paper_2112_12994_amd")
