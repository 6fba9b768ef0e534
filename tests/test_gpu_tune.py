"""Block-length autotuner (tls_autotune, tls_get_tuning, tls_set_tuning):
the table holds admissible lengths for the measured buckets, fits on the
tuned context take their block length from it, and a tuned fit equals, bit
for bit, the same fit with that length given explicitly, alone and in a
batch; a stored table reproduces the results in another context."""
import numpy as np
import pytest

import synth
from tests.gpu_common import capi, say, to_dev

pytestmark = pytest.mark.gpu


def _fits(seed, ps, ns):
    rng = np.random.default_rng(seed)
    return [(synth.ar_series(int(n), p, rng, 0.3, 0.9), p) for p, n in zip(ps, ns)]


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_table_drives_block_length(prec):
    c = capi()
    say("autotune", prec)
    with c.Context(0) as ctx:
        k = ctx.autotune(prec, 4, 64, 1 << 12, 1 << 16)
        t = ctx.tuning()
        say("   entries", k, "distinct lengths", sorted(set(int(x) for x in t if x)))
        assert k > 0 and int(np.count_nonzero(t)) == k
        for pb in range(2, 7):
            for mb in range(12, 17):
                lg = int(t[(prec * c.TUNE_PBUCKETS + pb) * c.TUNE_MBUCKETS + mb])
                if lg:
                    assert 7 <= lg <= 14 and (1 << lg) >= 2 * (1 << pb)
        for y, p in _fits(20 + prec, [5, 33, 60], [5000, 40000, 60000]):
            lg = int(t[c.tune_index(prec, p, y.size - p)])
            assert lg > 0
            out = ctx.fit(y, p, 1e-10, precision=prec, request_id=p)
            assert out["block_len"] == 1 << lg
            ref = ctx.fit(y, p, 1e-10, precision=prec, request_id=p, block_lg=lg)
            assert out["coef"].tobytes() == ref["coef"].tobytes()
            assert out["iters"] == ref["iters"]


def test_tuned_batch_equals_single_and_table_transfers():
    c = capi()
    say("autotune batch")
    work = _fits(30, [4, 17, 40, 64, 9, 50], [4096, 20000, 90000, 150000, 3000, 60000])
    ys, ps = [y for y, _ in work], [p for _, p in work]
    with c.Context(0) as ctx:
        ctx.autotune(0, 4, 64, 1 << 12, 1 << 18)
        table = ctx.tuning()
        s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=5)
        assert s == c.TLS_OK
        for i, (y, p) in enumerate(work):
            single = ctx.fit(y, p, 1e-10, request_id=5 + i)
            assert outs[i]["coef"].tobytes() == single["coef"].tobytes()
            assert outs[i]["block_len"] == single["block_len"]
    with c.Context(0) as ctx2:
        assert ctx2.set_tuning(table) == c.TLS_OK
        assert np.array_equal(ctx2.tuning(), table)
        s, outs2 = ctx2.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=5)
        for a, b in zip(outs, outs2):
            assert a["coef"].tobytes() == b["coef"].tobytes()


def test_tuning_rejects_bad_input():
    c = capi()
    with c.Context(0) as ctx:
        t = np.zeros(c.TUNE_ENTRIES, dtype=np.int8)
        t[5] = 3  # below the shortest block
        assert ctx.set_tuning(t) == c.TLS_EINVAL
        assert not ctx.tuning().any()
        for args in [(2, 4, 64, 1 << 12, 1 << 14), (0, 0, 8, 100, 200), (0, 9, 8, 100, 200),
                     (0, 4, 2000, 1 << 20, 1 << 21), (0, 4, 64, 100, 1 << 14),
                     (0, 4, 64, 1 << 14, 1 << 12)]:
            with pytest.raises(c.TlsError) as e:
                ctx.autotune(*args)
            assert e.value.status == c.TLS_EINVAL
