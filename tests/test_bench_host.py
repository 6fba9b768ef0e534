"""Host-side logic of bench.py: the algorithmic byte count of the fused pass,
the source-hash gate on the committed HBM counter summary, the rocprofv3
kernel-statistics summary, and the one-GPU refusal."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

import bench


def test_fused_pass_bytes_ar100():
    # n = 2^22, p = 100, B = 1024 (512 complex bins), 4535 blocks taken 4
    # at a time (1134 groups), FP64: spectra 4535*512*16, u read + written
    # 2*(2^22-100)*8, v's spectrum 512*16, partial sums 101*1134*8
    expect = 4535 * 512 * 16 + 2 * (4194304 - 100) * 8 + 512 * 16 + 101 * 1134 * 8
    assert expect == 105182448
    assert bench.fused_pass_bytes(1 << 22, 100, 1024, 4535, 8) == expect


def _profile(path, source_hash, value, kernel="toep_pass_kernel<double, 9, 64, 3>"):
    with open(path, "w") as fh:
        fh.write("# test profile\n")
        fh.write(f"source_hash: {source_hash}\n")
        fh.write(f"kernel: {kernel}\n")
        fh.write(f"hbm_bytes_per_dispatch: {value}\n")


def test_hbm_profile_gate(tmp_path, monkeypatch):
    path = str(tmp_path / "prof.txt")
    monkeypatch.setattr(bench, "hbm_profile_name", lambda w, p: path)
    assert bench.read_hbm_profile("ar100", "f64") == (None, "no counter profile")
    _profile(path, bench.pass_source_hash(), 12345)
    value, src = bench.read_hbm_profile("ar100", "f64")
    assert value == 12345.0
    _profile(path, "0" * 16, 12345)
    value, why = bench.read_hbm_profile("ar100", "f64")
    assert value is None and "changed" in why
    _profile(path, bench.pass_source_hash(), 12345, "toep_pass_kernel<float, 9, 64, 3>")
    value, why = bench.read_hbm_profile("ar100", "f64")
    assert value is None and "covers" in why
    assert bench.read_hbm_profile("ar100", "f64", "toep_pass_kernel<float")[0] == 12345.0


def test_committed_profile_matches_sources():
    """The committed counter summary was taken from the pass as it is now."""
    value, src = bench.read_hbm_profile("ar100", "f64")
    assert value is not None, src
    assert value > bench.fused_pass_bytes(1 << 22, 100, 1024, 4535, 8) * 0.5


@pytest.mark.parametrize("workload", ["ar100", "ar500", "batch"])
def test_committed_mfma_profile_matches_qr_sources(workload):
    """The committed FP64-MFMA summaries were taken from the QR kernels as
    they are now (else the bench line drops its qr_fp64_mfma field)."""
    rec = bench.read_mfma_profile(workload)
    assert rec is not None
    assert rec["kernels"] and 0.0 < rec["util_over_mfma_kernels"] < 1.0


def test_kernel_stats_summary(tmp_path):
    d = tmp_path / "run" / "node"
    d.mkdir(parents=True)
    (d / "ar_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage"\n'
        '"void tls::(anonymous namespace)::toep_pass_kernel<double, 9, 64, 3>(double const*)",'
        '4,3000,750,75.0\n'
        '"tls::(anonymous namespace)::colsum_kernel<256>(double const*)",4,1000,250,25.0\n')
    out = str(tmp_path / "summary.txt")
    bench.prof_summary("stats", [str(tmp_path / "run")], out, "cmd", "title")
    lines = open(out).read().splitlines()
    assert lines[0] == "# title" and lines[1] == "# command: cmd"
    assert lines[2] == f"source_hash: {bench.pass_source_hash()}"
    rows = [l.split() for l in lines[4:]]
    assert " ".join(rows[0][:-4]) == "toep_pass_kernel<double, 9, 64, 3>"
    assert rows[0][-4:] == ["4", "3.0", "0.75", "75.00"]
    assert " ".join(rows[1][:-4]) == "colsum_kernel<256>"
    assert rows[1][-1] == "25.00"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
