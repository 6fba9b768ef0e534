"""Write the FP64 QR oracle's solutions of the configured workloads that the
GPU parity tests compare against (each file: phi_1..phi_p, then ||b - X phi*||,
kappa(X), ||X||_2):

  ar100_seed{1..9}_oracle.txt  AR(100), n = 2^22, synth.workload_ar100(seed=s)
                               (the kappa-stratified seeds beside seed 0)
  ar500_prefix_oracle.txt      AR(500): the first 2^20 samples of
                               synth.workload_ar500(seed=0)

Calls only oracle/ and synth/.  Run from the repository root:
    python tests/golden/make_config_oracles.py [ar100|ar500]
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
AR500_PREFIX = 1 << 20


def write(name, y, p, what):
    fit = oracle.fit_qr(y, p)
    smax = float(np.linalg.svd(fit["R"], compute_uv=False)[0])
    out = np.concatenate([fit["phi"], [fit["rnorm"], fit["kappa"], smax]])
    header = (f"FP64 QR oracle (oracle.fit_qr) on {what}.\n"
              f"Rows: phi_1..phi_{p}, ||b - X phi*||, kappa(X), ||X||_2.  "
              "Written by make_config_oracles.py.")
    np.savetxt(os.path.join(HERE, name), out, fmt="%.17e", header=header)
    print(name, "kappa %.3e rnorm %.6e" % (fit["kappa"], fit["rnorm"]), flush=True)


def main():
    which = sys.argv[1:] or ["ar100", "ar500"]
    if "ar100" in which:
        for s in range(1, 10):
            f = synth.workload_ar100(seed=s)
            write(f"ar100_seed{s}_oracle.txt", f.y, f.p,
                  f"synth.workload_ar100(seed={s}): AR(100), n = 2^22")
    if "ar500" in which:
        f = synth.workload_ar500(seed=0)
        write("ar500_prefix_oracle.txt", f.y[:AR500_PREFIX], f.p,
              "the first 2^20 samples of synth.workload_ar500(seed=0): AR(500)")


if __name__ == "__main__":
    main()
