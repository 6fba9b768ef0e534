"""Write ar100_seed0_oracle.txt: the FP64 QR oracle's solution for the AR(100),
n = 2^22, seed-0 workload (phi_1..phi_100, then ||r*||, kappa(X), ||X||_2).

Calls only oracle/ and synth/.  Run from the repository root:
    python tests/golden/make_ar100_oracle.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    f = synth.workload_ar100(seed=0)
    fit = oracle.fit_qr(f.y, f.p)
    smax = float(np.linalg.svd(fit["R"], compute_uv=False)[0])
    out = np.concatenate([fit["phi"], [fit["rnorm"], fit["kappa"], smax]])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ar100_seed0_oracle.txt")
    header = ("FP64 QR oracle (oracle.fit_qr) on synth.workload_ar100(seed=0): AR(100), n = 2^22.\n"
              "Rows: phi_1..phi_100, ||b - X phi*||, kappa(X), ||X||_2.  Written by make_ar100_oracle.py.")
    np.savetxt(path, out, fmt="%.17e", header=header)
    print("kappa", fit["kappa"], "rnorm", fit["rnorm"])


if __name__ == "__main__":
    main()
