"""Writes tests/golden/c2_curve.json: the FP64 oracle's error curve for the twelve covariance
tensors of the plain GPU configuration (Matern nu in {1/2, 3/2, 5/2} x ell in {0.1, 0.3, 1.0}
and Slater exp(-alpha r / ell) with alpha = 1 at the same ell; sigma2 = 1; centred 256^3 vertex
grid of [-1, 1]^3, Sec. 3.7 eqs. (3.25)-(3.27)): the relative Frobenius error E_FN (eq. (3.26))
at Tucker ranks r = 4, 8, 16, 32 after HOSVD and after two Tucker-ALS sweeps (Sec. 3.2).
Calls only the oracle.

    python tests/golden/make_c2_curve.py        # about a minute on the host cores
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import oracle as o  # noqa: E402

N = 256
RANKS = (4, 8, 16, 32)


def main():
    o.build()
    g = o.Grid(n=(N, N, N), b=(1.0, 1.0, 1.0), layout=o.CENTERED)
    rows = []
    for ks in synth.c2_kernels(include_slater=True):
        t0 = time.time()
        k = o.Kernel(ks.family, nu=ks.nu, ell=ks.ell, sigma2=ks.sigma2, alpha=ks.alpha, p=ks.p)
        A = o.grid_eval(k, g)
        f = o.hosvd_factors(A)
        row = {"family": int(ks.family), "nu": ks.nu, "ell": ks.ell, "alpha": ks.alpha, "p": ks.p,
               "ranks": list(RANKS), "hosvd": [], "hooi2": []}
        for r in RANKS:
            t = o.hosvd(A, (r, r, r), f)
            row["hosvd"].append(t.rel_err)
            row["hooi2"].append(o.hooi(A, t, sweeps=2).rel_err)
        rows.append(row)
        print(row["family"], row["nu"], row["ell"], ["%.3e" % e for e in row["hooi2"]],
              "%.1f s" % (time.time() - t0), flush=True)
    doc = {"source": "tests/golden/make_c2_curve.py (FP64 oracle)", "n": N, "layout": "centred", "b": 1.0,
           "tensors": rows}
    with open(os.path.join(HERE, "c2_curve.json"), "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
