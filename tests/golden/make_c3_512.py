"""Writes tests/golden/c3_512.npz: the FP64 oracle's compression of the precision-study tensor
(Matern nu = 3/2, ell = 0.2, sigma2 = 1, centred 512^3 vertex grid of [-1, 1]^3; Sec. 3.7
eq. (3.25)) at eps = 1e-4 and 1e-6: HOSVD with the eps rule, then two Tucker-ALS sweeps
(Sec. 3.2).  Calls only the oracle.

    python tests/golden/make_c3_512.py          # ~minutes on the host cores, ~3 GB of memory
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as o  # noqa: E402

N, NU, ELL = 512, 1.5, 0.2
EPS = (1e-4, 1e-6)


def main():
    o.build()
    k = o.Kernel(o.MATERN, nu=NU, ell=ELL)
    g = o.Grid(n=(N, N, N), b=(1.0, 1.0, 1.0), layout=o.CENTERED)
    t0 = time.time()
    A = o.grid_eval(k, g)
    factors = o.hosvd_factors(A)
    na2 = o.sumsq(A)
    out = {"n": np.int64(N), "nu": np.float64(NU), "ell": np.float64(ELL), "norm_a2": np.float64(na2),
           "eps": np.asarray(EPS, dtype=np.float64)}
    for k_ in range(3):
        out["lam%d" % k_] = np.asarray(factors[k_][0][:48], dtype=np.float64)
    print("grid + Grams + eigensolves %.1f s" % (time.time() - t0), flush=True)
    for i, eps in enumerate(EPS):
        t1 = time.time()
        ranks = o.eps_ranks([f[0] for f in factors], na2, eps)
        t = o.hosvd(A, tuple(ranks), factors)
        t = o.hooi(A, t, sweeps=2)
        out["ranks%d" % i] = np.asarray(t.ranks if hasattr(t, "ranks") else ranks, dtype=np.int64)
        out["rel_err%d" % i] = np.float64(t.rel_err)
        out["core%d" % i] = np.asarray(t.core, dtype=np.float64)
        for k_ in range(3):
            out["U%d_%d" % (i, k_)] = np.asarray(t.U[k_], dtype=np.float64)
        print("eps %g ranks %s E %.6e (%.1f s)" % (eps, ranks, t.rel_err, time.time() - t1), flush=True)
    np.savez(os.path.join(HERE, "c3_512.npz"), **out)


if __name__ == "__main__":
    main()
