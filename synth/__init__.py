"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws parameters and random vectors.  It holds none of the method's
arithmetic (no kernel evaluation, no grid, no contraction), so that the GPU library and the
CPU oracle can both be fed from it without sharing any computation.

Every workload is an analytic covariance function sampled on a grid; nothing here stands in
for a dataset.  All draws use numpy's ``default_rng`` with the master seed 1711 and fixed
draw order, so a workload is fully determined by its name.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MASTER_SEED = 1711

MATERN, SLATER, GAUSS = 0, 1, 2
CENTERED, OFFSET = 0, 1


@dataclass(frozen=True)
class KernelSpec:
    family: int
    nu: float = 0.5
    ell: float = 1.0
    sigma2: float = 1.0
    alpha: float = 1.0
    p: float = 1.0


@dataclass(frozen=True)
class GridSpec:
    n: tuple
    b: tuple = (1.0, 1.0, 1.0)
    layout: int = CENTERED


def cube(n: int, b: float = 1.0, layout: int = CENTERED) -> GridSpec:
    return GridSpec(n=(n, n, n), b=(b, b, b), layout=layout)


# --- plain method, FP64: exponential kernel on a 64^3 centred grid, ranks 1..16 -----------
def c1_small():
    return KernelSpec(MATERN, nu=0.5, ell=0.3), cube(64), list(range(1, 17))


# --- plain method on the GPU, FP32, 256^3: 9 Matern + 3 Slater ----------------------------
NUS = (0.5, 1.5, 2.5)
ELLS_C2 = (0.1, 0.3, 1.0)


def c2_kernels(include_slater: bool = True):
    ks = [KernelSpec(MATERN, nu=nu, ell=ell) for nu in NUS for ell in ELLS_C2]
    if include_slater:
        ks += [KernelSpec(SLATER, alpha=1.0, p=1.0, ell=ell) for ell in ELLS_C2]
    return ks


def c2_grid(n: int = 256, layout: int = CENTERED) -> GridSpec:
    return cube(n, 1.0, layout)


# --- precision study: Matern 3/2, ell = 0.2, 512^3 ----------------------------------------
def c3(n: int = 512):
    return KernelSpec(MATERN, nu=1.5, ell=0.2), cube(n), (1e-4, 1e-6)


# --- uneven batch: 256 tensors -------------------------------------------------------------
BATCH_SIZES = (32, 48, 64, 96, 128, 192, 256)


def uneven_batch(count: int = 256, seed: int = MASTER_SEED, sizes=BATCH_SIZES):
    """Per tensor, in order: n uniform over `sizes`, nu uniform over {1/2,3/2,5/2},
    ell = exp(U(ln 0.05, ln 1)); sigma2 = 1, centred grid on [-1,1]^3."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        nu = float(rng.choice(np.asarray(NUS)))
        ell = float(np.exp(rng.uniform(np.log(0.05), np.log(1.0))))
        out.append((KernelSpec(MATERN, nu=nu, ell=ell), cube(n)))
    return out


# --- serving: Poisson stream of mixed requests ---------------------------------------------
STREAM_SIZES = (64, 128, 256, 384)


@dataclass(frozen=True)
class Request:
    rid: int
    t_arrive: float
    kind: str               # "compress" | "matvec" | "trace" | "quadform"
    kernel: KernelSpec = None
    grid: GridSpec = None
    target: int = -1        # for follow-ups: index of an earlier compress request (-1: any)


def serving_stream(rate: float, count: int, seed: int = MASTER_SEED, sizes=STREAM_SIZES):
    """Exponential inter-arrival times at `rate` req/s; 70% compress (offset layout, so the
    covariance follow-ups are defined), 30% follow-ups split evenly among matvec, trace and
    quadratic form on a uniformly chosen earlier compress."""
    rng = np.random.default_rng([seed, int(rate * 1000)])
    t = 0.0
    reqs = []
    compress_ids = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        u = float(rng.uniform())
        if u < 0.7 or not compress_ids:
            n = int(rng.choice(np.asarray(sizes)))
            nu = float(rng.choice(np.asarray(NUS)))
            ell = float(np.exp(rng.uniform(np.log(0.05), np.log(1.0))))
            reqs.append(Request(rid, t, "compress", KernelSpec(MATERN, nu=nu, ell=ell),
                                cube(n, 1.0, OFFSET)))
            compress_ids.append(rid)
        else:
            kind = ("matvec", "trace", "quadform")[int(rng.integers(0, 3))]
            target = int(compress_ids[int(rng.integers(0, len(compress_ids)))])
            reqs.append(Request(rid, t, kind, target=target))
    return reqs


# --- random vectors ------------------------------------------------------------------------
def normal_vector(shape, stream: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Seeded N(0,1) draws rounded to float32 (the input of the covariance matvec)."""
    rng = np.random.default_rng([seed, 7, int(stream)])
    return rng.standard_normal(size=tuple(shape)).astype(np.float32)


def random_tensor(shape, stream: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Seeded U(-1,1) float64 tensor (generic non-symmetric test input)."""
    rng = np.random.default_rng([seed, 11, int(stream)])
    return rng.uniform(-1.0, 1.0, size=tuple(shape))

