"""FP64 CPU oracle for the Tucker compression of Matern / Slater covariance tensors.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this module.  It shares no code with the GPU library and neither
imports the other.  The heavy loops live in ``oracle.c`` (explicit loops, IEEE double, no
BLAS/LAPACK); this file strings them together in the order the paper describes.

Paper: Litvinenko et al., "Tucker tensor analysis of Matern functions in spatial statistics"
(arXiv 1711.06874).

Readings where the paper is silent (each one is also listed in the design notes):
  * grid: centred vertex grid x_i = -b + i h, h = 2b/(n-1) (Sec. 3.7 eq. (3.25)); the offset
    layout x_i = i h holds the generator at every node difference (Sec. 3.6 needs the
    generator at offsets 0..n-1 to build Toeplitz factors defined by their first column);
  * Slater family sigma2 * exp(-alpha (r/ell)^p) (Sec. 3.7 eq. (3.27) with amplitude/scale);
  * HOSVD factors from the Gram matrices A_(k) A_(k)^T (same subspaces as the SVD of A_(k),
    Sec. 3.2); eigenvectors signed so the largest-magnitude entry is positive;
  * eps rank rule (not given in the paper): per mode, the smallest r with
    sum_{i>r} lambda_i <= eps^2 ||A||^2 / 3, the standard HOSVD truncation, which guarantees
    a relative Frobenius error <= eps;
  * HOOI: Gauss-Seidel sweeps over modes 1,2,3, core from the last single-hole tensor;
    "converged" means | ||G|| - ||G_prev|| | <= 1e-13 ||A|| (at most 50 sweeps).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MATERN, SLATER, GAUSS, SPECTRAL = 0, 1, 2, 3
CENTERED, OFFSET = 0, 1


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no fast-math, no FP contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.tko_kernel.restype = ctypes.c_double
    lib.tko_kernel.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6
    lib.tko_grid_coords.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, dp]
    lib.tko_grid_eval.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5 + [ip, dp, ctypes.c_int, dp]
    lib.tko_grid_eval_metric.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5 + [ip, dp, ctypes.c_int, dp, dp]
    lib.tko_bessel_k.restype = ctypes.c_double
    lib.tko_bessel_k.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.tko_gram.argtypes = [dp, ip, ctypes.c_int, dp]
    lib.tko_jacobi_eig.restype = ctypes.c_int
    lib.tko_jacobi_eig.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_double]
    lib.tko_mode_product.argtypes = [dp, ip, ctypes.c_int, dp, ctypes.c_int, dp]
    lib.tko_sumsq.restype = ctypes.c_double
    lib.tko_sumsq.argtypes = [dp, ctypes.c_size_t]
    lib.tko_diff_sumsq.restype = ctypes.c_double
    lib.tko_diff_sumsq.argtypes = [dp, dp, ctypes.c_size_t]
    lib.tko_cov_rows.argtypes = [dp, ip, ip, ip, dp, ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.c_int, dp]
    lib.tko_num_threads.restype = ctypes.c_int
    lib.tko_set_num_threads.argtypes = [ctypes.c_int]
    lib.tko_cholesky.restype = ctypes.c_int
    lib.tko_cholesky.argtypes = [ctypes.c_int, dp]
    lib.tko_chol_solve.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(v):
    arr = (ctypes.c_int * len(v))(*[int(x) for x in v])
    return arr


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().tko_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops (results do not depend on it)."""
    _load().tko_set_num_threads(int(n))


# ----------------------------------------------------------------------------------------
# Covariance functions and the collocation tensor
# ----------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Kernel:
    """family MATERN (nu, ell), SLATER (alpha, p, ell), GAUSS (ell) or SPECTRAL (the Matern
    spectral density, alpha, nu); every family is scaled by sigma2.  metric: the diagonal of the
    anisotropic distance r^2 = sum_k metric_k x_k^2 (Sec. 2.2), None for ||x||."""
    family: int = MATERN
    nu: float = 0.5
    ell: float = 1.0
    sigma2: float = 1.0
    alpha: float = 1.0
    p: float = 1.0
    metric: tuple = None


@dataclass(frozen=True)
class Grid:
    n: tuple = (8, 8, 8)
    b: tuple = (1.0, 1.0, 1.0)
    layout: int = CENTERED


def kernel_value(k: Kernel, r: float) -> float:
    """Covariance value at distance r (Sec. 2.2 eq. (2.3); Sec. 3.7 eqs. (3.27), (3.28))."""
    return float(_load().tko_kernel(k.family, k.nu, k.ell, k.sigma2, k.alpha, k.p, float(r)))


def bessel_k(nu: float, x: float) -> float:
    """K_nu(x) from its integral representation (trapezoidal rule), any real order, x > 0."""
    return float(_load().tko_bessel_k(float(nu), float(x)))


def grid_coords(n: int, b: float, layout: int) -> np.ndarray:
    x = np.empty(n, dtype=np.float64)
    _load().tko_grid_coords(int(n), float(b), int(layout), _dp(x))
    return x


def grid_eval(k: Kernel, g: Grid) -> np.ndarray:
    """Collocation tensor A[i0,i1,i2] = k(||x_i||) on the grid (Sec. 3.7 eq. (3.25))."""
    A = np.empty(tuple(g.n), dtype=np.float64)
    if k.metric is None:
        _load().tko_grid_eval(k.family, k.nu, k.ell, k.sigma2, k.alpha, k.p, _ip(g.n),
                              (ctypes.c_double * 3)(*g.b), int(g.layout), _dp(A))
    else:
        _load().tko_grid_eval_metric(k.family, k.nu, k.ell, k.sigma2, k.alpha, k.p, _ip(g.n),
                                     (ctypes.c_double * 3)(*g.b), int(g.layout),
                                     (ctypes.c_double * 3)(*[float(a) for a in k.metric]), _dp(A))
    return A


# ----------------------------------------------------------------------------------------
# Linear-algebra primitives
# ----------------------------------------------------------------------------------------

def gram(X: np.ndarray, mode: int) -> np.ndarray:
    """G_k = X_(k) X_(k)^T (Sec. 3.2: HOSVD works on the mode unfoldings)."""
    X = _f64(X)
    d = X.shape
    G = np.empty((d[mode], d[mode]), dtype=np.float64)
    _load().tko_gram(_dp(X), _ip(d), int(mode), _dp(G))
    return G


def jacobi_eig(S: np.ndarray, max_sweeps: int = 60, tol: float = 1e-15):
    """Full symmetric eigendecomposition by two-sided Jacobi; descending, sign-normalised."""
    S = _f64(S)
    n = S.shape[0]
    lam = np.empty(n, dtype=np.float64)
    V = np.empty((n, n), dtype=np.float64)
    sweeps = _load().tko_jacobi_eig(n, _dp(S), _dp(lam), _dp(V), int(max_sweeps), float(tol))
    return lam, V, int(sweeps)


def mode_product(X: np.ndarray, mode: int, M: np.ndarray) -> np.ndarray:
    """Y = X x_mode M with M of shape (J, X.shape[mode]) (Sec. 3.1 contracted products)."""
    X = _f64(X)
    M = _f64(M)
    d = list(X.shape)
    assert M.shape[1] == d[mode]
    e = list(d)
    e[mode] = M.shape[0]
    Y = np.empty(tuple(e), dtype=np.float64)
    _load().tko_mode_product(_dp(X), _ip(d), int(mode), _dp(M), int(M.shape[0]), _dp(Y))
    return Y


def sumsq(X: np.ndarray) -> float:
    X = _f64(X)
    return float(_load().tko_sumsq(_dp(X), X.size))


def diff_sumsq(X: np.ndarray, Y: np.ndarray) -> float:
    X = _f64(X)
    Y = _f64(Y)
    assert X.shape == Y.shape
    return float(_load().tko_diff_sumsq(_dp(X), _dp(Y), X.size))


# ----------------------------------------------------------------------------------------
# Tucker format: HOSVD, eps rank rule, HOOI (Sec. 3.1 eq. (3.4), Sec. 3.2)
# ----------------------------------------------------------------------------------------

@dataclass
class Tucker:
    U: list                      # three factor matrices, n_k x r_k, orthonormal columns
    core: np.ndarray             # r1 x r2 x r3
    norm_a2: float = 0.0         # ||A||_F^2
    rel_err: float = float("nan")
    lambdas: list = field(default_factory=list)   # HOSVD Gram eigenvalues per mode (all n_k)
    history: list = field(default_factory=list)   # ||core|| after every HOOI mode update
    sweeps: int = 0

    @property
    def ranks(self):
        return tuple(int(u.shape[1]) for u in self.U)


def project_core(A: np.ndarray, U) -> np.ndarray:
    """G = A x_1 U1^T x_2 U2^T x_3 U3^T."""
    X = A
    for k in range(3):
        X = mode_product(X, k, U[k].T)
    return X


def reconstruct(core: np.ndarray, U) -> np.ndarray:
    """A_(r) = G x_1 U1 x_2 U2 x_3 U3 (Sec. 3.1, Tucker format in contracted-product form)."""
    X = core
    for k in (2, 1, 0):
        X = mode_product(X, k, U[k])
    return X


def hosvd_factors(A: np.ndarray):
    """Full eigendecompositions of the three mode Grams: (lambda_k, V_k) for k = 0,1,2."""
    out = []
    for k in range(3):
        lam, V, sweeps = jacobi_eig(gram(A, k))
        if sweeps < 0:
            raise RuntimeError("Jacobi did not converge")
        out.append((lam, V))
    return out


def eps_ranks(lambdas, norm_a2: float, eps: float, cap=None):
    """Per-mode truncation: smallest r >= 1 with sum_{i>r} lambda_i <= eps^2 ||A||^2 / 3."""
    ranks = []
    for k, lam in enumerate(lambdas):
        budget = eps * eps * norm_a2 / 3.0
        n = lam.shape[0]
        r = n
        for cand in range(1, n + 1):
            tail = float(np.sum(np.maximum(lam[cand:], 0.0)))
            if tail <= budget:
                r = cand
                break
        if cap is not None:
            r = min(r, int(cap[k]))
        ranks.append(r)
    return tuple(ranks)


def hosvd(A: np.ndarray, ranks, factors=None) -> Tucker:
    """Truncated HOSVD: U_k = leading r_k eigenvectors of A_(k)A_(k)^T, G = A x_k U_k^T."""
    A = _f64(A)
    if factors is None:
        factors = hosvd_factors(A)
    U = [factors[k][1][:, : min(int(ranks[k]), A.shape[k])].copy() for k in range(3)]
    core = project_core(A, U)
    na2 = sumsq(A)
    t = Tucker(U=U, core=core, norm_a2=na2, lambdas=[f[0] for f in factors])
    t.rel_err = rel_error(A, t)
    return t


def hooi(A: np.ndarray, init: Tucker, sweeps=None, converge_tol: float = 1e-13,
         max_sweeps: int = 50) -> Tucker:
    """Tucker-ALS (HOOI), Sec. 3.2: for each mode, build the single-hole tensor
    B_k = A x_{j != k} U_j^T with the latest factors and replace U_k by the leading r_k
    eigenvectors of B_(k) B_(k)^T; the core is B_3 x_3 U_3^T after the last update.

    sweeps=None runs to convergence (| ||G|| - ||G_prev|| | <= converge_tol ||A||)."""
    A = _f64(A)
    U = [u.copy() for u in init.U]
    r = [u.shape[1] for u in U]
    na = float(np.sqrt(init.norm_a2 if init.norm_a2 > 0 else sumsq(A)))
    prev = float(np.sqrt(sumsq(init.core)))
    history = [prev]
    nsweeps = sweeps if sweeps is not None else max_sweeps
    done = 0
    core = init.core
    for _ in range(nsweeps):
        for k in range(3):
            B = A
            for j in range(3):
                if j != k:
                    B = mode_product(B, j, U[j].T)
            lam, V, s = jacobi_eig(gram(B, k))
            if s < 0:
                raise RuntimeError("Jacobi did not converge")
            U[k] = V[:, : r[k]].copy()
            core = mode_product(B, k, U[k].T)
            history.append(float(np.sqrt(sumsq(core))))
        done += 1
        cur = history[-1]
        if sweeps is None and abs(cur - prev) <= converge_tol * na:
            break
        prev = cur
    t = Tucker(U=U, core=core, norm_a2=init.norm_a2, lambdas=init.lambdas, history=history,
               sweeps=done)
    t.rel_err = rel_error(A, t)
    return t


def rel_error(A: np.ndarray, t: Tucker) -> float:
    """E_FN = ||A - A_(r)||_F / ||A||_F with an explicit reconstruction (Sec. 3.7 eq. (3.26))."""
    Ah = reconstruct(t.core, t.U)
    return float(np.sqrt(diff_sumsq(A, Ah) / sumsq(A)))


def compress(k: Kernel, g: Grid, ranks=None, eps: float = 0.0, sweeps=2,
             A: np.ndarray = None) -> Tucker:
    """Task 1 of Sec. 2.1 on the collocation tensor: HOSVD (fixed ranks or the eps rule),
    then `sweeps` HOOI sweeps (None = to convergence, 0 = HOSVD only)."""
    if A is None:
        A = grid_eval(k, g)
    factors = hosvd_factors(A)
    na2 = sumsq(A)
    if ranks is None:
        if not eps > 0:
            raise ValueError("either ranks or eps > 0 is required")
        ranks = eps_ranks([f[0] for f in factors], na2, eps)
    ranks = tuple(min(int(r), A.shape[i]) for i, r in enumerate(ranks))
    t = hosvd(A, ranks, factors)
    if sweeps != 0:
        t = hooi(A, t, sweeps=sweeps)
    return t


# ----------------------------------------------------------------------------------------
# Covariance operator in Kronecker-Toeplitz form (Sec. 3.6, Sec. 4 eq. (4.1), (4.3))
# ----------------------------------------------------------------------------------------

def cov_offsets(g: Grid):
    """(off, m): the operator acts on m_k points per axis with T_{ij} = u[off_k + |i-j|].
    Offset layout: off = 0, m = n.  Odd centred layout n = 2k+1: off = k (the origin node),
    m = k+1 (the non-negative sector).  Even centred grids have no origin node: None."""
    off, m = [], []
    for n in g.n:
        if g.layout == OFFSET:
            off.append(0)
            m.append(n)
        elif n % 2 == 1:
            off.append((n - 1) // 2)
            m.append((n + 1) // 2)
        else:
            return None
    return tuple(off), tuple(m)


def cov_matvec_rows(t: Tucker, g: Grid, z: np.ndarray, rows) -> np.ndarray:
    """y_i = sum_j C_ij z_j for the requested flat row indices, with the covariance generated
    by the reconstructed Tucker tensor: C_ij = A_(r)(off + |i - j|) (per axis)."""
    return cov_rows_from_generator(reconstruct(t.core, t.U), g, z, rows)


def cov_rows_from_generator(Q: np.ndarray, g: Grid, z: np.ndarray, rows) -> np.ndarray:
    """y_i = sum_j Q(off + |i - j|) z_j (per-axis offsets) for a generator tensor Q."""
    om = cov_offsets(g)
    if om is None:
        raise ValueError("covariance operator needs an origin node (offset or odd centred grid)")
    off, m = om
    Q = _f64(Q)
    z = _f64(z).reshape(-1)
    assert z.size == m[0] * m[1] * m[2]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.empty(rows.size, dtype=np.float64)
    _load().tko_cov_rows(_dp(Q), _ip(Q.shape), _ip(off), _ip(m), _dp(z),
                         rows.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), int(rows.size),
                         _dp(y))
    return y


def cov_matvec(t: Tucker, g: Grid, z: np.ndarray) -> np.ndarray:
    om = cov_offsets(g)
    if om is None:
        raise ValueError("covariance operator needs an origin node")
    m = om[1]
    return cov_matvec_rows(t, g, z, np.arange(m[0] * m[1] * m[2])).reshape(m)


def cov_trace(t: Tucker, g: Grid) -> float:
    """trace(C) = (number of points) * A_(r)(origin): every diagonal entry of the Toeplitz
    covariance is the generator's value at offset 0 (Sec. 4, trace/diag via the origin)."""
    om = cov_offsets(g)
    if om is None:
        raise ValueError("covariance operator needs an origin node")
    off, m = om
    Q = reconstruct(t.core, t.U)
    return float(m[0] * m[1] * m[2] * Q[off[0], off[1], off[2]])


def cov_trace_kron(t: Tucker, g: Grid) -> float:
    """trace(sum_abc G_abc T(u1a) (x) T(u2b) (x) T(u3c)) = sum_abc G_abc prod_k trace T(u_k)
    (Sec. 4 eq. (4.3)); trace T(u) = m * u[off]."""
    om = cov_offsets(g)
    if om is None:
        raise ValueError("covariance operator needs an origin node")
    off, m = om
    tr = [m[k] * t.U[k][off[k], :] for k in range(3)]
    total = 0.0
    r = t.core.shape
    for a in range(r[0]):
        for b in range(r[1]):
            for c in range(r[2]):
                total += t.core[a, b, c] * tr[0][a] * tr[1][b] * tr[2][c]
    return float(total)


def quadratic_form(t: Tucker, g: Grid, z: np.ndarray) -> float:
    """z^T C z with the plain matrix-vector product."""
    y = cov_matvec(t, g, z)
    return float(np.dot(_f64(z).reshape(-1), y.reshape(-1)))


# ----------------------------------------------------------------------------------------
# Multigrid Tucker (Sec. 3.2, last paragraph; Sec. 3.7 Fig. 7)
# ----------------------------------------------------------------------------------------

def multigrid_sizes(n: int, levels: int) -> list:
    """Points per axis from the coarsest level to n: each coarser level has (n + 1) // 2 points
    (dyadic refinement: 2^k + 1 -> 2^(k-1) + 1 nests the vertex grids; 2^k -> 2^(k-1))."""
    sizes = [int(n)]
    for _ in range(int(levels)):
        sizes.append((sizes[-1] + 1) // 2)
    return sizes[::-1]


def interpolate_factor(U: np.ndarray, x_coarse: np.ndarray, x_fine: np.ndarray) -> np.ndarray:
    """Each column of U, read as a function sampled at x_coarse (uniform), linearly interpolated
    to the nodes x_fine of the same interval."""
    nc = x_coarse.shape[0]
    h = (x_coarse[-1] - x_coarse[0]) / (nc - 1)
    V = np.empty((x_fine.shape[0], U.shape[1]), dtype=np.float64)
    for j, x in enumerate(x_fine):
        t = (x - x_coarse[0]) / h
        i = min(max(int(np.floor(t)), 0), nc - 2)
        w = t - i
        for c in range(U.shape[1]):
            V[j, c] = (1.0 - w) * U[i, c] + w * U[i + 1, c]
    return V


def orthonormalize(U: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt, applied twice (columns orthonormal to rounding)."""
    Q = _f64(U).copy()
    for _ in range(2):
        for c in range(Q.shape[1]):
            for p in range(c):
                Q[:, c] -= np.dot(Q[:, p], Q[:, c]) * Q[:, p]
            Q[:, c] /= np.sqrt(np.dot(Q[:, c], Q[:, c]))
    return Q


def multigrid_compress(k: Kernel, g: Grid, ranks, levels: int, sweeps=2) -> Tucker:
    """Multigrid Tucker: truncated HOSVD only on the coarsest grid; on each finer grid the
    factors of the previous level, interpolated to the new nodes and orthonormalised, start
    `sweeps` Tucker-ALS sweeps (None = to convergence) on that level's tensor.  No Gram of a
    fine-grid tensor is formed."""
    sizes = [multigrid_sizes(n, levels) for n in g.n]
    t = None
    xs_prev = None
    for lev in range(levels + 1):
        gl = Grid(n=tuple(s[lev] for s in sizes), b=g.b, layout=g.layout)
        A = grid_eval(k, gl)
        xs = [grid_coords(gl.n[a], gl.b[a], gl.layout) for a in range(3)]
        r = tuple(min(int(ranks[a]), gl.n[a]) for a in range(3))
        if t is None:
            t = hosvd(A, r)
        else:
            U = [orthonormalize(interpolate_factor(t.U[a], xs_prev[a], xs[a])) for a in range(3)]
            init = Tucker(U=U, core=project_core(A, U), norm_a2=sumsq(A))
            init.rel_err = rel_error(A, init)
            t = init
        if sweeps != 0:
            t = hooi(A, t, sweeps=sweeps)
        xs_prev = xs
    return t


# ----------------------------------------------------------------------------------------
# Separable covariance: rank-1 Kronecker algebra (Sec. 4, "Separable covariance matrices")
# ----------------------------------------------------------------------------------------

def cov_factor_1d(k: Kernel, n: int, b: float, layout: int = CENTERED, nugget: float = 0.0) -> np.ndarray:
    """C_k[i, j] = k(|x_i - x_j|) on one axis of the grid, plus nugget on the diagonal.  For
    the Gaussian exp(-|x - y|^2 / ell^2) the 3-D covariance is exactly C_1 (x) C_2 (x) C_3."""
    x = grid_coords(n, b, layout)
    C = np.empty((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            C[i, j] = kernel_value(k, abs(x[i] - x[j]))
    C[np.diag_indices(n)] += nugget
    return C


def cholesky(C: np.ndarray) -> np.ndarray:
    """Lower-triangular L with C = L L^T (plain algorithm in oracle.c)."""
    L = _f64(C).copy()
    info = _load().tko_cholesky(L.shape[0], _dp(L))
    if info != 0:
        raise np.linalg.LinAlgError(f"not positive definite at pivot {info - 1}")
    return L


def chol_solve(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with (L L^T) X = B (B: n or n x nrhs)."""
    X = _f64(B).copy()
    vec = X.ndim == 1
    if vec:
        X = X.reshape(-1, 1)
    X = np.ascontiguousarray(X)
    _load().tko_chol_solve(L.shape[0], _dp(_f64(L)), X.shape[1], _dp(X))
    return X.reshape(-1) if vec else X


def kron1_logdet(Ls) -> float:
    """log det(C_1 (x) C_2 (x) C_3) = sum_j (prod_{i != j} n_i) log det C_j, with
    log det C_j = 2 sum_i log L_j[i, i] (the log-determinant lemma of Sec. 4)."""
    ns = [L.shape[0] for L in Ls]
    N = int(np.prod(ns))
    return float(sum((N // ns[j]) * 2.0 * np.sum(np.log(np.diag(Ls[j]))) for j in range(len(Ls))))


def kron1_solve(Ls, z: np.ndarray) -> np.ndarray:
    """w = (C_1 (x) C_2 (x) C_3)^-1 z = z x_1 C_1^-1 x_2 C_2^-1 x_3 C_3^-1 (the inverse lemma of
    Sec. 4), each C_j^-1 applied along its mode by forward and back substitution."""
    W = _f64(z).reshape([L.shape[0] for L in Ls]).copy()
    for mode, L in enumerate(Ls):
        M = np.moveaxis(W, mode, 0)
        shp = M.shape
        X = chol_solve(L, np.ascontiguousarray(M.reshape(shp[0], -1)))
        W = np.moveaxis(X.reshape(shp), 0, mode)
    return np.ascontiguousarray(W)


def kron1_chol_apply(Ls, z: np.ndarray) -> np.ndarray:
    """y = (L_1 (x) L_2 (x) L_3) z (the Cholesky lemma of Sec. 4: L = L_1 (x) L_2 (x) L_3)."""
    Y = _f64(z).reshape([L.shape[0] for L in Ls])
    for mode, L in enumerate(Ls):
        Y = mode_product(Y, mode, L)
    return Y


def kron1_loglik(Ls, z: np.ndarray) -> float:
    """Gaussian log-likelihood of z under N(0, C_1 (x) C_2 (x) C_3):
    -1/2 (N log(2 pi) + log det C + z^T C^-1 z)."""
    zf = _f64(z).reshape(-1)
    w = kron1_solve(Ls, zf).reshape(-1)
    return float(-0.5 * (zf.size * np.log(2.0 * np.pi) + kron1_logdet(Ls) + np.dot(zf, w)))


# ----------------------------------------------------------------------------------------
# Sinc-quadrature canonical (CP) tensor and canonical-to-Tucker (Sec. 3.4, Sec. 3.5)
# ----------------------------------------------------------------------------------------

def laplace_weight(nu: float, ell: float, t: float) -> float:
    """omega(t) with Matern_nu(r) = int_0^inf omega(t) exp(-r^2 t) dt (sigma2 = 1), nu = 1/2,
    3/2, 5/2.  Sec. 3.5 gives exp(-2 sqrt(a p)) = sqrt(a/pi) int t^-3/2 exp(-a/t - p t) dt
    (p = r^2); with c = sqrt(2 nu)/ell and g(t) = c/(2 sqrt(pi)) t^-3/2 exp(-c^2/(4t)) that is
    e^{-c r} = int g(t) e^{-r^2 t} dt.  Since s^j e^{-s} = c^j d^j/dc^j e^{-c r} (s = c r),
    the polynomial factors of the half-integer closed forms act on g:
      nu = 1/2: g;   nu = 3/2: (1 - c d/dc) g = g c^2/(2t);
      nu = 5/2: (1 - c d/dc + c^2/3 d^2/dc^2) g = g c^4/(12 t^2)."""
    m = int(round(nu - 0.5))
    c = np.sqrt(2.0 * nu) / ell
    g = c / (2.0 * np.sqrt(np.pi)) * t ** -1.5 * np.exp(-c * c / (4.0 * t))
    return g * {0: 1.0, 1: c * c / (2.0 * t), 2: c ** 4 / (12.0 * t * t)}[m]


def sinc_cp(k: Kernel, g: Grid, M: int, C0: float = 1.0):
    """Rank R = 2M+1 canonical tensor of the Matern collocation tensor (Sec. 3.4 eq. (3.9),
    (3.10) and (3.13), collocation form): with t = (c^2/4) e^u the Laplace integral becomes
    int_R omega(t(u)) t(u) e^{-r^2 t(u)} du, and the sinc rule with step h = C0 log(M)/M and
    nodes u_k = k h, k = -M..M gives
        A(x) ~ sum_k w_k prod_l exp(-t_k x_l^2),  w_k = sigma2 h omega(t_k) t_k.
    Returns (Q, w, t): Q[l] is n_l x R with columns w_k^(1/3) exp(-t_k x_{l,i}^2)."""
    if k.family != MATERN or abs(k.nu - round(k.nu - 0.5) - 0.5) > 1e-12 or k.nu > 2.6:
        raise ValueError("sinc CP: Matern nu in {1/2, 3/2, 5/2}")
    h = C0 * np.log(M) / M
    c = np.sqrt(2.0 * k.nu) / k.ell
    u = h * np.arange(-M, M + 1, dtype=np.float64)
    t = (c * c / 4.0) * np.exp(u)
    w = np.array([k.sigma2 * h * laplace_weight(k.nu, k.ell, tk) * tk for tk in t])
    Q = []
    for a in range(3):
        x = grid_coords(g.n[a], g.b[a], g.layout)
        Qa = np.empty((g.n[a], t.size))
        for i in range(g.n[a]):
            for j in range(t.size):
                Qa[i, j] = np.cbrt(w[j]) * np.exp(-t[j] * x[i] * x[i])
        Q.append(Qa)
    return Q, w, t


def cp_full(Q) -> np.ndarray:
    """The full tensor sum_k q1_k (x) q2_k (x) q3_k."""
    n = [q.shape[0] for q in Q]
    A = np.zeros(n)
    for j in range(Q[0].shape[1]):
        A += np.einsum("i,j,k->ijk", Q[0][:, j], Q[1][:, j], Q[2][:, j])
    return A


def cp_norm2(Q) -> float:
    """||sum_k q1_k (x) q2_k (x) q3_k||^2 = sum_{k,k'} prod_l <q_l,k, q_l,k'>."""
    P = Q[0].T @ Q[0] * (Q[1].T @ Q[1]) * (Q[2].T @ Q[2])
    return float(P.sum())


def c2t_core(Q, V) -> np.ndarray:
    """Core of the projection of the CP tensor onto the factor spans:
    G = sum_k (V1^T q1_k) (x) (V2^T q2_k) (x) (V3^T q3_k)."""
    P = [V[a].T @ Q[a] for a in range(3)]
    r = [p.shape[0] for p in P]
    G = np.zeros(r)
    for j in range(Q[0].shape[1]):
        G += np.einsum("a,b,c->abc", P[0][:, j], P[1][:, j], P[2][:, j])
    return G


def c2t(Q, ranks, sweeps=0) -> Tucker:
    """Canonical-to-Tucker (Sec. 3.4, after eq. (3.14)): RHOSVD initial guess -- the leading
    left singular vectors of each side matrix Q_l, here the leading eigenvectors of Q_l Q_l^T
    (Jacobi) -- then `sweeps` ALS sweeps on the canonical data: for mode l the single-hole
    tensor B = CP x_{j != l} V_j^T has the unfolding Q_l W with W[k] = (V_j^T q_j,k) (x)
    (V_m^T q_m,k), so B_(l) B_(l)^T = Q_l (W W^T) Q_l^T, W W^T = P_j^T P_j o P_m^T P_m.  No full
    tensor is formed; the error against the canonical tensor follows from Pythagoras,
    ||CP - T||^2 = ||CP||^2 - ||G||^2."""
    V = []
    for a in range(3):
        lam, E, s = jacobi_eig(Q[a] @ Q[a].T)
        V.append(E[:, : int(ranks[a])].copy())
    history = []
    for _ in range(int(sweeps)):
        for a in range(3):
            j, m = [x for x in range(3) if x != a]
            Pj = V[j].T @ Q[j]
            Pm = V[m].T @ Q[m]
            Wg = (Pj.T @ Pj) * (Pm.T @ Pm)
            lam, E, s = jacobi_eig(Q[a] @ Wg @ Q[a].T)
            V[a] = E[:, : int(ranks[a])].copy()
            history.append(float(np.sqrt(sumsq(c2t_core(Q, V)))))
    core = c2t_core(Q, V)
    n2 = cp_norm2(Q)
    t = Tucker(U=V, core=core, norm_a2=n2, history=history, sweeps=int(sweeps))
    t.rel_err = float(np.sqrt(max(n2 - sumsq(core), 0.0) / n2))
    return t


# ----------------------------------------------------------------------------------------
# Seeded N(0,1) inputs: Philox4x32-10 and the Box-Muller transform
# ----------------------------------------------------------------------------------------
# (not part of the paper's method: the matvec and quadratic form take z as an input; this is
# the published counter-based generator the device implements on its own, written out here
# from its definition: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
# 3", SC'11)

_PHILOX_M = (0xD2511F53, 0xCD9E8D57)   # round multipliers
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)   # key increments (golden ratio, sqrt(3) - 1)


def philox4x32_10(counters, key) -> np.ndarray:
    """Philox4x32 with ten rounds.  counters: (N, 4) words; key: two words.  One round maps
    (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
    with hi/lo the upper/lower 32 bits of the 64-bit product; the key grows by the Weyl
    increments before every round but the first.  Returns the (N, 4) output words."""
    c = np.asarray(counters, dtype=np.uint64).reshape(-1, 4) & 0xFFFFFFFF
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    mask = np.uint64(0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _PHILOX_W[0]) & 0xFFFFFFFF
            k1 = (k1 + _PHILOX_W[1]) & 0xFFFFFFFF
        p0 = c[:, 0] * np.uint64(_PHILOX_M[0])      # < 2^64: exact in uint64
        p1 = c[:, 2] * np.uint64(_PHILOX_M[1])
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = np.stack([hi1 ^ c[:, 1] ^ np.uint64(k0), lo1, hi0 ^ c[:, 3] ^ np.uint64(k1), lo0], axis=1)
    return c.astype(np.uint32)


def philox_blocks(key, counter0: int, nblocks: int) -> np.ndarray:
    """Words of counter blocks counter0 .. counter0 + nblocks - 1, counter (c mod 2^32,
    c / 2^32, 0, 0)."""
    c = np.arange(nblocks, dtype=np.uint64) + np.uint64(counter0)
    ctr = np.zeros((nblocks, 4), dtype=np.uint64)
    ctr[:, 0] = c & np.uint64(0xFFFFFFFF)
    ctr[:, 1] = c >> np.uint64(32)
    return philox4x32_10(ctr, key)


def normal_philox(count: int, seed: int, stream: int) -> np.ndarray:
    """count N(0,1) values as float32: block c gives the FP64 uniforms
    u_a = ((x1 2^32 + x0) >> 11) 2^-53, u_b = ((x3 2^32 + x2) >> 11) 2^-53 and, by the
    Box-Muller transform, z[2c] = rho cos(phi), z[2c+1] = rho sin(phi), rho = sqrt(-2 log(1 - u_a)),
    phi = 2 pi u_b, each rounded once to float."""
    nb = (count + 1) // 2
    w = philox_blocks((seed, stream), 0, nb).astype(np.uint64)
    ua = (((w[:, 1] << np.uint64(32)) | w[:, 0]) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    ub = (((w[:, 3] << np.uint64(32)) | w[:, 2]) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(1.0 - ua))
    phi = 2.0 * np.pi * ub
    z = np.empty(2 * nb, dtype=np.float64)
    z[0::2] = rho * np.cos(phi)
    z[1::2] = rho * np.sin(phi)
    return z[:count].astype(np.float32)
