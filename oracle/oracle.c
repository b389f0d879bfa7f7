/*
 * FP64 CPU oracle for the Tucker compression of Matern / Slater covariance tensors.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file;
 * it exists so that tests, the smoke check and the benchmark's CPU-baseline leg can compare
 * the GPU library against a plain, slow, obviously correct implementation.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Paper: Litvinenko, Keyes, Khoromskaia, Khoromskij, Matthies, "Tucker tensor analysis of
 * Matern functions in spatial statistics" (arXiv 1711.06874).
 *
 * Everything here is IEEE double with explicit loops: no BLAS, no LAPACK.  Where OpenMP is
 * used, every output element is produced by exactly one thread with a fixed summation order,
 * so the results do not depend on the thread count.
 *
 * Layout conventions: a tensor X of dims (d0,d1,d2) is C-order (last index fastest).
 * Matrices are row-major.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------ */
/* Covariance functions                                                                 */
/* ------------------------------------------------------------------------------------ */

/* Modified Bessel function of the second kind at half-integer order nu = m + 1/2, from the
 * terminating series  K_{m+1/2}(x) = sqrt(pi/(2x)) e^{-x} sum_{k=0}^{m} (m+k)!/(k!(m-k)!) (2x)^{-k}
 * (Abramowitz & Stegun 10.2.15 / DLMF 10.49.12).  Valid for x > 0. */
static double bessel_k_half_integer(int m, double x)
{
    double sum = 0.0;
    for (int k = 0; k <= m; ++k) {
        double fact_mk = 1.0, fact_k = 1.0, fact_m_k = 1.0;
        for (int i = 2; i <= m + k; ++i) fact_mk *= i;
        for (int i = 2; i <= k; ++i) fact_k *= i;
        for (int i = 2; i <= m - k; ++i) fact_m_k *= i;
        sum += fact_mk / (fact_k * fact_m_k) * pow(2.0 * x, -(double)k);
    }
    return sqrt(M_PI / (2.0 * x)) * exp(-x) * sum;
}

/* K_nu(x) for any real order and x > 0 from the integral representation
 *   K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt          (DLMF 10.32.9),
 * summed by the trapezoidal rule.  The integrand is even and analytic in the strip
 * |Im t| < pi/2 (where Re cosh t > 0); relative to its value at t = 0 it stays bounded in the
 * strip |Im t| < min(pi/4, 1/sqrt(x)) (there exp(-x cosh t) grows by at most exp(x(1 - cos y))),
 * so the rule with step h = min(1/16, 0.1/sqrt(x)) errs by about exp(-2 pi d / h) <= e^-39
 * relative.  Every term is positive, so the sum is accurate to a few ulp.  Summation stops
 * once x cosh t - |nu| t exceeds 760 and grows (the rest of the terms lie below the double
 * range).  A plain, slow route: hundreds of exponentials per value. */
double tko_bessel_k(double nu, double x)
{
    const double h = fmin(1.0 / 16.0, 0.1 / sqrt(x));
    nu = fabs(nu);
    if (!(x > 0.0)) return NAN;
    /* compensated (Kahan) summation: hundreds of terms would otherwise add ~n u of rounding */
    double sum = 0.5 * exp(-x), comp = 0.0;   /* t = 0 carries half weight (even integrand) */
    for (int k = 1; k < 1000000; ++k) {
        double t = k * h;
        double e = -x * cosh(t);
        double term = 0.5 * (exp(e + nu * t) + exp(e - nu * t)) - comp;
        double next = sum + term;
        comp = (next - sum) - term;
        sum = next;
        if (-e - nu * t > 760.0 && x * sinh(t) > nu) break;
    }
    return sum * h;
}

/* Matern covariance, Sec. 2.2 eq. (2.3):
 *   C_{nu,ell}(r) = 2^{1-nu}/Gamma(nu) * (sqrt(2 nu) r/ell)^nu * K_nu(sqrt(2 nu) r/ell),
 * scaled by the variance sigma2.  Half-integer nu = m + 1/2 (m <= 8) takes the terminating
 * Bessel series; any other nu > 0 the integral above.  The value at r = 0 is the limit sigma2.
 * Returns NaN for nu <= 0. */
double tko_matern(double nu, double ell, double sigma2, double r)
{
    if (!(nu > 0.0)) return NAN;
    if (r == 0.0) return sigma2;
    double s = sqrt(2.0 * nu) * r / ell;
    int m = (int)floor(nu);
    double k;
    if (fabs(nu - (m + 0.5)) <= 1e-12 && m <= 8) k = bessel_k_half_integer(m, s);
    else k = tko_bessel_k(nu, s);
    /* 2^{1-nu}/Gamma(nu) s^nu in log form (s^nu alone may overflow for large nu) */
    double c = exp((1.0 - nu) * log(2.0) - lgamma(nu) + nu * log(s)) * k;
    return sigma2 * c;
}

/* Matern spectral density in d = 3 (the Fourier side of Diagram 1 in Sec. 2.2; Sec. 3.7
 * eq. (3.28) with its constant written out):
 *   f_{alpha,nu}(rho) = Gamma(nu + 3/2) alpha^{2 nu} / (pi^{3/2} Gamma(nu)) (alpha^2 + rho^2)^{-(nu + 3/2)},
 * a probability density on R^3, scaled by sigma2. */
double tko_spectral(double nu, double alpha, double sigma2, double rho)
{
    if (!(nu > 0.0) || !(alpha > 0.0)) return NAN;
    double lc = lgamma(nu + 1.5) - lgamma(nu) + 2.0 * nu * log(alpha) - 1.5 * log(M_PI);
    return sigma2 * exp(lc - (nu + 1.5) * log(alpha * alpha + rho * rho));
}

/* p-Slater function, Sec. 3.7 eq. (3.27): C(r) = exp(-r^p), generalised here with an
 * amplitude sigma2, a rate alpha and a length ell:  sigma2 * exp(-alpha * (r/ell)^p).  */
double tko_slater(double alpha, double p, double ell, double sigma2, double r)
{
    if (r == 0.0) return sigma2;
    return sigma2 * exp(-alpha * pow(r / ell, p));
}

/* Gaussian covariance (the nu -> infinity limit named in Sec. 2.2; the separable rank-1
 * example of Sec. 4.4):  sigma2 * exp(-(r/ell)^2). */
double tko_gauss(double ell, double sigma2, double r)
{
    double t = r / ell;
    return sigma2 * exp(-(t * t));
}

/* family: 0 = Matern, 1 = Slater, 2 = Gauss, 3 = Matern spectral density (alpha, nu) */
double tko_kernel(int family, double nu, double ell, double sigma2, double alpha, double p,
                  double r)
{
    switch (family) {
    case 0: return tko_matern(nu, ell, sigma2, r);
    case 1: return tko_slater(alpha, p, ell, sigma2, r);
    case 2: return tko_gauss(ell, sigma2, r);
    case 3: return tko_spectral(nu, alpha, sigma2, r);
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Collocation grid and tensor, Sec. 3.7 eq. (3.25)                                      */
/* ------------------------------------------------------------------------------------ */

/* Node coordinates along one axis.  layout 0 (centred): x_i = -b + i h, i = 0..n-1, with
 * h = 2b/(n-1) (the paper's vertex grid, written 0-based).  layout 1 (offset): x_i = i h with
 * the same h, i.e. every difference between two nodes of the centred grid. */
void tko_grid_coords(int n, double b, int layout, double *x)
{
    double h = 2.0 * b / (double)(n - 1);
    for (int i = 0; i < n; ++i) x[i] = (layout == 0) ? (-b + (double)i * h) : ((double)i * h);
}

/* A[i0,i1,i2] = k(r) with r = sqrt((a0 x^2 + a1 y^2) + a2 z^2): the anisotropic distance of
 * Sec. 2.2 with a positive diagonal metric a (metric == NULL: the identity, r = ||x||). */
void tko_grid_eval_metric(int family, double nu, double ell, double sigma2, double alpha, double p,
                          const int n[3], const double b[3], int layout, const double *metric,
                          double *A)
{
    double a0 = metric ? metric[0] : 1.0, a1 = metric ? metric[1] : 1.0, a2 = metric ? metric[2] : 1.0;
    double *x = (double *)malloc(sizeof(double) * (size_t)(n[0] + n[1] + n[2]));
    double *y = x + n[0], *z = y + n[1];
    tko_grid_coords(n[0], b[0], layout, x);
    tko_grid_coords(n[1], b[1], layout, y);
    tko_grid_coords(n[2], b[2], layout, z);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n[0]; ++i)
        for (int j = 0; j < n[1]; ++j)
            for (int k = 0; k < n[2]; ++k) {
                double r = sqrt((a0 * x[i] * x[i] + a1 * y[j] * y[j]) + a2 * z[k] * z[k]);
                A[((size_t)i * n[1] + j) * n[2] + k] =
                    tko_kernel(family, nu, ell, sigma2, alpha, p, r);
            }
    free(x);
}

/* A[i0,i1,i2] = k(||(x_i0, y_i1, z_i2)||) with r = sqrt((x^2 + y^2) + z^2). */
void tko_grid_eval(int family, double nu, double ell, double sigma2, double alpha, double p,
                   const int n[3], const double b[3], int layout, double *A)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)(n[0] + n[1] + n[2]));
    double *y = x + n[0], *z = y + n[1];
    tko_grid_coords(n[0], b[0], layout, x);
    tko_grid_coords(n[1], b[1], layout, y);
    tko_grid_coords(n[2], b[2], layout, z);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n[0]; ++i)
        for (int j = 0; j < n[1]; ++j)
            for (int k = 0; k < n[2]; ++k) {
                double r = sqrt((x[i] * x[i] + y[j] * y[j]) + z[k] * z[k]);
                A[((size_t)i * n[1] + j) * n[2] + k] =
                    tko_kernel(family, nu, ell, sigma2, alpha, p, r);
            }
    free(x);
}

/* ------------------------------------------------------------------------------------ */
/* Unfolding and Gram matrices, Sec. 3.2 (HOSVD works on the unfoldings A_(k))           */
/* ------------------------------------------------------------------------------------ */

/* Mode-k unfolding: the n_k x (prod of the other two dims) matrix whose row i holds every
 * entry of X with index i in mode k; columns run over the remaining two indices in their
 * natural (C) order. */
void tko_unfold(const double *X, const int d[3], int mode, double *M)
{
    int a = (mode == 0) ? 1 : 0;           /* the two remaining modes, in order */
    int c = (mode == 2) ? 1 : 2;
    size_t cols = (size_t)d[a] * d[c];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < d[mode]; ++i)
        for (int u = 0; u < d[a]; ++u)
            for (int v = 0; v < d[c]; ++v) {
                int idx[3];
                idx[mode] = i; idx[a] = u; idx[c] = v;
                M[(size_t)i * cols + (size_t)u * d[c] + v] =
                    X[((size_t)idx[0] * d[1] + idx[1]) * d[2] + idx[2]];
            }
}

/* Blocked dot product: blocks of 256 terms, each summed left to right, then the block sums
 * left to right.  Fixed order, independent of threading. */
static double dot_blocked(const double *a, const double *b, size_t len)
{
    double total = 0.0;
    for (size_t s = 0; s < len; s += 256) {
        size_t e = (s + 256 < len) ? s + 256 : len;
        double part = 0.0;
        for (size_t t = s; t < e; ++t) part += a[t] * b[t];
        total += part;
    }
    return total;
}

/* G = M M^T for a rows x cols row-major M (full symmetric result). */
void tko_gram_rows(const double *M, int rows, size_t cols, double *G)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < rows; ++i)
        for (int j = i; j < rows; ++j) {
            double v = dot_blocked(M + (size_t)i * cols, M + (size_t)j * cols, cols);
            G[(size_t)i * rows + j] = v;
            G[(size_t)j * rows + i] = v;
        }
}

/* G_k = A_(k) A_(k)^T  (n_k x n_k). */
void tko_gram(const double *X, const int d[3], int mode, double *G)
{
    size_t cols = (size_t)d[0] * d[1] * d[2] / (size_t)d[mode];
    double *M = (double *)malloc(sizeof(double) * (size_t)d[mode] * cols);
    tko_unfold(X, d, mode, M);
    tko_gram_rows(M, d[mode], cols, G);
    free(M);
}

/* ------------------------------------------------------------------------------------ */
/* Symmetric eigensolver: two-sided Jacobi with parallel (round-robin) ordering           */
/* (Golub & Van Loan, "Matrix Computations", symmetric Jacobi: sym.schur2 rotations;    */
/* the parallel ordering applies n/2 disjoint rotations per step).                      */
/* ------------------------------------------------------------------------------------ */

static double off_norm(const double *A, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double row = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != i) row += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        s += row;
    }
    return sqrt(s);
}

static double fro_norm(const double *A, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double row = 0.0;
        for (int j = 0; j < n; ++j) row += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        s += row;
    }
    return sqrt(s);
}

/* Full eigendecomposition of the symmetric n x n matrix S (row-major, not modified).
 * On return lambda[0..n-1] is in descending order (stable sort) and V (n x n row-major)
 * holds the matching unit eigenvectors in its columns, each signed so that its entry of
 * largest magnitude is positive (entries within 1e-10 relative of that maximum count as
 * ties, and the lowest index among them decides).
 * Stops when off(A) <= max(tol, n u) * ||S||_F (u = 2^-52) or after max_sweeps sweeps;
 * returns the number of sweeps done (or -1 if it did not converge). */
int tko_jacobi_eig(int n, const double *S, double *lambda, double *V, int max_sweeps, double tol)
{
    int m = n + (n & 1);                    /* round-robin needs an even player count */
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *W = (double *)malloc(sizeof(double) * (size_t)n * n);   /* W = V^T: row j = vector j */
    int *pp = (int *)malloc(sizeof(int) * (size_t)(m / 2));
    int *qq = (int *)malloc(sizeof(int) * (size_t)(m / 2));
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    memcpy(A, S, sizeof(double) * (size_t)n * n);
    memset(W, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) W[(size_t)i * n + i] = 1.0;

    /* off(A) cannot be driven much below n u ||A||_F in floating point (each rotation leaves
     * O(u) residue in the rows it touches), so the tolerance is never set below that level */
    if (tol < (double)n * 2.220446049250313e-16) tol = (double)n * 2.220446049250313e-16;
    double fnorm = fro_norm(A, n);
    int sweeps = 0, converged = 0;
    if (n == 1 || off_norm(A, n) <= tol * fnorm) converged = 1;
    while (!converged && sweeps < max_sweeps) {
        for (int step = 0; step < m - 1; ++step) {
            /* circle-method pairing for this step */
            int np = 0;
            for (int k = 0; k < m / 2; ++k) {
                int a, b;
                if (k == 0) { a = m - 1; b = step; }
                else { a = (step + k) % (m - 1); b = (step - k + (m - 1)) % (m - 1); }
                if (a >= n || b >= n) continue;        /* the dummy player when n is odd */
                if (a > b) { int t = a; a = b; b = t; }
                pp[np] = a; qq[np] = b; ++np;
            }
            /* rotation angles from the current matrix (sym.schur2) */
            for (int k = 0; k < np; ++k) {
                int p = pp[k], q = qq[k];
                double apq = A[(size_t)p * n + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    double tau = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
                    double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                            : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                cs[2 * k] = c; cs[2 * k + 1] = s;
            }
            /* A <- J^T A : rows p, q */
#pragma omp parallel for schedule(static)
            for (int k = 0; k < np; ++k) {
                int p = pp[k], q = qq[k];
                double c = cs[2 * k], s = cs[2 * k + 1];
                if (s == 0.0) continue;
                double *rp = A + (size_t)p * n, *rq = A + (size_t)q * n;
                for (int j = 0; j < n; ++j) {
                    double x = rp[j], y = rq[j];
                    rp[j] = c * x - s * y;
                    rq[j] = s * x + c * y;
                }
                double *wp = W + (size_t)p * n, *wq = W + (size_t)q * n;  /* V <- V J */
                for (int j = 0; j < n; ++j) {
                    double x = wp[j], y = wq[j];
                    wp[j] = c * x - s * y;
                    wq[j] = s * x + c * y;
                }
            }
            /* A <- A J : columns p, q */
#pragma omp parallel for schedule(static)
            for (int i = 0; i < n; ++i) {
                double *row = A + (size_t)i * n;
                for (int k = 0; k < np; ++k) {
                    double c = cs[2 * k], s = cs[2 * k + 1];
                    if (s == 0.0) continue;
                    int p = pp[k], q = qq[k];
                    double x = row[p], y = row[q];
                    row[p] = c * x - s * y;
                    row[q] = s * x + c * y;
                }
            }
        }
        ++sweeps;
        if (off_norm(A, n) <= tol * fnorm) converged = 1;
    }

    /* stable sort by descending eigenvalue */
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 1; i < n; ++i) {                     /* insertion sort: stable */
        int key = order[i];
        double kv = A[(size_t)key * n + key];
        int j = i - 1;
        while (j >= 0 && A[(size_t)order[j] * n + order[j]] < kv) { order[j + 1] = order[j]; --j; }
        order[j + 1] = key;
    }
    for (int jj = 0; jj < n; ++jj) {
        int src = order[jj];
        lambda[jj] = A[(size_t)src * n + src];
        const double *w = W + (size_t)src * n;
        double amax = 0.0;
        for (int i = 0; i < n; ++i) if (fabs(w[i]) > amax) amax = fabs(w[i]);
        int lead = 0;
        for (int i = 0; i < n; ++i)
            if (fabs(w[i]) >= amax * (1.0 - 1e-10)) { lead = i; break; }
        double sgn = (w[lead] < 0.0) ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) V[(size_t)i * n + jj] = sgn * w[i];
    }
    free(order); free(cs); free(qq); free(pp); free(W); free(A);
    return converged ? sweeps : -1;
}

/* ------------------------------------------------------------------------------------ */
/* Mode-k product, Sec. 3.1 (contracted product notation, eq. (3.3)-(3.4))               */
/* ------------------------------------------------------------------------------------ */

/* Y = X x_k M, with M a J x d[k] row-major matrix: Y[..j..] = sum_i M[j][i] X[..i..].
 * Y has dims d with d[k] replaced by J.  The projection X x_k U^T uses M = U^T; the
 * reconstruction core x_k U uses M = U. */
void tko_mode_product(const double *X, const int d[3], int mode, const double *M, int J,
                      double *Y)
{
    int e[3] = {d[0], d[1], d[2]};
    e[mode] = J;
    size_t xs[3] = {(size_t)d[1] * d[2], (size_t)d[2], 1};   /* strides of X */
#pragma omp parallel for schedule(static)
    for (int i0 = 0; i0 < e[0]; ++i0)
        for (int i1 = 0; i1 < e[1]; ++i1)
            for (int i2 = 0; i2 < e[2]; ++i2) {
                int o[3] = {i0, i1, i2};
                int j = o[mode];
                o[mode] = 0;                                   /* X index with mode-k index 0 */
                const double *xb = X + o[0] * xs[0] + o[1] * xs[1] + o[2] * xs[2];
                const double *mrow = M + (size_t)j * d[mode];
                double s = 0.0;
                for (int i = 0; i < d[mode]; ++i) s += mrow[i] * xb[(size_t)i * xs[mode]];
                Y[((size_t)i0 * e[1] + i1) * e[2] + i2] = s;
            }
}

/* Sum of squares of a vector, blocked as in dot_blocked. */
double tko_sumsq(const double *x, size_t len) { return dot_blocked(x, x, len); }

/* ||X - Y||_F^2 with the same blocked order. */
double tko_diff_sumsq(const double *X, const double *Y, size_t len)
{
    double total = 0.0;
    for (size_t s = 0; s < len; s += 256) {
        size_t e = (s + 256 < len) ? s + 256 : len;
        double part = 0.0;
        for (size_t t = s; t < e; ++t) { double d = X[t] - Y[t]; part += d * d; }
        total += part;
    }
    return total;
}

/* ------------------------------------------------------------------------------------ */
/* Covariance operator generated by a tensor on the non-negative offsets, Sec. 3.6      */
/* (eq. (3.16)-(3.18): Kronecker sums of symmetric Toeplitz matrices defined by their    */
/* first columns) and Sec. 4 eq. (4.1).                                                  */
/* ------------------------------------------------------------------------------------ */

/* Q is a generator tensor of dims q[3]; the operator acts on m[0] x m[1] x m[2] points with
 *   C[(i),(j)] = Q[off0 + |i0-j0|, off1 + |i1-j1|, off2 + |i2-j2|].
 * For each requested row index rows[t] (a flat C-order index into the m-grid) it returns
 * y[t] = sum_j C[row, j] z[j], the plain definition of the matrix-vector product. */
void tko_cov_rows(const double *Q, const int q[3], const int off[3], const int m[3],
                  const double *z, const long long *rows, int nrows, double *y)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nrows; ++t) {
        long long r = rows[t];
        int i2 = (int)(r % m[2]);
        int i1 = (int)((r / m[2]) % m[1]);
        int i0 = (int)(r / ((long long)m[2] * m[1]));
        double total = 0.0;
        for (int j0 = 0; j0 < m[0]; ++j0) {
            int a = off[0] + abs(i0 - j0);
            double plane = 0.0;
            for (int j1 = 0; j1 < m[1]; ++j1) {
                int bb = off[1] + abs(i1 - j1);
                const double *qrow = Q + ((size_t)a * q[1] + bb) * q[2];
                const double *zrow = z + ((size_t)j0 * m[1] + j1) * m[2];
                double line = 0.0;
                for (int j2 = 0; j2 < m[2]; ++j2) line += qrow[off[2] + abs(i2 - j2)] * zrow[j2];
                plane += line;
            }
            total += plane;
        }
        y[t] = total;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Separable (rank-1 Kronecker) covariance, Sec. 4 "Separable covariance matrices":      */
/* C = C_1 (x) C_2 (x) C_3, Cholesky, inverse and log-determinant per factor.            */
/* ------------------------------------------------------------------------------------ */

/* In-place Cholesky C = L L^T of a symmetric positive definite n x n matrix (row-major; the
 * lower triangle receives L, the strict upper triangle is zeroed).  Plain column-by-column
 * algorithm: L_jj = sqrt(C_jj - sum_k L_jk^2), L_ij = (C_ij - sum_k L_ik L_jk) / L_jj.
 * Returns 0, or j + 1 if the j-th pivot is not positive. */
int tko_cholesky(int n, double *C)
{
    for (int j = 0; j < n; ++j) {
        double d = C[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= C[(size_t)j * n + k] * C[(size_t)j * n + k];
        if (!(d > 0.0)) return j + 1;
        double ljj = sqrt(d);
        C[(size_t)j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (int i = j + 1; i < n; ++i) {
            double v = C[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= C[(size_t)i * n + k] * C[(size_t)j * n + k];
            C[(size_t)i * n + j] = v / ljj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) C[(size_t)i * n + j] = 0.0;
    return 0;
}

/* Solve (L L^T) x = b for `nrhs` right-hand sides stored as the columns of B (n x nrhs,
 * row-major), in place: forward substitution with L, then back substitution with L^T. */
void tko_chol_solve(int n, const double *L, int nrhs, double *B)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < n; ++i) {
            double v = B[(size_t)i * nrhs + c];
            for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * B[(size_t)k * nrhs + c];
            B[(size_t)i * nrhs + c] = v / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double v = B[(size_t)i * nrhs + c];
            for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * B[(size_t)k * nrhs + c];
            B[(size_t)i * nrhs + c] = v / L[(size_t)i * n + i];
        }
    }
}

int tko_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops (timing runs only: every result is independent of it). */
void tko_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
