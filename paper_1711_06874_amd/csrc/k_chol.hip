// Separable (rank-1 Kronecker) covariance C = C_1 (x) C_2 (x) C_3 (Sec. 4, "Separable covariance
// matrices"): the 1-D factors, their Cholesky factors, log-determinants and inverses.  The
// products that apply them along a mode of an n1 x n2 x n3 vector run on the FP64 small-product
// kernel (k_small.hip).
//
// Cholesky: blocked right-looking, CB = 64 columns per step.  One work-group factors the
// diagonal block in LDS (column by column: pivot, scaling, rank-1 update of the block's
// trailing part) and also forms the inverse of its triangular factor; the panel below is then
// L21 = A21 L11^-T as one product with that inverse, and the trailing matrix takes
// A22 -= L21 L21^T as another.  A pivot that is not positive records its index (plus one)
// in `info` and the factor turns to NaN from there on.
#include "tk_kernels.h"

namespace tk {

namespace {
constexpr int CB = 64;
}

// C[i][j] = k(|x_i - x_j|) + nugget [i == j] on the nodes x_i = x0 + i h (the grid's own
// coordinates, so |x_i - x_j| is the node distance the 3-D grid sees on this axis).
__global__ void __launch_bounds__(256) k_cov1d(double* __restrict__ C, int n, double x0, double h, KernelParams kp,
                                               double nugget)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (long)i * n);
    const double xi = x0 + (double)i * h, xj = x0 + (double)j * h;
    double v = cov_value(kp, fabs(xi - xj));
    if (i == j) v += nugget;
    C[e] = v;
}

// Factor the nb x nb diagonal block at (k0, k0) of A (row-major, ld n) in place, zero its strict
// upper part, and write the inverse of its lower-triangular factor to inv (nb x nb, ld CB).
__global__ void __launch_bounds__(256) k_potrf_block(double* __restrict__ A, int n, int k0, int nb,
                                                     double* __restrict__ inv, int* __restrict__ info)
{
    __shared__ double L[CB][CB + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < nb * nb; e += 256) {
        const int r = e / nb, c = e - r * nb;
        L[r][c] = (c <= r) ? A[(long)(k0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            const double d = L[j][j];
            if (!(d > 0.0) && *info == 0) *info = k0 + j + 1;
            L[j][j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < nb; i += 256) L[i][j] /= L[j][j];
        __syncthreads();
        const int m = nb - j - 1;
        for (int e = tid; e < m * m; e += 256) {
            const int i = j + 1 + e / m, c = j + 1 + e % m;
            if (c <= i) L[i][c] -= L[i][j] * L[c][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int r = e / nb, c = e - r * nb;
        A[(long)(k0 + r) * n + k0 + c] = (c <= r) ? L[r][c] : 0.0;
    }
    // inv = L^-1, column c by forward substitution in thread c (it reads back only its own
    // column, so no barrier is needed)
    if (tid < nb) {
        const int c = tid;
        for (int i = 0; i < nb; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= L[i][k] * inv[(long)k * CB + c];
            inv[(long)i * CB + c] = (i < c) ? 0.0 : v / L[i][i];
        }
    }
}

// A21 (rows x nb at (k0 + nb, k0), ld n) = T (rows x nb, ld CB)
__global__ void __launch_bounds__(256) k_store_panel(double* __restrict__ A, int n, int k0, int nb, int rows,
                                                     const double* __restrict__ T)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * nb) return;
    const int r = (int)(e / nb), c = (int)(e - (long)r * nb);
    A[(long)(k0 + nb + r) * n + k0 + c] = T[(long)r * CB + c];
}

// Zero the strict upper triangle of A (the trailing updates write full squares).
__global__ void __launch_bounds__(256) k_zero_upper(double* __restrict__ A, int n)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (long)i * n);
    if (j > i) A[e] = 0.0;
}

// out[0] = 2 sum_i log L[i][i] (fixed order: per-thread strided sums, then a fixed tree)
__global__ void __launch_bounds__(256) k_logdet(const double* __restrict__ L, int n, double* __restrict__ out)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += log(L[(long)i * n + i]);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = 2.0 * ((red[0] + red[1]) + (red[2] + red[3]));
}

// X = L^-1 for a lower-triangular n x n L (row-major): column j by forward substitution in
// thread j; X is zero above the diagonal.  Every lane of a wave runs the same row loop (rows
// above its own column contribute zeros), so the L entries are wave-wide broadcasts.
__global__ void __launch_bounds__(256) k_trinv(const double* __restrict__ L, int n, double* __restrict__ X)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = j < n;
    const int jj = live ? j : 0;
    const int jw = (blockIdx.x * blockDim.x + (threadIdx.x & ~63));   // first column of the wave
    for (int i = 0; i < n; ++i) {
        double v = (i == jj) ? 1.0 : 0.0;
        if (i >= jw) {
            for (int k = jw; k < i; ++k) v -= L[(long)i * n + k] * (live && k >= jj ? X[(long)k * n + jj] : 0.0);
        }
        if (live) X[(long)i * n + jj] = (i < jj) ? 0.0 : v / L[(long)i * n + i];
    }
}

hipError_t launch_cov1d(double* C, int n, double x0, double h, const KernelParams& kp, double nugget, hipStream_t s)
{
    const long tot = (long)n * n;
    hipLaunchKernelGGL(k_cov1d, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, C, n, x0, h, kp, nugget);
    return hipGetLastError();
}

size_t cholesky_work_bytes(int n) { return sizeof(double) * ((size_t)CB * CB + (size_t)n * CB) + 256; }

hipError_t launch_cholesky(double* A, int n, void* work, int* info, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    double* inv = (double*)work;
    double* T = inv + CB * CB;
    hipError_t e;
    for (int k0 = 0; k0 < n; k0 += CB) {
        const int nb = (n - k0 < CB) ? n - k0 : CB;
        hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(256), 0, s, A, n, k0, nb, inv, info);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int rows = n - k0 - nb;
        if (rows <= 0) break;
        // T = A21 L11^-T
        GemmArgs g{};
        g.M = rows; g.N = nb; g.K = nb; g.batch = 1;
        g.A = A + (long)(k0 + nb) * n + k0; g.sAm = n; g.sAk = 1;
        g.B = inv; g.sBk = 1; g.sBn = CB;
        g.C = T; g.sCm = CB; g.sCn = 1;
        g.alpha = 1.0; g.beta = 0.0;
        if ((e = launch_gemm<double, double, double>(g, s)) != hipSuccess) return e;
        const long pt = (long)rows * nb;
        hipLaunchKernelGGL(k_store_panel, dim3((unsigned)((pt + 255) / 256)), dim3(256), 0, s, A, n, k0, nb, rows, T);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // A22 -= T T^T
        GemmArgs u{};
        u.M = rows; u.N = rows; u.K = nb; u.batch = 1;
        u.A = T; u.sAm = CB; u.sAk = 1;
        u.B = T; u.sBk = 1; u.sBn = CB;
        u.C = A + (long)(k0 + nb) * n + k0 + nb; u.sCm = n; u.sCn = 1;
        u.alpha = -1.0; u.beta = 1.0;
        if ((e = launch_gemm<double, double, double>(u, s)) != hipSuccess) return e;
    }
    const long tot = (long)n * n;
    hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A, n);
    return hipGetLastError();
}

hipError_t launch_logdet_chol(const double* L, int n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_logdet, dim3(1), dim3(256), 0, s, L, n, out);
    return hipGetLastError();
}

hipError_t launch_trinv(const double* L, int n, double* X, hipStream_t s)
{
    hipLaunchKernelGGL(k_trinv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L, n, X);
    return hipGetLastError();
}

}  // namespace tk
