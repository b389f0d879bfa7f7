// Separable (rank-1 Kronecker) covariance C = C_1 (x) C_2 (x) C_3 (Sec. 4, "Separable covariance
// matrices"): the 1-D factors, their Cholesky factors, log-determinants and inverses.  The
// products that apply them along a mode of an n1 x n2 x n3 vector run on the FP64 small-product
// kernel (k_small.hip).
//
// Cholesky: blocked right-looking, CB = 64 columns per step.  One wavefront factors the
// diagonal block (rows in registers: pivot, scaling, rank-1 update of the block's trailing
// part); the panel below is then L21 = A21 L11^-T by forward substitution, one thread per row
// (k_trsm_panel), and the lower tiles of the trailing matrix take A22 -= L21 L21^T on FP64 MFMA
// (k_syrk_lower).  A pivot that is not positive records its index (plus one) in `info` and the
// factor turns to NaN from there on.
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

// Factor the nb x nb diagonal block at (k0, k0) of A (row-major, ld n) in place and zero its
// strict upper part.  One wavefront, lane i holding row i of the block in registers (the column
// loops are unrolled, so every register index is static).  Column j: the pivot comes from lane j,
// the lanes below scale their entry, publish it in LDS, and update their row with the broadcast
// column.  A wavefront orders its own LDS accesses, so no barrier is needed.
__global__ void __launch_bounds__(64) k_potrf_block(double* __restrict__ A, int n, int k0, int nb,
                                                    int* __restrict__ info)
{
    __shared__ double col[CB];
    __shared__ double Ls[CB][CB + 1];
    const int i = threadIdx.x;
    const bool live = i < nb;
    double a[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) a[c] = (live && c <= i && c < nb) ? A[(long)(k0 + i) * n + k0 + c] : 0.0;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        if (j < nb) {
            const double d = __shfl(a[j], j, 64);
            if (i == 0 && !(d > 0.0) && *info == 0) *info = k0 + j + 1;
            const double ljj = sqrt(d);
            const double lij = (i > j) ? a[j] / ljj : (i == j ? ljj : 0.0);
            a[j] = lij;
            col[i] = (i > j && live) ? lij : 0.0;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = j + 1; c < CB; ++c) a[c] -= lij * col[c];
            __builtin_amdgcn_wave_barrier();
        }
    }
    // rows to LDS (lower triangle, zeros above), then out to A row by row (coalesced)
#pragma unroll
    for (int c = 0; c < CB; ++c) Ls[i][c] = (c <= i) ? a[c] : 0.0;
    __builtin_amdgcn_wave_barrier();
    for (int r = 0; r < nb; ++r)
        if (live) A[(long)(k0 + r) * n + k0 + i] = Ls[r][i];
}

// The panel below the diagonal block: L21 = A21 L11^-T, row by row (L11 y^T = x^T by forward
// substitution, one thread per row, L11 staged in LDS), written to A21 (ld n) and to T (ld CB)
// for the trailing update.  Only full CB x CB diagonal blocks have a panel below them.
__global__ void __launch_bounds__(256) k_trsm_panel(double* __restrict__ A, int n, int k0, int rows,
                                                    double* __restrict__ T)
{
    __shared__ double Ls[CB][CB + 1];
    __shared__ double rdiag[CB];
    for (int e = threadIdx.x; e < CB * CB; e += 256) {
        const int r = e / CB, c = e - r * CB;
        Ls[r][c] = (c <= r) ? A[(long)(k0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < CB) rdiag[threadIdx.x] = 1.0 / Ls[threadIdx.x][threadIdx.x];
    __syncthreads();
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    double* x = A + (long)(k0 + CB + r) * n + k0;
    double y[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) y[j] = x[j];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        double v = y[j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= y[k] * Ls[j][k];
        y[j] = v * rdiag[j];
    }
    double* t = T + (long)r * CB;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        x[j] = y[j];
        t[j] = y[j];
    }
}

// Trailing update of the blocked factorisation, lower tiles only: C[i][j] -= sum_k T[i][k] T[j][k]
// for the 64 x 64 tiles (ti >= tj) of the rows x rows matrix C (ld n); T is rows x nb (ld CB).
// Tiles above the diagonal are skipped: the factorisation reads only the lower part, and the
// strict upper part is cleared at the end.  One work-group per tile: the two T panels are staged
// in LDS k-major, 32 k at a time, and four waves each form a 32 x 32 block from 2 x 2 FP64 MFMA
// 16 x 16 accumulators.
constexpr int SB = 64;
constexpr int SK = 32;
__global__ void __launch_bounds__(256) k_syrk_lower(double* __restrict__ C, int n, int rows,
                                                   const double* __restrict__ T, int nb)
{
    __shared__ double As[SK][SB + 1], Bs[SK][SB + 1];
    const int pidx = blockIdx.x;
    int ti = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= pidx) ++ti;
    while (ti * (ti + 1) / 2 > pidx) --ti;
    const int tj = pidx - ti * (ti + 1) / 2;
    const int r0a = ti * SB, r0b = tj * SB;
    const bool diag = (ti == tj);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    f64x4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < nb; kc += SK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < SB * SK / 256; ++q) {
            const int e = tid + 256 * q, m = e / SK, k = e - m * SK;
            const int ra = r0a + m, rb = r0b + m, kg = kc + k;
            As[k][m] = (ra < rows && kg < nb) ? T[(long)ra * CB + kg] : 0.0;
            if (!diag) Bs[k][m] = (rb < rows && kg < nb) ? T[(long)rb * CB + kg] : 0.0;
        }
        __syncthreads();
        const double (*Bp)[SB + 1] = diag ? As : Bs;
#pragma unroll
        for (int ks = 0; ks < SK; ks += 4) {
            const int kr = ks + (lane >> 4);
            const double a0 = As[kr][wm + (lane & 15)], a1 = As[kr][wm + 16 + (lane & 15)];
            const double b0 = Bp[kr][wn + (lane & 15)], b1 = Bp[kr][wn + 16 + (lane & 15)];
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = r0a + wm + 16 * bi + 4 * v + (lane >> 4);
                const int gj = r0b + wn + 16 * bj + (lane & 15);
                if (gi < rows && gj < rows) C[(long)gi * n + gj] -= acc[bi * 2 + bj][v];
            }
}

// Zero the strict upper triangle of A (the trailing updates leave values above the diagonal).
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

// Diagonal block b of X = L^-1 (lower-triangular, row-major, ld n): the inverse of the
// nb x nb block L_bb, lane c taking column c by forward substitution on the block in LDS.
__global__ void __launch_bounds__(64) k_trinv_diag(const double* __restrict__ L, int n, double* __restrict__ X)
{
    __shared__ double Ls[CB][CB + 1];
    const int r0 = blockIdx.x * CB;
    const int nb = min(CB, n - r0);
    const int i = threadIdx.x;
    const bool live = i < nb;
    for (int r = 0; r < nb; ++r) Ls[r][i] = live ? L[(long)(r0 + r) * n + r0 + i] : 0.0;
    __builtin_amdgcn_wave_barrier();
    double x[CB];
#pragma unroll
    for (int r = 0; r < CB; ++r) {
        double v = (r == i) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < r; ++k) v -= Ls[r][k] * x[k];
        x[r] = (r < i || r >= nb) ? 0.0 : v / Ls[r][r];
        if (live && r < nb) X[(long)(r0 + r) * n + r0 + i] = x[r];
    }
}

hipError_t launch_cov1d(double* C, int n, double x0, double h, const KernelParams& kp, double nugget, hipStream_t s)
{
    const long tot = (long)n * n;
    hipLaunchKernelGGL(k_cov1d, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, C, n, x0, h, kp, nugget);
    return hipGetLastError();
}

size_t cholesky_work_bytes(int n) { return sizeof(double) * ((size_t)n * CB) + 256; }

hipError_t launch_cholesky(double* A, int n, void* work, int* info, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    double* T = (double*)work;
    hipError_t e;
    for (int k0 = 0; k0 < n; k0 += CB) {
        const int nb = (n - k0 < CB) ? n - k0 : CB;
        hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(64), 0, s, A, n, k0, nb, info);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int rows = n - k0 - nb;
        if (rows <= 0) break;
        // L21 = A21 L11^-T, into A and T (a panel follows only full blocks: nb == CB here)
        hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, A, n, k0, rows, T);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // A22 -= T T^T (lower tiles)
        const long nt = (rows + SB - 1) / SB;
        hipLaunchKernelGGL(k_syrk_lower, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s,
                           A + (long)(k0 + nb) * n + k0 + nb, n, rows, (const double*)T, nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
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

// Blocked: X's strict upper part is cleared, the diagonal blocks are inverted in one launch,
// then block row b (b = 1, 2, ...) takes X[b, 0:b] = -X_bb (L[b, 0:b] X[0:b, 0:b]) as two
// products (X[0:b, 0:b] is final by then).  work: CB x n doubles.
hipError_t launch_trinv(const double* L, int n, double* X, double* work, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    const long tot = (long)n * n;
    hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nbk = (n + CB - 1) / CB;
    hipLaunchKernelGGL(k_trinv_diag, dim3(nbk), dim3(64), 0, s, L, n, X);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int bi = 1; bi < nbk; ++bi) {
        const int r0 = bi * CB, rows = (n - r0 < CB) ? n - r0 : CB;
        // work (rows x r0, ld r0) = L[r0:r0+rows, 0:r0] X[0:r0, 0:r0]
        GemmArgs g{};
        g.M = rows; g.N = r0; g.K = r0; g.batch = 1;
        g.A = L + (long)r0 * n; g.sAm = n; g.sAk = 1;
        g.B = X; g.sBk = n; g.sBn = 1;
        g.C = work; g.sCm = r0; g.sCn = 1;
        g.alpha = 1.0; g.beta = 0.0;
        if ((e = launch_gemm<double, double, double>(g, s)) != hipSuccess) return e;
        // X[r0:r0+rows, 0:r0] = -X_bb work
        GemmArgs h{};
        h.M = rows; h.N = r0; h.K = rows; h.batch = 1;
        h.A = X + (long)r0 * n + r0; h.sAm = n; h.sAk = 1;
        h.B = work; h.sBk = r0; h.sBn = 1;
        h.C = X + (long)r0 * n; h.sCm = n; h.sCn = 1;
        h.alpha = -1.0; h.beta = 0.0;
        if ((e = launch_gemm<double, double, double>(h, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tk
