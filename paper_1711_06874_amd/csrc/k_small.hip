// Small dense products and reductions used around the big contractions: single-hole
// contractions of the HOOI sweep with the small factors, small Gram matrices B B^T, the
// eigensolver's G Q products, core contractions, conversions and FP64 dot products.
//
// The products are batched, with arbitrary element strides on every operand and FP64
// accumulation on mfma_f64_16x16x4f64: one wavefront computes a (16 TM) x (16 TN) block of one
// item's output (TM, TN in {1, 2}, chosen from M and N so that small ranks do not pay for a
// 32 x 32 block).  Operands are read straight from memory (they are small and cached), four
// k-steps of 4 at a time, all loads of a group issued before its products (for K >= 128 four
// wavefronts split K, their sums added in a fixed order); lane l supplies
// A[m0 + l % 16][k + l / 16] and B[k + l / 16][n0 + l % 16] and receives the outputs of rows
// 4 v + l / 16, column l % 16 of each 16 x 16 tile.  The sum over k (and, in the batch-reducing
// form, over the batch, outermost) runs in a fixed order.
#include "tk_kernels.h"

namespace tk {

namespace {
constexpr int GKU = 4;   // k-steps of 4 whose operands are loaded together
}

// KS wavefronts per block: wavefront w takes the w-th of KS near-equal K ranges (multiples of 16),
// and the KS partial sums are added in the order w = 0, 1, ... through LDS.
template <typename TA, typename TB, typename TC, int TM, int TN, int KS>
__global__ void __launch_bounds__(64 * KS) k_gemm(GemmArgs g)
{
    g.A = bshift(g.A, g.bs);
    g.B = bshift(g.B, g.bs);
    g.C = bshift(g.C, g.bs);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kq = ((g.K + KS - 1) / KS + 4 * GKU - 1) / (4 * GKU) * (4 * GKU);
    const int kbeg = wv * kq, kend = (kbeg + kq < g.K) ? kbeg + kq : g.K;
    const int lr = lane & 15, lk = lane >> 4;
    const int tiles_n = (g.N + 16 * TN - 1) / (16 * TN);
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m0 = tm * 16 * TM, n0 = tn * 16 * TN;
    // batch-reducing form: one output, the batch loop runs inside (fixed order)
    const long b_first = g.reduce_batch ? 0 : (long)blockIdx.y;
    const long b_last = g.reduce_batch ? (long)g.batch : (long)blockIdx.y + 1;
    TC* C = (TC*)g.C + (g.reduce_batch ? 0 : (long)blockIdx.y * g.sCb);
    bool mv[TM], nv[TN];
    long aoff[TM], boff[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + 16 * i + lr;
        mv[i] = gm < g.M;
        aoff[i] = (long)(mv[i] ? gm : 0) * g.sAm;
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int gn = n0 + 16 * j + lr;
        nv[j] = gn < g.N;
        boff[j] = (long)(nv[j] ? gn : 0) * g.sBn;
    }
    f64x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    // k-groups of 4 GKU, double-buffered in registers: the loads of group g + 1 are in flight while
    // group g's products run (the order of the sum over k is unchanged)
    for (long b = b_first; b < b_last; ++b) {
        const TA* A = (const TA*)g.A + b * g.sAb;
        const TB* B = (const TB*)g.B + b * g.sBb;
        auto load = [&](int k0, double (&av)[GKU][TM], double (&bv)[GKU][TN]) {
#pragma unroll
            for (int u = 0; u < GKU; ++u) {
                const int k = k0 + 4 * u + lk;
                const bool kv = k < kend;
#pragma unroll
                for (int i = 0; i < TM; ++i) av[u][i] = (kv && mv[i]) ? (double)A[aoff[i] + (long)k * g.sAk] : 0.0;
#pragma unroll
                for (int j = 0; j < TN; ++j) bv[u][j] = (kv && nv[j]) ? (double)B[(long)k * g.sBk + boff[j]] : 0.0;
            }
        };
        auto products = [&](int k0, const double (&av)[GKU][TM], const double (&bv)[GKU][TN]) {
#pragma unroll
            for (int u = 0; u < GKU; ++u) {
                if (k0 + 4 * u < kend) {
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][i], bv[u][j], acc[i][j], 0, 0, 0);
                }
            }
        };
        double a0[GKU][TM], b0[GKU][TN], a1[GKU][TM], b1[GKU][TN];
        int k0 = kbeg;
        if (k0 < kend) load(k0, a0, b0);
        while (k0 < kend) {
            const int k1 = k0 + 4 * GKU;
            if (k1 < kend) load(k1, a1, b1);
            products(k0, a0, b0);
            if (k1 >= kend) break;
            const int k2 = k1 + 4 * GKU;
            if (k2 < kend) load(k2, a0, b0);
            products(k1, a1, b1);
            k0 = k2;
        }
    }
    if constexpr (KS > 1) {
        __shared__ double part[KS - 1][TM * TN * 4][64];
        if (wv > 0) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) part[wv - 1][(i * TN + j) * 4 + v][lane] = acc[i][j][v];
        }
        __syncthreads();
        if (wv > 0) return;
#pragma unroll
        for (int w = 1; w < KS; ++w)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[i][j][v] += part[w - 1][(i * TN + j) * 4 + v][lane];
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + 16 * i + 4 * v + lk, gn = n0 + 16 * j + lr;
                if (gm < g.M && gn < g.N) {
                    TC* c = C + (long)gm * g.sCm + (long)gn * g.sCn;
                    double val = g.alpha * acc[i][j][v];
                    if (g.beta != 0.0) val += g.beta * (double)(*c);
                    *c = (TC)val;
                }
            }
}

// Products with K >= 128 split K over four wavefronts (a choice that depends on the shape only, so
// one problem and a batch of problems of that shape take the same sums).
template <typename TA, typename TB, typename TC, int TM, int TN>
static hipError_t launch_gemm_tiles(const GemmArgs& a, hipStream_t s)
{
    const long tiles = (long)((a.M + 16 * TM - 1) / (16 * TM)) * ((a.N + 16 * TN - 1) / (16 * TN));
    const unsigned gy = a.reduce_batch ? 1u : (unsigned)a.batch;
    const unsigned gz = a.nb > 1 ? (unsigned)a.nb : 1u;
    if (a.K >= 128)
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TM, TN, 4>), dim3((unsigned)tiles, gy, gz), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TM, TN, 1>), dim3((unsigned)tiles, gy, gz), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename TA, typename TB, typename TC>
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s)
{
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return hipSuccess;
    if (!a.reduce_batch && a.batch > 65535) return hipErrorInvalidValue;
    const bool wm = a.M > 16, wn = a.N > 16;
    if (wm && wn) return launch_gemm_tiles<TA, TB, TC, 2, 2>(a, s);
    if (wm) return launch_gemm_tiles<TA, TB, TC, 2, 1>(a, s);
    if (wn) return launch_gemm_tiles<TA, TB, TC, 1, 2>(a, s);
    return launch_gemm_tiles<TA, TB, TC, 1, 1>(a, s);
}

template hipError_t launch_gemm<double, double, double>(const GemmArgs&, hipStream_t);
template hipError_t launch_gemm<float, double, double>(const GemmArgs&, hipStream_t);
template hipError_t launch_gemm<double, float, double>(const GemmArgs&, hipStream_t);
template hipError_t launch_gemm<double, double, float>(const GemmArgs&, hipStream_t);
template hipError_t launch_gemm<float, float, float>(const GemmArgs&, hipStream_t);
template hipError_t launch_gemm<double, float, float>(const GemmArgs&, hipStream_t);
template hipError_t launch_gemm<float, double, float>(const GemmArgs&, hipStream_t);

// ------------------------------------------------------------------------ conversions ----
__global__ void k_f64_to_f32(const double* __restrict__ x, float* __restrict__ y, long n, long bs)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bshift(y, bs)[i] = (float)bshift(x, bs)[i];
}
__global__ void k_f32_to_f64(const float* __restrict__ x, double* __restrict__ y, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}
__global__ void k_fill_f64(double* __restrict__ x, double v, long n, long bs)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bshift(x, bs)[i] = v;
}
__global__ void k_copy_f64(const double* __restrict__ x, double* __restrict__ y, long n, long bs)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bshift(y, bs)[i] = bshift(x, bs)[i];
}

// dst[b * words + i] = word i of problem b's record at src + b * bs
__global__ void k_gather_u32(const uint32_t* __restrict__ src, long bs, int words, uint32_t* __restrict__ dst)
{
    const int i = threadIdx.x;
    if (i < words) dst[(long)blockIdx.z * words + i] = bshift(src, bs)[i];
}

hipError_t launch_gather_u32(const void* src, long bs, int words, void* dst, int nb, hipStream_t s)
{
    if (words < 1 || words > 64 || nb < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_u32, dim3(1, 1, nb), dim3(64), 0, s, (const uint32_t*)src, bs, words,
                       (uint32_t*)dst);
    return hipGetLastError();
}

hipError_t launch_convert_f64_to_f32(const double* x, float* y, long n, hipStream_t s, Bat bt)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((n + 255) / 256), 1, bt.nb), dim3(256), 0, s, x, y, n, bt.bs);
    return hipGetLastError();
}
hipError_t launch_convert_f32_to_f64(const float* x, double* y, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* x, double v, long n, hipStream_t s, Bat bt)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256), 1, bt.nb), dim3(256), 0, s, x, v, n, bt.bs);
    return hipGetLastError();
}
hipError_t launch_copy_f64(const double* x, double* y, long n, hipStream_t s, Bat bt)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + 255) / 256), 1, bt.nb), dim3(256), 0, s, x, y, n, bt.bs);
    return hipGetLastError();
}

// ------------------------------------------------------------------- dot products ----
// Two-level deterministic reduction: block b sums a fixed strided subset into partials[b],
// then one block adds the partials in order.
template <typename T>
__global__ void __launch_bounds__(256) k_dot_partial(const T* __restrict__ x, const T* __restrict__ y,
                                                     long n, double* __restrict__ partials)
{
    __shared__ double red[4];
    double s = 0.0;
    long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        s += (double)x[i] * (double)y[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partials, int nparts,
                                                         int width, double* __restrict__ out, long bs)
{
    // out[w] = sum_p partials[p * width + w], fixed order per thread then a fixed tree
    __shared__ double red[256];
    partials = bshift(partials, bs);
    out = bshift(out, bs);
    for (int w = 0; w < width; ++w) {
        double s = 0.0;
        for (int p = threadIdx.x; p < nparts; p += 256) s += partials[(long)p * width + w];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[w] = red[0];
        __syncthreads();
    }
}

hipError_t launch_reduce_partials(const double* partials, int nparts, int width, double* out, hipStream_t s, Bat bt)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(1, 1, bt.nb), dim3(256), 0, s, partials, nparts, width, out, bt.bs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T* x, const T* y, long n, double* partials, int nparts, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(nparts), dim3(256), 0, s, x, y, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partials, nparts, 1, out, s);
}
template hipError_t launch_dot<float>(const float*, const float*, long, double*, int, double*, hipStream_t);
template hipError_t launch_dot<double>(const double*, const double*, long, double*, int, double*, hipStream_t);

}  // namespace tk
