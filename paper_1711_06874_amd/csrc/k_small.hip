// Small dense products and reductions used around the big contractions: single-hole
// contractions of the HOOI sweep with the small factors, small Gram matrices B B^T, the
// eigensolver's G Q products, core contractions, conversions and FP64 dot products.
//
// The products are batched, with arbitrary element strides on every operand, FP64
// accumulation and a 32 x 32 output tile per 256-thread work-group (2 x 2 outputs per
// thread); operands are staged through LDS in 64-deep K chunks, the next chunk being loaded into
// registers while the current one is multiplied.
#include "tk_kernels.h"

namespace tk {

namespace {
constexpr int GT = 32;   // output tile edge
constexpr int GK = 64;   // K chunk
}

template <typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g)
{
    constexpr int PER = GT * GK / 256;     // elements of each operand a thread stages per chunk
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    g.A = bshift(g.A, g.bs);
    g.B = bshift(g.B, g.bs);
    g.C = bshift(g.C, g.bs);
    const int tid = threadIdx.x;
    const int tiles_n = (g.N + GT - 1) / GT;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m0 = tm * GT, n0 = tn * GT;
    const int tx = tid % 16, ty = tid / 16;           // outputs (m0 + ty + 16i, n0 + tx + 16j)
    double acc[2][2] = {{0, 0}, {0, 0}};
    // batch-reducing form: one output, the batch loop runs inside (fixed order)
    const long b_first = g.reduce_batch ? 0 : (long)blockIdx.y;
    const long b_last = g.reduce_batch ? (long)g.batch : (long)blockIdx.y + 1;
    TC* C = (TC*)g.C + (g.reduce_batch ? 0 : (long)blockIdx.y * g.sCb);
    const int kchunks = (g.K + GK - 1) / GK;
    const long nchunks = (b_last - b_first) * kchunks;
    // staging positions: consecutive threads walk the unit-stride index of each operand
    int am[PER], ak[PER], bn[PER], bk[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = tid + e * 256;
        if (g.sAm == 1) { am[e] = idx % GT; ak[e] = idx / GT; } else { ak[e] = idx % GK; am[e] = idx / GK; }
        if (g.sBn == 1) { bn[e] = idx % GT; bk[e] = idx / GT; } else { bk[e] = idx % GK; bn[e] = idx / GK; }
    }
    double ra[PER], rb[PER];
    auto load = [&](long q) {
        const long b = b_first + q / kchunks;
        const int k0 = (int)(q % kchunks) * GK;
        const TA* A = (const TA*)g.A + b * g.sAb;
        const TB* B = (const TB*)g.B + b * g.sBb;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int gm = m0 + am[e], gk = k0 + ak[e];
            ra[e] = (gm < g.M && gk < g.K) ? (double)A[(long)gm * g.sAm + (long)gk * g.sAk] : 0.0;
            const int gn = n0 + bn[e], gk2 = k0 + bk[e];
            rb[e] = (gn < g.N && gk2 < g.K) ? (double)B[(long)gk2 * g.sBk + (long)gn * g.sBn] : 0.0;
        }
    };
    if (nchunks > 0) load(0);
    for (long q = 0; q < nchunks; ++q) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            As[ak[e]][am[e]] = ra[e];
            Bs[bk[e]][bn[e]] = rb[e];
        }
        __syncthreads();
        if (q + 1 < nchunks) load(q + 1);     // in flight while this chunk is multiplied
#pragma unroll 16
        for (int kk = 0; kk < GK; ++kk) {
            const double a0 = As[kk][ty], a1 = As[kk][ty + 16];
            const double b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
            acc[0][0] += a0 * b0; acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0; acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
            if (gm < g.M && gn < g.N) {
                TC* c = C + (long)gm * g.sCm + (long)gn * g.sCn;
                double v = g.alpha * acc[i][j];
                if (g.beta != 0.0) v += g.beta * (double)(*c);
                *c = (TC)v;
            }
        }
}

template <typename TA, typename TB, typename TC>
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s)
{
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return hipSuccess;
    long tiles = (long)((a.M + GT - 1) / GT) * ((a.N + GT - 1) / GT);
    unsigned gy = a.reduce_batch ? 1u : (unsigned)a.batch;
    const unsigned gz = a.nb > 1 ? (unsigned)a.nb : 1u;
    hipLaunchKernelGGL((k_gemm<TA, TB, TC>), dim3((unsigned)tiles, gy, gz), dim3(256), 0, s, a);
    return hipGetLastError();
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
