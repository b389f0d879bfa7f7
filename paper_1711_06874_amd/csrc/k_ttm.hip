// a5/a6/a7: the contractions that stream the full tensor A (HOOI single-hole products, the
// core, and the reconstruction error of Sec. 3.7 eq. (3.26)).
//
//   ttm_last : T[row, c] = sum_k A[row, k] U[k, c]      A viewed as (n0 n1) x n2   (A x_3 U^T)
//   ttm_first: S[a, col] = sum_i U[i, a] A[i, col]      A viewed as n0 x (n1 n2)   (A x_1 U^T)
//   recon_diff: sum over A of A^2 and (A - H U^T)^2,    H = G x_1 U1 x_2 U2 as (n0 n1) x r
//
// All three read A exactly once with coalesced loads.  The TTMs stage 64 x 64 float tiles in
// LDS (the next tile and U chunk are loaded into registers while the current one is multiplied)
// and contract them on FP32 MFMA (16x16x4) with FP32 accumulation; the error norm
// reconstructs A on FP64 MFMA.  The rank dimension r is covered by NB = ceil(r/16) blocks of
// 16.  The error sums are accumulated per thread in FP64 and reduced in a fixed order (per
// work-group partials, then one ordered pass).
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr int TR = 64;       // rows (or columns) of A per work-group
constexpr int BK = 64;       // contraction chunk
constexpr int LDA = BK + 4;  // LDS pitch: lanes of one MFMA operand read hit distinct banks

// A TR x BK float tile of a row-major matrix (row pitch ld), four float4 per thread: loaded into
// registers (tile_load, rows >= nrows or columns >= ncols read as zero) while the previous tile
// is multiplied, then written to S[TR][LDA] (tile_store).
constexpr int TQ = (TR * BK / 4) / 256;      // float4 per thread

__device__ __forceinline__ void tile_load(float4 (&v)[TQ], const float* __restrict__ X, long ld, long row0,
                                          long nrows, long col0, long ncols, int tid)
{
    const bool vec = ((ld & 3) == 0) && ((col0 & 3) == 0);
#pragma unroll
    for (int e = 0; e < TQ; ++e) {
        int q = tid + 256 * e;           // float4 index within the tile
        int r = q / (BK / 4), c4 = (q % (BK / 4)) * 4;
        long gr = row0 + r, gc = col0 + c4;
        v[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gr < nrows) {
            const float* p = X + gr * ld + gc;
            if (vec && gc + 3 < ncols) v[e] = *reinterpret_cast<const float4*>(p);
            else {
                if (gc + 0 < ncols) v[e].x = p[0];
                if (gc + 1 < ncols) v[e].y = p[1];
                if (gc + 2 < ncols) v[e].z = p[2];
                if (gc + 3 < ncols) v[e].w = p[3];
            }
        }
    }
}

__device__ __forceinline__ void tile_store(float (*S)[LDA], const float4 (&v)[TQ], int tid)
{
#pragma unroll
    for (int e = 0; e < TQ; ++e) {
        int q = tid + 256 * e;
        int r = q / (BK / 4), c4 = (q % (BK / 4)) * 4;
        *reinterpret_cast<float4*>(&S[r][c4]) = v[e];
    }
}

// The BK x NB*16 chunk of U (n x r row-major) from row k0, zero beyond n and r: UQ values per
// thread, loaded with the A tile and stored beside it.
template <int NB>
struct UChunk {
    static constexpr int UQ = (BK * NB * 16 + 255) / 256;
    float v[UQ];
    __device__ __forceinline__ void load(const float* __restrict__ U, int k0, int n, int r, int tid)
    {
#pragma unroll
        for (int i = 0; i < UQ; ++i) {
            const int e = tid + 256 * i;
            const int kk = e / (NB * 16), j = e % (NB * 16);
            v[i] = (e < BK * NB * 16 && k0 + kk < n && j < r) ? U[(long)(k0 + kk) * r + j] : 0.f;
        }
    }
    __device__ __forceinline__ void store(float (*Us)[NB * 16], int tid) const
    {
#pragma unroll
        for (int i = 0; i < UQ; ++i) {
            const int e = tid + 256 * i;
            if (e < BK * NB * 16) Us[e / (NB * 16)][e % (NB * 16)] = v[i];
        }
    }
};

// T = A x_3 U^T.  Work-group: 64 rows of A (4 waves x 16 rows); U chunk in LDS.
template <int NB>
__global__ void __launch_bounds__(256) k_ttm_last(const float* __restrict__ A, long rows, int n2,
                                                  const float* __restrict__ U, int r, float* __restrict__ T,
                                                  long bs)
{
    A = bshift(A, bs);
    U = bshift(U, bs);
    T = bshift(T, bs);
    __shared__ __attribute__((aligned(16))) float As[TR][LDA];
    __shared__ float Us[BK][NB * 16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long row0 = (long)blockIdx.x * TR;
    f32x4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float4 tv[TQ];
    UChunk<NB> uc;
    tile_load(tv, A, n2, row0, rows, 0, n2, tid);
    uc.load(U, 0, n2, r, tid);
    for (int k0 = 0; k0 < n2; k0 += BK) {
        tile_store(As, tv, tid);
        uc.store(Us, tid);
        __syncthreads();
        if (k0 + BK < n2) {            // the next chunk is in flight while this one is multiplied
            tile_load(tv, A, n2, row0, rows, k0 + BK, n2, tid);
            uc.load(U, k0 + BK, n2, r, tid);
        }
#pragma unroll 4
        for (int ks = 0; ks < BK; ks += 4) {
            float a = As[16 * w + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float bb = Us[ks + (lane >> 4)][16 * b + (lane & 15)];
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, acc[b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            long row = row0 + 16 * w + 4 * (lane >> 4) + v;
            int c = 16 * b + (lane & 15);
            if (row < rows && c < r) T[row * r + c] = acc[b][v];
        }
}

// S = A x_1 U^T.  Work-group: 64 columns of A (4 waves x 16 columns), all n0 rows.
template <int NB>
__global__ void __launch_bounds__(256) k_ttm_first(const float* __restrict__ A, int n0, long cols,
                                                   const float* __restrict__ U, int r, float* __restrict__ S,
                                                   long bs)
{
    A = bshift(A, bs);
    U = bshift(U, bs);
    S = bshift(S, bs);
    __shared__ __attribute__((aligned(16))) float As[TR][LDA];   // [k = i0][col]
    __shared__ float Us[BK][NB * 16];                            // [k][a]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long col0 = (long)blockIdx.x * TR;
    f32x4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float4 tv[TQ];
    UChunk<NB> uc;
    tile_load(tv, A, cols, 0, n0, col0, cols, tid);
    uc.load(U, 0, n0, r, tid);
    for (int k0 = 0; k0 < n0; k0 += BK) {
        tile_store(As, tv, tid);
        uc.store(Us, tid);
        __syncthreads();
        if (k0 + BK < n0) {            // the next chunk is in flight while this one is multiplied
            tile_load(tv, A, cols, k0 + BK, n0, col0, cols, tid);
            uc.load(U, k0 + BK, n0, r, tid);
        }
#pragma unroll 4
        for (int ks = 0; ks < BK; ks += 4) {
            // B operand: A[k][col], k = ks + lane/16, col = 16w + lane%16
            float bb = As[ks + (lane >> 4)][16 * w + (lane & 15)];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float a = Us[ks + (lane >> 4)][16 * b + (lane & 15)];   // A operand: U^T[a][k]
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, acc[b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int a = 16 * b + 4 * (lane >> 4) + v;
            long col = col0 + 16 * w + (lane & 15);
            if (a < r && col < cols) S[(long)a * cols + col] = acc[b][v];
        }
}

// Partial sums of A^2 and (A - H U3^T)^2 for 64 rows of A per work-group, in FP64: H and U3
// are double and the reconstruction runs on mfma_f64_16x16x4 (D[i][j] at lane j + 16 (i%4),
// register i/4), so the measured error has no FP32 arithmetic floor.
// H: rows x r (ld r), U3: n2 x r (ld r); the contraction runs over r rounded up to 4.
// Wave w reconstructs rows 16w..16w+15 of the tile: its H fragments stay in registers for the
// whole work-group, the U3^T chunk of 64 columns is staged in LDS, and the A values of the
// next chunk are loaded into registers while the current chunk is multiplied.
template <int NB>
__global__ void __launch_bounds__(256) k_recon_diff(const float* __restrict__ A, long rows, int n2,
                                                    const double* __restrict__ H, const double* __restrict__ U3,
                                                    int r, double* __restrict__ partials, long bs)
{
    A = bshift(A, bs);
    H = bshift(H, bs);
    U3 = bshift(U3, bs);
    partials = bshift(partials, bs);
    constexpr int KC = NB * 16;                // contraction capacity (zero beyond r)
    constexpr int KS = KC / 4;                 // MFMA k-steps at most
    __shared__ double Ut[KC][TR + 1];          // [c][k] for a 64-column chunk of U3^T
    __shared__ double red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long row0 = (long)blockIdx.x * TR;
    const int ks_n = ((r + 3) & ~3) / 4;
    // A operand (H): row 16w + lane%16, contraction index 4 ks + lane/16
    double af[KS];
    {
        const long row = row0 + 16 * w + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int c = 4 * ks + (lane >> 4);
            af[ks] = (row < rows && c < r) ? H[row * r + c] : 0.0;
        }
    }
    // this lane's A values: rows 16w + 4v + lane/16, columns 16cb + lane%16 of the chunk
    float xa[16];
    auto load_x = [&](int k0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long row = row0 + 16 * w + 4 * v + (lane >> 4);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int col = k0 + 16 * cb + (lane & 15);
                xa[v * 4 + cb] = (row < rows && col < n2) ? A[row * n2 + col] : 0.f;
            }
        }
    };
    double d2 = 0.0, a2 = 0.0;
    load_x(0);
    for (int k0 = 0; k0 < n2; k0 += TR) {
        __syncthreads();
        for (int e = tid; e < TR * KC; e += 256) {
            const int kk = e / KC, c = e % KC;
            Ut[c][kk] = (k0 + kk < n2 && c < r) ? U3[(long)(k0 + kk) * r + c] : 0.0;
        }
        __syncthreads();
        float xc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) xc[q] = xa[q];
        if (k0 + TR < n2) load_x(k0 + TR);     // in flight while this chunk is multiplied
#pragma unroll
        for (int cb = 0; cb < TR / 16; ++cb) {
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks < ks_n) {
                    const double b = Ut[4 * ks + (lane >> 4)][16 * cb + (lane & 15)];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], b, acc, 0, 0, 0);
                }
            }
            const int col = k0 + 16 * cb + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long row = row0 + 16 * w + 4 * v + (lane >> 4);
                if (row < rows && col < n2) {
                    const double x = (double)xc[v * 4 + cb];
                    const double d = x - acc[v];
                    d2 += d * d;
                    a2 += x * x;
                }
            }
        }
    }
    d2 = wave_sum(d2);
    a2 = wave_sum(a2);
    if (lane == 0) { red[0][w] = d2; red[1][w] = a2; }
    __syncthreads();
    if (tid == 0) {   // (||A||^2, ||A - A_r||^2) of this work-group
        partials[2 * blockIdx.x + 0] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        partials[2 * blockIdx.x + 1] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    }
}

// Generic (any type) partial sums of X^2 and (X - Y)^2.
template <typename T>
__global__ void __launch_bounds__(256) k_diff_norm(const T* __restrict__ X, const T* __restrict__ Y, long n,
                                                   double* __restrict__ partials, long bs)
{
    X = bshift(X, bs);
    Y = bshift(Y, bs);
    partials = bshift(partials, bs);
    __shared__ double red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double d2 = 0.0, a2 = 0.0;
    long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + tid; i < n; i += stride) {
        double x = (double)X[i], d = x - (double)Y[i];
        d2 += d * d;
        a2 += x * x;
    }
    d2 = wave_sum(d2);
    a2 = wave_sum(a2);
    if (lane == 0) { red[0][w] = d2; red[1][w] = a2; }
    __syncthreads();
    if (tid == 0) {   // (||A||^2, ||A - A_r||^2) of this work-group
        partials[2 * blockIdx.x + 0] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        partials[2 * blockIdx.x + 1] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    }
}

}  // namespace

hipError_t launch_ttm_last_f32(const float* A, long rows, int n2, const float* U, int r, float* T, hipStream_t s,
                               Bat bt)
{
    dim3 grid((unsigned)((rows + TR - 1) / TR), 1, bt.nb);
    if (r <= 16) hipLaunchKernelGGL(k_ttm_last<1>, grid, dim3(256), 0, s, A, rows, n2, U, r, T, bt.bs);
    else if (r <= 32) hipLaunchKernelGGL(k_ttm_last<2>, grid, dim3(256), 0, s, A, rows, n2, U, r, T, bt.bs);
    else hipLaunchKernelGGL(k_ttm_last<3>, grid, dim3(256), 0, s, A, rows, n2, U, r, T, bt.bs);
    return hipGetLastError();
}

hipError_t launch_ttm_first_f32(const float* A, int n0, long cols, const float* U, int r, float* S, hipStream_t s,
                                Bat bt)
{
    dim3 grid((unsigned)((cols + TR - 1) / TR), 1, bt.nb);
    if (r <= 16) hipLaunchKernelGGL(k_ttm_first<1>, grid, dim3(256), 0, s, A, n0, cols, U, r, S, bt.bs);
    else if (r <= 32) hipLaunchKernelGGL(k_ttm_first<2>, grid, dim3(256), 0, s, A, n0, cols, U, r, S, bt.bs);
    else hipLaunchKernelGGL(k_ttm_first<3>, grid, dim3(256), 0, s, A, n0, cols, U, r, S, bt.bs);
    return hipGetLastError();
}

int recon_diff_parts(long rows) { return (int)((rows + TR - 1) / TR); }

hipError_t launch_recon_diff_f32(const float* A, long rows, int n2, const double* H, const double* U3, int r,
                                 double* partials, hipStream_t s, Bat bt)
{
    dim3 grid((unsigned)recon_diff_parts(rows), 1, bt.nb);
    if (r <= 16)
        hipLaunchKernelGGL(k_recon_diff<1>, grid, dim3(256), 0, s, A, rows, n2, H, U3, r, partials, bt.bs);
    else if (r <= 32)
        hipLaunchKernelGGL(k_recon_diff<2>, grid, dim3(256), 0, s, A, rows, n2, H, U3, r, partials, bt.bs);
    else
        hipLaunchKernelGGL(k_recon_diff<3>, grid, dim3(256), 0, s, A, rows, n2, H, U3, r, partials, bt.bs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diff_norm(const T* X, const T* Y, long n, double* partials, int nparts, hipStream_t s, Bat bt)
{
    hipLaunchKernelGGL(k_diff_norm<T>, dim3(nparts, 1, bt.nb), dim3(256), 0, s, X, Y, n, partials, bt.bs);
    return hipGetLastError();
}
template hipError_t launch_diff_norm<float>(const float*, const float*, long, double*, int, hipStream_t, Bat);
template hipError_t launch_diff_norm<double>(const double*, const double*, long, double*, int, hipStream_t, Bat);

}  // namespace tk
