// a8: mode products with symmetric Toeplitz matrices for the Kronecker-format covariance
// matvec (Sec. 3.6 eq. (3.16)-(3.18); Sec. 4 eq. (4.1) with a general vector z).
//
// T(u)_{ij} = u[off + |i - j|] is never materialised: each MFMA operand that belongs to a
// Toeplitz factor is read from the generator u held in LDS at index off + |i - j|.
//
//   left : Out[s][g][i'][n] (+)= sum_{b < nb} sum_{i < K} u_{g,b}[off + |i' - i|] In[s][g][b][i][n]
//   right: Out[row][b][j']    = sum_{j < K} In[row][j] u_b[off + |j - j'|]
//
// Generators are addressed as gen[idx * gs_idx + col * gs_col] with col = g * gstride_g +
// b * gstride_b (left) or col = b (right).  Work-group tile: 64 x 64 outputs, 4 waves of
// 32 x 32 (2 x 2 MFMA 16x16x4 blocks); K is staged in chunks of 16 (double) / 32 (float).
// FP32 data run on mfma_f32_16x16x4f32, FP64 data on mfma_f64_16x16x4f64.
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr int TT = 64;

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef f32x4 acc_t;
    static constexpr int BK = 32;
    __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // D[i][j]: lane j + 16 (i/4), register i%4
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
    typedef f64x4 acc_t;
    static constexpr int BK = 16;
    __device__ static acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // D[i][j]: lane j + 16 (i%4), register i/4
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

}  // namespace

template <typename T>
__global__ void __launch_bounds__(256) k_toep_left(ToepLeftArgs a)
{
    constexpr int BK = Mfma<T>::BK;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* gen_s = reinterpret_cast<T*>(smem_raw);                  // glen entries
    T (*Bs)[TT + 1] = reinterpret_cast<T (*)[TT + 1]>(gen_s + a.glen_pad);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tiles_n = (a.N + TT - 1) / TT;
    const int i0 = (blockIdx.x / tiles_n) * TT, n0 = (blockIdx.x % tiles_n) * TT;
    const long s = blockIdx.y, g = blockIdx.z;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    typename Mfma<T>::acc_t acc[2][2];
    for (int x = 0; x < 2; ++x) for (int y = 0; y < 2; ++y) for (int v = 0; v < 4; ++v) acc[x][y][v] = 0;

    const T* In = (const T*)a.In + s * a.sIs + g * a.sIg;
    for (int b = 0; b < a.nb; ++b) {
        __syncthreads();
        const T* gen = (const T*)a.gen + (g * a.gstride_g + b * a.gstride_b) * a.gs_col;
        for (int e = tid; e < a.glen; e += 256) gen_s[e] = gen[(long)e * a.gs_idx];
        const T* Inb = In + b * a.sIb;
        for (int k0 = 0; k0 < a.K; k0 += BK) {
            __syncthreads();
            for (int e = tid; e < BK * TT; e += 256) {
                int kk = e / TT, nn = e % TT;
                int gi = k0 + kk, gn = n0 + nn;
                Bs[kk][nn] = (gi < a.K && gn < a.N) ? Inb[(long)gi * a.sIi + gn] : (T)0;
            }
            __syncthreads();
#pragma unroll 4
            for (int ks = 0; ks < BK; ks += 4) {
                int gi = k0 + ks + (lane >> 4);
                T av[2], bv[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    int ip = i0 + wm + 16 * x + (lane & 15);
                    int d = ip - gi;
                    d = d < 0 ? -d : d;
                    av[x] = (ip < a.M && gi < a.K) ? gen_s[a.off + d] : (T)0;
                }
#pragma unroll
                for (int y = 0; y < 2; ++y) bv[y] = Bs[ks + (lane >> 4)][wn + 16 * y + (lane & 15)];
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::mma(av[x], bv[y], acc[x][y]);
            }
        }
    }
    T* Out = (T*)a.Out + s * a.sOs + g * a.sOg;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int ip = i0 + wm + 16 * x + Mfma<T>::row(lane, v);
                int nn = n0 + wn + 16 * y + (lane & 15);
                if (ip < a.M && nn < a.N) {
                    T* o = Out + (long)ip * a.sOi + nn;
                    *o = a.accumulate ? (T)(*o + acc[x][y][v]) : (T)acc[x][y][v];
                }
            }
}

template <typename T>
__global__ void __launch_bounds__(256) k_toep_right(ToepRightArgs a)
{
    constexpr int BK = Mfma<T>::BK;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T (*As)[BK + 1] = reinterpret_cast<T (*)[BK + 1]>(smem_raw);
    T* gen_s = reinterpret_cast<T*>(smem_raw + sizeof(T) * TT * (BK + 1));   // span * glen entries
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long NC = (long)a.nb * a.m;                   // output columns (b, j')
    const int tiles_n = (int)((NC + TT - 1) / TT);
    const long r0 = (long)(blockIdx.x / tiles_n) * TT;
    const long c0 = (long)(blockIdx.x % tiles_n) * TT;
    const int b_lo = (int)(c0 / a.m);
    int b_hi = (int)((c0 + TT - 1) / a.m);
    if (b_hi > a.nb - 1) b_hi = a.nb - 1;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    for (int e = tid; e < (b_hi - b_lo + 1) * a.glen; e += 256) {
        int bb = b_lo + e / a.glen, idx = e % a.glen;
        gen_s[e] = ((const T*)a.gen)[(long)idx * a.gs_idx + (long)bb * a.gs_col];
    }
    // per-lane output columns of the two 16-wide blocks
    int jp[2], gb[2];
    bool cin[2];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        long c = c0 + wn + 16 * y + (lane & 15);
        cin[y] = c < NC;
        int b = cin[y] ? (int)(c / a.m) : b_lo;
        jp[y] = cin[y] ? (int)(c - (long)b * a.m) : 0;
        gb[y] = (b - b_lo) * a.glen;
    }
    typename Mfma<T>::acc_t acc[2][2];
    for (int x = 0; x < 2; ++x) for (int y = 0; y < 2; ++y) for (int v = 0; v < 4; ++v) acc[x][y][v] = 0;
    const T* In = (const T*)a.In;
    for (int k0 = 0; k0 < a.K; k0 += BK) {
        __syncthreads();
        for (int e = tid; e < TT * BK; e += 256) {
            int rr = e / BK, kk = e % BK;
            long gr = r0 + rr;
            int gk = k0 + kk;
            As[rr][kk] = (gr < a.R && gk < a.K) ? In[gr * a.ldi + gk] : (T)0;
        }
        __syncthreads();
#pragma unroll 4
        for (int ks = 0; ks < BK; ks += 4) {
            int j = k0 + ks + (lane >> 4);
            T av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = As[wm + 16 * x + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                int d = j - jp[y];
                d = d < 0 ? -d : d;
                bv[y] = (cin[y] && j < a.K) ? gen_s[gb[y] + a.off + d] : (T)0;
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::mma(av[x], bv[y], acc[x][y]);
        }
    }
    T* Out = (T*)a.Out;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                long rr = r0 + wm + 16 * x + Mfma<T>::row(lane, v);
                long c = c0 + wn + 16 * y + (lane & 15);
                if (rr < a.R && c < NC) Out[rr * a.ldo + c] = acc[x][y][v];
            }
}

template <typename T>
hipError_t launch_toep_left(const ToepLeftArgs& a, int nslab, int ngroup, hipStream_t s)
{
    if (a.M <= 0 || a.N <= 0 || nslab <= 0 || ngroup <= 0) return hipSuccess;
    long tiles = (long)((a.M + TT - 1) / TT) * ((a.N + TT - 1) / TT);
    size_t shm = sizeof(T) * ((size_t)a.glen_pad + (size_t)Mfma<T>::BK * (TT + 1));
    hipLaunchKernelGGL(k_toep_left<T>, dim3((unsigned)tiles, nslab, ngroup), dim3(256), shm, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_toep_right(const ToepRightArgs& a, hipStream_t s)
{
    if (a.R <= 0 || a.m <= 0 || a.nb <= 0) return hipSuccess;
    long NC = (long)a.nb * a.m;
    long tiles = ((a.R + TT - 1) / TT) * ((NC + TT - 1) / TT);
    int span = (TT + a.m - 1) / a.m + 1;
    if (span > a.nb) span = a.nb;
    size_t shm = sizeof(T) * ((size_t)TT * (Mfma<T>::BK + 1) + (size_t)span * a.glen);
    hipLaunchKernelGGL(k_toep_right<T>, dim3((unsigned)tiles), dim3(256), shm, s, a);
    return hipGetLastError();
}

template hipError_t launch_toep_left<float>(const ToepLeftArgs&, int, int, hipStream_t);
template hipError_t launch_toep_left<double>(const ToepLeftArgs&, int, int, hipStream_t);
template hipError_t launch_toep_right<float>(const ToepRightArgs&, hipStream_t);
template hipError_t launch_toep_right<double>(const ToepRightArgs&, hipStream_t);

hipError_t kron_set_attributes()
{
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_toep_left<float>, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_toep_left<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_toep_right<float>, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024)) != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_toep_right<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
}

}  // namespace tk
