// Seeded N(0,1) input vectors drawn on the device: the counter-based generator Philox4x32-10
// (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as
// 1, 2, 3", SC'11) keyed by (seed, stream), then the Box-Muller transform in FP64, rounded once
// to float.  Counter block c = (c mod 2^32, c / 2^32, 0, 0) gives four 32-bit words x0..x3;
// u_a = ((x1 << 32 | x0) >> 11) 2^-53 and u_b = ((x3 << 32 | x2) >> 11) 2^-53 lie in [0, 1);
// rho = sqrt(-2 log(1 - u_a)), phi = 2 pi u_b, and the block's normals are element 2c
// (rho cos phi) and element 2c + 1 (rho sin phi).
#include "tk_kernels.h"

namespace tk {

namespace {

// One Philox4x32 round with multipliers 0xD2511F53, 0xCD9E8D57; the key moves by the Weyl
// constants 0x9E3779B9, 0xBB67AE85 between rounds.
__device__ __forceinline__ uint4 philox_block(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__global__ void __launch_bounds__(256) k_philox_words(uint32_t k0, uint32_t k1, unsigned long long c0, long nblocks,
                                                      uint4* __restrict__ out)
{
    const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    const unsigned long long c = c0 + (unsigned long long)b;
    out[b] = philox_block(make_uint4((uint32_t)c, (uint32_t)(c >> 32), 0u, 0u), k0, k1);
}

__global__ void __launch_bounds__(256) k_philox_normal(uint32_t k0, uint32_t k1, long count, float* __restrict__ z)
{
    const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * b >= count) return;
    const unsigned long long c = (unsigned long long)b;
    const uint4 x = philox_block(make_uint4((uint32_t)c, (uint32_t)(c >> 32), 0u, 0u), k0, k1);
    const double ua = (double)((((unsigned long long)x.y << 32) | x.x) >> 11) * 0x1.0p-53;
    const double ub = (double)((((unsigned long long)x.w << 32) | x.z) >> 11) * 0x1.0p-53;
    const double rho = sqrt(-2.0 * log(1.0 - ua));
    const double phi = 6.283185307179586 * ub;
    z[2 * b] = (float)(rho * cos(phi));
    if (2 * b + 1 < count) z[2 * b + 1] = (float)(rho * sin(phi));
}

}  // namespace

hipError_t launch_philox_words(uint32_t k0, uint32_t k1, unsigned long long c0, long nblocks, uint32_t* out,
                               hipStream_t s)
{
    if (nblocks < 0) return hipErrorInvalidValue;
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_words, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0, s, k0, k1, c0, nblocks,
                       reinterpret_cast<uint4*>(out));
    return hipGetLastError();
}

hipError_t launch_philox_normal(uint32_t k0, uint32_t k1, long count, float* z, hipStream_t s)
{
    if (count < 0) return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    const long blocks = (count + 1) / 2;
    hipLaunchKernelGGL(k_philox_normal, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s, k0, k1, count, z);
    return hipGetLastError();
}

}  // namespace tk
