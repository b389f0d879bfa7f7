// Device-side helpers shared by the gfx950 kernels of the Tucker engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// MFMA operand / result layouts used below (lane l of a 64-wide wave):
//  mfma_f32_32x32x2f32 : A[i][k] at lane i + 32k, B[k][j] at lane j + 32k,
//                        D[i][j] at lane j + 32((i/4)%2), register (i%4) + 4(i/8)
//  mfma_f32_16x16x4f32 : A[i][k] at lane i + 16k, B[k][j] at lane j + 16k,
//                        D[i][j] at lane j + 16(i/4), register i%4
//  mfma_f64_16x16x4f64 : A[i][k] at lane i + 16k, B[k][j] at lane j + 16k,
//                        D[i][j] at lane j + 16(i%4), register i/4
//  mfma_f32_32x32x16_bf16: A[i][k] at lane i + 32(k/8), element k%8 (same for B[k][j] with j),
//                        D as for 32x32x2
//  mfma_f32_16x16x32_bf16: A[i][k] at lane i + 16(k/8), element k%8, D as for 16x16x4 f32

// Batched launches: grid z runs over problems of equal shape whose device workspaces lie `bs`
// bytes apart; a kernel moves each of its workspace pointers by blockIdx.z * bs (null pointers
// stay null).  With one problem (grid z = 1) nothing moves.
template <typename T>
__device__ __forceinline__ T* bshift(T* p, long bs)
{
    return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)((long)blockIdx.z * bs)) : p;
}

// Covariance families (values match the public tk_family enum).
enum { FAM_MATERN = 0, FAM_SLATER = 1, FAM_GAUSS = 2 };

struct KernelParams {
    int family;
    int half;          // Matern: nu = half + 1/2 (0, 1, 2)
    double inv_len;    // Matern: sqrt(2 nu)/ell ; Slater/Gauss: 1/ell
    double sigma2;
    double alpha;
    double p;
};

// Covariance value at distance r, evaluated in double from the closed forms
//   Matern nu=1/2: e^{-s},  nu=3/2: (1+s)e^{-s},  nu=5/2: (1 + s + s^2/3)e^{-s},  s = sqrt(2nu) r/ell
//   Slater: exp(-alpha (r/ell)^p),  Gauss: exp(-(r/ell)^2)
__device__ __forceinline__ double cov_value(const KernelParams& kp, double r)
{
    double v;
    if (kp.family == FAM_MATERN) {
        double s = r * kp.inv_len;
        double poly = (kp.half == 0) ? 1.0 : (kp.half == 1) ? (1.0 + s) : (1.0 + s + s * s * (1.0 / 3.0));
        v = poly * exp(-s);
    } else if (kp.family == FAM_SLATER) {
        double t = r * kp.inv_len;
        double tp = (kp.p == 1.0) ? t : ((t == 0.0) ? 0.0 : pow(t, kp.p));
        v = exp(-kp.alpha * tp);
    } else {
        double t = r * kp.inv_len;
        v = exp(-(t * t));
    }
    return kp.sigma2 * v;
}

// e^{-s} for s >= 0 to about 2e-10 relative, for values that are rounded once to float:
// 2^u with u = -s log2(e) = k + f (k an integer, |f| <= 1/2), 2^f = e^{f ln 2} from its
// degree-8 Taylor polynomial (remainder below 0.35^9 / 9!), and 2^k applied exactly.
__device__ __forceinline__ double exp_neg_for_float(double s)
{
    if (s > 256.0) return 0.0;   // far below the float range
    const double u = -s * 1.4426950408889634;
    const double k = rint(u);
    const double f = (u - k) * 0.6931471805599453;
    double p = 1.0 / 40320.0;
    p = fma(p, f, 1.0 / 5040.0);
    p = fma(p, f, 1.0 / 720.0);
    p = fma(p, f, 1.0 / 120.0);
    p = fma(p, f, 1.0 / 24.0);
    p = fma(p, f, 1.0 / 6.0);
    p = fma(p, f, 0.5);
    p = fma(p, f, 1.0);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)k);
}

// cov_value at r = sqrt(r2) for a value rounded once to float: the same closed forms, with the
// radius from the hardware reciprocal square root refined by one Newton step (relative error
// ~1e-14) and exp_neg_for_float.
__device__ __forceinline__ double cov_value_for_float(const KernelParams& kp, double r2)
{
    double r = 0.0;
    if (r2 > 0.0) {
        double y = __builtin_amdgcn_rsq(r2);
        y = y * fma(-0.5 * r2 * y, y, 1.5);
        r = r2 * y;
    }
    double v;
    if (kp.family == FAM_MATERN) {
        double s = r * kp.inv_len;
        double poly = (kp.half == 0) ? 1.0 : (kp.half == 1) ? (1.0 + s) : (1.0 + s + s * s * (1.0 / 3.0));
        v = poly * exp_neg_for_float(s);
    } else if (kp.family == FAM_SLATER) {
        double t = r * kp.inv_len;
        double tp = (kp.p == 1.0) ? t : ((t == 0.0) ? 0.0 : pow(t, kp.p));
        v = exp_neg_for_float(kp.alpha * tp);
    } else {
        double t = r * kp.inv_len;
        v = exp_neg_for_float(t * t);
    }
    return kp.sigma2 * v;
}

// Wave-level sum (64 lanes) of a double.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_sumf(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Split a float into bf16 high and low parts: x ~ hi + lo with |x - hi - lo| <~ 2^-16 |x|.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}
