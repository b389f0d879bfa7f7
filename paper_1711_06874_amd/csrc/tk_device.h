// Device-side helpers shared by the gfx950 kernels of the Tucker engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

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
// The offset is applied as byte pointer arithmetic (not through an integer), so the compiler
// still sees a global-memory pointer and emits global loads and stores: a flat access would
// also count against the LDS wait counter and make every LDS wait drain the loads in flight.
template <typename T>
__device__ __forceinline__ T* bshift(T* p, long bs)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (long)blockIdx.z * bs) : p;
}

// Covariance families (values match the public tk_family enum).
enum { FAM_MATERN = 0, FAM_SLATER = 1, FAM_GAUSS = 2, FAM_SPECTRAL = 3 };

struct KernelParams {
    int family;
    int half;          // Matern: nu = half + 1/2 (0, 1, 2); -1: any other order (Bessel route)
    double inv_len;    // Matern: sqrt(2 nu)/ell ; Slater/Gauss: 1/ell
    double sigma2;
    double alpha;      // Slater rate; spectral density: alpha^2
    double p;
    double nu;         // Matern (general order), spectral density
    double lpref;      // log of the constant: Matern 2^{1-nu}/Gamma(nu); spectral
                       // Gamma(nu+3/2) alpha^{2nu} / (pi^{3/2} Gamma(nu))
    double axs[3];     // per-axis coordinate scale sqrt(a_k) of the anisotropic metric (1: none)
};

// 1/Gamma(1+z) = sum_j c_{j+1} z^j with the coefficients c_k of 1/Gamma(z) = sum_k c_k z^k
// (Abramowitz & Stegun 6.1.34), split into its even part E(z^2) and odd part z O(z^2):
//   rgam_even(m2) = c1 + c3 m2 + c5 m2^2 + ...,  rgam_odd(m2) = c2 + c4 m2 + c6 m2^2 + ...
// Used for |z| <= 1/2, where the 26-term series is exact to double rounding.
__device__ __forceinline__ double rgam_even(double m2)
{
    const double c[13] = {1.0, -0.6558780715202538, 0.1665386113822915, -0.0096219715278770,
                          -0.0011651675918591, 0.0001280502823882, -0.0000012504934821, -0.0000002056338417,
                          0.0000000050020075, 0.0000000001043427, -0.0000000000036968, -0.0000000000000206,
                          0.0000000000000014};
    double v = c[12];
    for (int j = 11; j >= 0; --j) v = fma(v, m2, c[j]);
    return v;
}
__device__ __forceinline__ double rgam_odd(double m2)
{
    const double c[13] = {0.5772156649015329, -0.0420026350340952, -0.0421977345555443, 0.0072189432466630,
                          -0.0002152416741149, -0.0000201348547807, 0.0000011330272320, 0.0000000061160950,
                          -0.0000000011812746, 0.0000000000077823, 0.0000000000005100, -0.0000000000000054,
                          0.0000000000000001};
    double v = c[12];
    for (int j = 11; j >= 0; --j) v = fma(v, m2, c[j]);
    return v;
}

// Modified Bessel function of the second kind K_nu(x), nu >= 0, x > 0, in FP64.
// nu = N + mu with N = round(nu), |mu| <= 1/2; K_mu and K_{mu+1} come from
//  - x <= 2: Temme's series (N. M. Temme, J. Comput. Phys. 19 (1975) 324): with
//    G1 = (1/Gamma(1-mu) - 1/Gamma(1+mu))/(2 mu), G2 = (1/Gamma(1-mu) + 1/Gamma(1+mu))/2,
//    sigma = mu ln(2/x):  f0 = mu pi/sin(mu pi) (G1 cosh sigma + G2 ln(2/x) sinh(sigma)/sigma),
//    p0 = (x/2)^-mu Gamma(1+mu)/2, q0 = (x/2)^mu Gamma(1-mu)/2, and for k >= 1
//    f_k = (k f_{k-1} + p_{k-1} + q_{k-1})/(k^2 - mu^2), p_k = p_{k-1}/(k - mu),
//    q_k = q_{k-1}/(k + mu), c_k = (x^2/4)^k/k!:  K_mu = sum c_k f_k,
//    K_{mu+1} = (2/x) sum c_k (p_k - k f_k);
//  - x > 2: Steed's evaluation of the continued fraction for K_{mu+1}/K_mu with the sum that
//    normalises K_mu (I. J. Thompson, A. R. Barnett, J. Comput. Phys. 64 (1986) 490);
// then the upward recurrence K_{m+1} = K_{m-1} + (2m/x) K_m, which is stable for K.
__device__ inline double bessel_k(double nu, double x)
{
    const int N = (int)floor(nu + 0.5);
    const double mu = nu - N, mu2 = mu * mu;
    double k0, k1;   // K_mu, K_{mu+1}
    if (x <= 2.0) {
        const double lx = log(2.0 / x);
        const double g1 = -rgam_odd(mu2);            // G1
        const double g2 = rgam_even(mu2);            // G2
        const double rgp = g2 - mu * g1;             // 1/Gamma(1+mu)
        const double rgm = g2 + mu * g1;             // 1/Gamma(1-mu)
        const double sg = mu * lx;
        const double pm = M_PI * mu;
        const double fpi = (fabs(pm) < 1e-8) ? 1.0 + pm * pm / 6.0 : pm / sin(pm);
        const double shs = (fabs(sg) < 1e-8) ? 1.0 + sg * sg / 6.0 : sinh(sg) / sg;
        const double es = exp(sg);
        double f = fpi * (g1 * cosh(sg) + g2 * lx * shs);
        double pk = 0.5 * es / rgp;
        double qk = 0.5 / (es * rgm);
        double ck = 1.0;
        const double d = 0.25 * x * x;
        double s0 = f, s1 = pk;
        for (int k = 1; k < 500; ++k) {
            const double kk = (double)k;
            f = (kk * f + pk + qk) / (kk * kk - mu2);
            ck *= d / kk;
            pk /= (kk - mu);
            qk /= (kk + mu);
            const double t0 = ck * f, t1 = ck * (pk - kk * f);
            s0 += t0;
            s1 += t1;
            if (fabs(t0) < 1e-17 * fabs(s0) && fabs(t1) < 1e-17 * fabs(s1)) break;
        }
        k0 = s0;
        k1 = s1 * (2.0 / x);
    } else {
        // continued fraction, evaluated forward (Steed): b_i = 2(x + i), a_i = -(mu^2 - (i-1/2)^2)
        // ... and the series S = sum of q_i times the fraction's increments; K_mu = sqrt(pi/2x) e^-x / S
        const double a1 = 0.25 - mu2;
        double b = 2.0 * (1.0 + x);
        double dd = 1.0 / b;
        double h = dd, dh = dd;
        double qm = 0.0, qc = 1.0;      // q_{i-1}, q_i of the three-term recurrence
        double cc = a1, qs = a1, a = -a1;
        double S = 1.0 + qs * dh;
        for (int i = 1; i < 2000; ++i) {
            a -= 2.0 * i;
            cc = -a * cc / (i + 1.0);
            const double qn = (qm - b * qc) / a;
            qm = qc;
            qc = qn;
            qs += cc * qn;
            b += 2.0;
            dd = 1.0 / (b + a * dd);
            dh = (b * dd - 1.0) * dh;
            h += dh;
            const double dS = qs * dh;
            S += dS;
            if (fabs(dS) < 1e-17 * fabs(S)) break;
        }
        h *= a1;
        k0 = sqrt(M_PI / (2.0 * x)) * exp(-x) / S;
        k1 = k0 * (mu + x + 0.5 - h) / x;
    }
    for (int k = 1; k <= N; ++k) {
        const double t = k0 + (2.0 * (mu + k) / x) * k1;
        k0 = k1;
        k1 = t;
    }
    return k0;
}

// Matern value at s = sqrt(2 nu) r / ell for an order without a closed form:
// 2^{1-nu}/Gamma(nu) s^nu K_nu(s) (Sec. 2.2 eq. (2.3)), the constant passed in log form.
__device__ inline double matern_general(const KernelParams& kp, double s)
{
    if (s == 0.0) return 1.0;
    if (s > 740.0) return 0.0;
    return exp(kp.lpref + kp.nu * log(s)) * bessel_k(kp.nu, s);
}

// Matern spectral density at rho (Diagram 1 of Sec. 2.2; eq. (3.28)):
// C (alpha^2 + rho^2)^{-(nu + 3/2)}, the log constant and alpha^2 passed in.
__device__ inline double spectral_value(const KernelParams& kp, double rho)
{
    return exp(kp.lpref - (kp.nu + 1.5) * log(kp.alpha + rho * rho));
}

// Covariance value at distance r, evaluated in double from the closed forms
//   Matern nu=1/2: e^{-s},  nu=3/2: (1+s)e^{-s},  nu=5/2: (1 + s + s^2/3)e^{-s},  s = sqrt(2nu) r/ell
//   (other orders: the Bessel route above),
//   Slater: exp(-alpha (r/ell)^p),  Gauss: exp(-(r/ell)^2),  spectral density: as above
__device__ __forceinline__ double cov_value(const KernelParams& kp, double r)
{
    double v;
    if (kp.family == FAM_MATERN && kp.half < 0) {
        v = matern_general(kp, r * kp.inv_len);
    } else if (kp.family == FAM_SPECTRAL) {
        v = spectral_value(kp, r);
    } else if (kp.family == FAM_MATERN) {
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
    if ((kp.family == FAM_MATERN && kp.half < 0) || kp.family == FAM_SPECTRAL) {
        v = (kp.family == FAM_SPECTRAL) ? spectral_value(kp, r) : matern_general(kp, r * kp.inv_len);
    } else if (kp.family == FAM_MATERN) {
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
