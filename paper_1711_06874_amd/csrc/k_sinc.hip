// Sinc-quadrature canonical (CP) tensor of a half-integer Matern covariance and the small pieces
// of its canonical-to-Tucker conversion (Sec. 3.4, with the Laplace-transform weights of Sec. 3.5).
//
// With c = sqrt(2 nu)/ell, the Matern value is a Laplace integral in r^2:
//   C(r) = sigma2 int_0^inf g(t) P(t) exp(-r^2 t) dt,  g(t) = c / (2 sqrt(pi)) t^(-3/2) exp(-c^2/(4t)),
// where P = 1, c^2/(2t) and c^4/(12 t^2) for nu = 1/2, 3/2, 5/2 (the polynomial factors of the
// closed forms act on exp(-c r) as derivatives in c).  The substitution t = (c^2/4) e^u and the
// sinc rule with step h = C0 log(M)/M at u_k = k h, k = -M..M, give the R = 2M + 1 term
// canonical tensor  A(x) ~ sum_k w_k prod_l exp(-t_k x_l^2),  w_k = sigma2 h g(t_k) P(t_k) t_k;
// its side matrices are Q_l[i][k] = w_k^(1/3) exp(-t_k x_{l,i}^2).
#include "tk_kernels.h"

namespace tk {

namespace {

__global__ void k_sinc_nodes(int M, double h, double c, int half, double sigma2, double* __restrict__ t,
                             double* __restrict__ w)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > 2 * M) return;
    const double u = h * (double)(k - M);
    const double tk = 0.25 * c * c * exp(u);
    // g(t_k) t_k = c / (2 sqrt(pi)) t_k^(-1/2) exp(-c^2 / (4 t_k)), and -c^2/(4 t_k) = -e^{-u}
    double g = c * 0.28209479177387814 / sqrt(tk) * exp(-exp(-u));
    if (half == 1) g *= c * c / (2.0 * tk);
    if (half == 2) g *= (c * c) * (c * c) / (12.0 * tk * tk);
    t[k] = tk;
    w[k] = sigma2 * h * g;
}

// Q_l[i][k] for the three axes (rows x0_l + i h_l): one thread per entry.
__global__ void __launch_bounds__(256) k_sinc_factors(GridAxes g, int R, const double* __restrict__ t,
                                                      const double* __restrict__ w, double* __restrict__ Q0,
                                                      double* __restrict__ Q1, double* __restrict__ Q2)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long n0 = (long)g.n[0] * R, n1 = (long)g.n[1] * R, n2 = (long)g.n[2] * R;
    int l;
    long f;
    if (e < n0) { l = 0; f = e; }
    else if (e < n0 + n1) { l = 1; f = e - n0; }
    else if (e < n0 + n1 + n2) { l = 2; f = e - n0 - n1; }
    else return;
    const int i = (int)(f / R), k = (int)(f - (long)i * R);
    const double x = g.x0[l] + (double)i * g.h[l];
    const double v = cbrt(w[k]) * exp(-t[k] * x * x);
    (l == 0 ? Q0 : (l == 1 ? Q1 : Q2))[f] = v;
}

__global__ void k_hadamard(const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ C, long n)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) C[e] = A[e] * B[e];
}

// KR[k][b r2 + c] = P1[b][k] P2[c][k]  (P_l: r_l x R row-major)
__global__ void k_khatri_rao(const double* __restrict__ P1, const double* __restrict__ P2, int R, int r1, int r2,
                             double* __restrict__ KR)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)R * r1 * r2;
    if (e >= tot) return;
    const int k = (int)(e / ((long)r1 * r2));
    const int bc = (int)(e - (long)k * r1 * r2);
    const int b = bc / r2, c = bc - b * r2;
    KR[e] = P1[(long)b * R + k] * P2[(long)c * R + k];
}

// out = sum_e A[e] B[e] C[e]  (one work-group, fixed summation order)
__global__ void __launch_bounds__(256) k_triple_sum(const double* __restrict__ A, const double* __restrict__ B,
                                                    const double* __restrict__ C, long n, double* __restrict__ out)
{
    __shared__ double red[4];
    double s = 0.0;
    for (long e = threadIdx.x; e < n; e += 256) s += A[e] * B[e] * C[e];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

unsigned blocks_for(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_sinc_nodes(int M, double h, double c, int half, double sigma2, double* t, double* w, hipStream_t s)
{
    if (M < 1 || half < 0 || half > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sinc_nodes, dim3(blocks_for(2 * M + 1)), dim3(256), 0, s, M, h, c, half, sigma2, t, w);
    return hipGetLastError();
}

hipError_t launch_sinc_factors(const GridAxes& g, int R, const double* t, const double* w, double* const Q[3],
                               hipStream_t s)
{
    const long tot = ((long)g.n[0] + g.n[1] + g.n[2]) * R;
    hipLaunchKernelGGL(k_sinc_factors, dim3(blocks_for(tot)), dim3(256), 0, s, g, R, t, w, Q[0], Q[1], Q[2]);
    return hipGetLastError();
}

hipError_t launch_hadamard(const double* A, const double* B, double* C, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_hadamard, dim3(blocks_for(n)), dim3(256), 0, s, A, B, C, n);
    return hipGetLastError();
}

hipError_t launch_khatri_rao(const double* P1, const double* P2, int R, int r1, int r2, double* KR, hipStream_t s)
{
    hipLaunchKernelGGL(k_khatri_rao, dim3(blocks_for((long)R * r1 * r2)), dim3(256), 0, s, P1, P2, R, r1, r2, KR);
    return hipGetLastError();
}

hipError_t launch_triple_sum(const double* A, const double* B, const double* C, long n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_triple_sum, dim3(1), dim3(256), 0, s, A, B, C, n, out);
    return hipGetLastError();
}

}  // namespace tk
