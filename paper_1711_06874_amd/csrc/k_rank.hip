// Small single-work-group kernels around the compression: the eps rank rule, compaction of
// truncated factors / cores, and the covariance trace.
#include "tk_kernels.h"

namespace tk {

// Rank rule for problem blockIdx.x: lam holds the `len` leading eigenvalues (descending) of a
// matrix whose eigenvalues sum to total[blockIdx.x * sTotal] (or to the sum of lam when
// total == nullptr).  rank = smallest r >= 1 with total - sum_{i<r} lam_i <= budget, capped at
// `len`; budget = (eps2 * a2 - d2) / 3 with a2 = scal[0], d2 = scal[1] (d2 optional).
// ok[blockIdx.x] = 1 if the rule was met within len, else 0.
__global__ void k_rank_rule(const double* __restrict__ lam, long sLam, int len, const double* __restrict__ total,
                            long sTotal, const double* __restrict__ scal, int has_d2, double eps2,
                            int* __restrict__ ranks, int* __restrict__ ok, long bs)
{
    if (threadIdx.x != 0) return;
    lam = bshift(lam, bs);
    total = bshift(total, bs);
    scal = bshift(scal, bs);
    ranks = bshift(ranks, bs);
    ok = bshift(ok, bs);
    const double* l = lam + blockIdx.x * sLam;
    double tot;
    if (total) tot = total[blockIdx.x * sTotal];
    else { tot = 0.0; for (int i = len - 1; i >= 0; --i) tot += fmax(l[i], 0.0); }
    double budget = (eps2 * scal[0] - (has_d2 ? scal[1] : 0.0)) / 3.0;
    int r = len, met = 0;
    double head = 0.0;
    for (int c = 1; c <= len; ++c) {
        head += fmax(l[c - 1], 0.0);
        if (tot - head <= budget) { r = c; met = 1; break; }
    }
    ranks[blockIdx.x] = r;
    ok[blockIdx.x] = met;
}

// Copy the leading d0 x d1 x d2 block of a D0 x D1 x D2 array (C-order) to a dense array.
template <typename TI, typename TO>
__global__ void k_copy_block(const TI* __restrict__ X, int D1, int D2, TO* __restrict__ Y, int d0, int d1, int d2)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long tot = (long)d0 * d1 * d2;
    if (e >= tot) return;
    int a = (int)(e / ((long)d1 * d2)), b = (int)((e / d2) % d1), c = (int)(e % d2);
    Y[e] = (TO)X[((long)a * D1 + b) * D2 + c];
}

template <typename TI, typename TO>
hipError_t launch_copy_block(const TI* X, int D1, int D2, TO* Y, int d0, int d1, int d2, hipStream_t s)
{
    long tot = (long)d0 * d1 * d2;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy_block<TI, TO>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, D1, D2, Y,
                       d0, d1, d2);
    return hipGetLastError();
}
template hipError_t launch_copy_block<double, double>(const double*, int, int, double*, int, int, int, hipStream_t);
template hipError_t launch_copy_block<double, float>(const double*, int, int, float*, int, int, int, hipStream_t);

__global__ void __launch_bounds__(256) k_extract_results(ExtractArgs a)
{
    const int b = blockIdx.z;
    const ResultDst& d = a.dst[b];
    const long e0 = (long)a.n[0] * d.r[0], e1 = e0 + (long)a.n[1] * d.r[1], e2 = e1 + (long)a.n[2] * d.r[2];
    const long tot = e2 + (long)d.r[0] * d.r[1] * d.r[2];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        if (e < e2) {
            const int k = (e < e0) ? 0 : (e < e1 ? 1 : 2);
            const long f = e - (k == 0 ? 0 : (k == 1 ? e0 : e1));
            const int r = d.r[k];
            const long i = f / r;
            const int c = (int)(f - i * r);
            const double v = bshift(a.Usrc[k], a.bs)[i * a.ld[k] + c];      // problem b = blockIdx.z
            d.U[k][f] = v;
            d.U32[k][f] = (float)v;
        } else {
            const long f = e - e2;
            const int d12 = d.r[1] * d.r[2];
            const int x = (int)(f / d12), rem = (int)(f - (long)x * d12);
            const int y = rem / d.r[2], z = rem - y * d.r[2];
            const double v = bshift(a.core_src, a.bs)[((long)x * a.Rc[1] + y) * a.Rc[2] + z];
            d.core[f] = v;
            d.core32[f] = (float)v;
        }
    }
}

hipError_t launch_extract_results(const ExtractArgs& a, hipStream_t s)
{
    if (a.nb < 1 || a.nb > BATCH_MAX) return hipErrorInvalidValue;
    long most = 0;
    for (int b = 0; b < a.nb; ++b) {
        const ResultDst& d = a.dst[b];
        long tot = (long)d.r[0] * d.r[1] * d.r[2];
        for (int k = 0; k < 3; ++k) tot += (long)a.n[k] * d.r[k];
        most = tot > most ? tot : most;
    }
    if (most <= 0) return hipSuccess;
    long blocks = (most + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_extract_results, dim3((unsigned)blocks, 1, a.nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rank_rule(const double* lam, long sLam, int len, int count, const double* total, long sTotal,
                            const double* scal, int has_d2, double eps2, int* ranks, int* ok, hipStream_t s, Bat bt)
{
    hipLaunchKernelGGL(k_rank_rule, dim3(count, 1, bt.nb), dim3(64), 0, s, lam, sLam, len, total, sTotal, scal,
                       has_d2, eps2, ranks, ok, bt.bs);
    return hipGetLastError();
}

// trace of the Kronecker-Toeplitz covariance:
//   out = m0 m1 m2 * sum_abc G[a][b][c] U1[off0][a] U2[off1][b] U3[off2][c]
__global__ void __launch_bounds__(256) k_cov_trace(const double* __restrict__ G, int r0, int r1, int r2,
                                                   const double* __restrict__ u0, const double* __restrict__ u1,
                                                   const double* __restrict__ u2, double scale,
                                                   double* __restrict__ out)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int e = threadIdx.x; e < r0 * r1 * r2; e += 256) {
        int a = e / (r1 * r2), b = (e / r2) % r1, c = e % r2;
        s += G[e] * u0[a] * u1[b] * u2[c];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = scale * ((red[0] + red[1]) + (red[2] + red[3]));
}

hipError_t launch_cov_trace(const double* G, int r0, int r1, int r2, const double* u0, const double* u1,
                            const double* u2, double scale, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_cov_trace, dim3(1), dim3(256), 0, s, G, r0, r1, r2, u0, u1, u2, scale, out);
    return hipGetLastError();
}

// E^2 = (d2 + t2) / a2 from scal = {a2, d2, t2, ...}; scal[3] = E.  With zero_t2 the t2 slot is
// cleared first (the error was measured directly, no extra term).
__global__ void k_final_err(double* scal, int zero_t2, long bs)
{
    scal = bshift(scal, bs);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (zero_t2) scal[2] = 0.0;
        double a2 = scal[0];
        scal[3] = a2 > 0.0 ? sqrt(fmax(scal[1] + scal[2], 0.0) / a2) : 0.0;
    }
}

hipError_t launch_final_err(double* scal, hipStream_t s, Bat bt, bool zero_t2)
{
    hipLaunchKernelGGL(k_final_err, dim3(1, 1, bt.nb), dim3(64), 0, s, scal, zero_t2 ? 1 : 0, bt.bs);
    return hipGetLastError();
}

// Zero the columns c >= rank_k of the three n_k x R_k factors and the core entries outside the
// leading r0 x r1 x r2 block (ranks from device memory), so that rank-R kernels evaluate the
// rank-r result exactly.  One launch: elements [off[k], off[k+1]) of the flat index space belong
// to factor k, the rest to the core.
struct MaskArgs {
    double* U[3];
    int R[3];
    long off[4];
    double* core;
    long total;
};

__global__ void k_mask_all(MaskArgs a, const int* __restrict__ ranks, long bs)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.total) return;
    ranks = bshift(ranks, bs);
    if (e < a.off[3]) {
        const int k = (e < a.off[1]) ? 0 : ((e < a.off[2]) ? 1 : 2);
        const long i = e - a.off[k];
        if ((int)(i % a.R[k]) >= ranks[k]) bshift(a.U[k], bs)[i] = 0.0;
    } else {
        const int i = (int)(e - a.off[3]);
        const int R12 = a.R[1] * a.R[2];
        const int x = i / R12, y = (i - x * R12) / a.R[2], z = i - x * R12 - y * a.R[2];
        if (x >= ranks[0] || y >= ranks[1] || z >= ranks[2]) bshift(a.core, bs)[i] = 0.0;
    }
}

hipError_t launch_mask_rank(double* const U[3], const int n[3], const int R[3], double* core, const int* ranks,
                            hipStream_t s, Bat bt)
{
    MaskArgs a{};
    a.off[0] = 0;
    for (int k = 0; k < 3; ++k) {
        a.U[k] = U[k];
        a.R[k] = R[k];
        a.off[k + 1] = a.off[k] + (long)n[k] * R[k];
    }
    a.core = core;
    a.total = a.off[3] + (long)R[0] * R[1] * R[2];
    hipLaunchKernelGGL(k_mask_all, dim3((unsigned)((a.total + 255) / 256), 1, bt.nb), dim3(256), 0, s, a, ranks,
                       bt.bs);
    return hipGetLastError();
}

}  // namespace tk
