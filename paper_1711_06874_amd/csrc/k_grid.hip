// a1: collocation tensor of a radial covariance function (Sec. 3.7 eq. (3.25)).
//
// A[i0,i1,i2] = sigma2 * k(||(x_i0, y_i1, z_i2)||), C-order.  Node coordinates and the radius
// are formed in double (x = x0 + i h, r = sqrt((x^2 + y^2) + z^2)).
//
// Double storage (k_grid_eval): the kernel in double with the library exponential, one thread
// per 4 consecutive elements of an i2-row.
//
// Float storage (k_grid_eval_f32): one wavefront per i2-row (i0, i1), each lane a float4 of the
// row.  When the first two axes carry the same nodes (equal n, first node, spacing and metric
// scale), x^2 + y^2 is symmetric in (i0, i1) (up to the last bit of a fused multiply-add, far
// below float resolution), so only rows with i0 <= i1 are evaluated and each is stored as row
// (i0, i1) and row (i1, i0).  The closed forms
// (Matern nu = 1/2, 3/2, 5/2, Slater with p = 1, Gauss) take exp(-s) = 2^k 2^f with
// u = -s log2(e) = k + f, |f| <= 1/2, in double, 2^f from the hardware FP32 exp2 of f (rounded
// to float), the polynomial factor and the scaling by 2^k in double, and one final rounding to
// float.  The value is within 3.2 * 2^-24 relative of the exact one (the exp2's 1 ulp of a value
// in [0.70, 1.42] is at most 2^-23 relative, f's rounding ln2 2^-26, the final rounding 2^-24);
// the other families take the double evaluation.
#include "tk_kernels.h"

#include <algorithm>
#include <cmath>

namespace tk {

template <typename T>
__global__ void __launch_bounds__(256) k_grid_eval(T* __restrict__ A, GridAxes g, KernelParamsBatch kps,
                                                   long total_quads, int quads_per_row, long bs)
{
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total_quads) return;
    A = bshift(A, bs);
    const KernelParams& kp = kps.k[blockIdx.z];
    long row;
    int i0, i1, i2;
    if (total_quads <= 0x7fffffffL) {
        // 32-bit unsigned divisions (a 64-bit division costs several times more)
        const unsigned q32 = (unsigned)q, qpr = (unsigned)quads_per_row, n1 = (unsigned)g.n[1];
        const unsigned row32 = q32 / qpr;
        const unsigned i0u = row32 / n1;
        i2 = (int)(q32 - row32 * qpr) * 4;
        i1 = (int)(row32 - i0u * n1);
        i0 = (int)i0u;
        row = (long)row32;
    } else {
        row = q / quads_per_row;
        i2 = (int)(q - row * quads_per_row) * 4;
        i1 = (int)(row % g.n[1]);
        i0 = (int)(row / g.n[1]);
    }
    // coordinates scaled by sqrt(a_k) for an anisotropic metric (exactly 1 otherwise)
    double x = (g.x0[0] + (double)i0 * g.h[0]) * kp.axs[0];
    double y = (g.x0[1] + (double)i1 * g.h[1]) * kp.axs[1];
    double xy = x * x + y * y;
    T out[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        double z = (g.x0[2] + (double)(i2 + t) * g.h[2]) * kp.axs[2];
        const double r2 = xy + z * z;
        if constexpr (sizeof(T) == 4) out[t] = (T)cov_value_for_float(kp, r2);
        else out[t] = (T)cov_value(kp, sqrt(r2));
    }
    T* dst = A + row * g.n[2] + i2;
    if (i2 + 4 <= g.n[2]) {
        if (sizeof(T) == 4 && (g.n[2] & 3) == 0) {
            *reinterpret_cast<float4*>(dst) = make_float4((float)out[0], (float)out[1], (float)out[2],
                                                          (float)out[3]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) dst[t] = out[t];
        }
    } else {
        for (int t = 0; t < 4 && i2 + t < g.n[2]; ++t) dst[t] = out[t];
    }
}

// exp(-s) scaled by the polynomial factor P(s), rounded once to float (see the header).
__device__ __forceinline__ float poly_exp_neg_f32(double s, double c0, double c1, double c2)
{
    const double u = s * -1.4426950408889634;
    const double k = rint(u);
    const float f = (float)(u - k);
    const double e = (double)__builtin_amdgcn_exp2f(f);
    const double poly = fma(fma(c2, s, c1), s, c0);
    return (float)ldexp(poly * e, (int)fmax(k, -2000.0));
}

enum { GF_M12 = 0, GF_M32 = 1, GF_M52 = 2, GF_SLATER1 = 3, GF_GAUSS = 4, GF_GENERAL = 5 };

__device__ __forceinline__ int grid_fast_kind(const KernelParams& kp)
{
    if (kp.family == FAM_MATERN && kp.half >= 0 && kp.half <= 2) return kp.half;
    if (kp.family == FAM_SLATER && kp.p == 1.0) return GF_SLATER1;
    if (kp.family == FAM_GAUSS) return GF_GAUSS;
    return GF_GENERAL;
}

template <int KIND>
__device__ __forceinline__ float grid_value_f32(const KernelParams& kp, double r2)
{
    if (KIND == GF_GENERAL) return (float)cov_value_for_float(kp, r2);
    double r = 0.0;
    if (r2 > 0.0) {
        double y = __builtin_amdgcn_rsq(r2);
        y = y * fma(-0.5 * r2 * y, y, 1.5);
        r = r2 * y;
    }
    const double t = r * kp.inv_len;
    const double sg = kp.sigma2;
    if (KIND == GF_M12) return poly_exp_neg_f32(t, sg, 0.0, 0.0);
    if (KIND == GF_M32) return poly_exp_neg_f32(t, sg, sg, 0.0);
    if (KIND == GF_M52) return poly_exp_neg_f32(t, sg, sg, sg * (1.0 / 3.0));
    if (KIND == GF_SLATER1) return poly_exp_neg_f32(kp.alpha * t, sg, 0.0, 0.0);
    return poly_exp_neg_f32(t * t, sg, 0.0, 0.0);
}

template <int KIND>
__device__ __forceinline__ void grid_row_f32(float* __restrict__ dst, float* __restrict__ dst2, const GridAxes& g,
                                             const KernelParams& kp, double xy, int qpr, int lane)
{
    const int n2 = g.n[2];
    const bool vec = (n2 & 3) == 0;
    for (int q = lane; q < qpr; q += 64) {
        const int i2 = 4 * q;
        float out[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double z = (g.x0[2] + (double)(i2 + t) * g.h[2]) * kp.axs[2];
            out[t] = grid_value_f32<KIND>(kp, xy + z * z);
        }
        if (vec) {
            const f32x4 v = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<f32x4*>(dst + i2) = v;
            if (dst2) *reinterpret_cast<f32x4*>(dst2 + i2) = v;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (i2 + t < n2) {
                    dst[i2 + t] = out[t];
                    if (dst2) dst2[i2 + t] = out[t];
                }
        }
    }
}

// Float storage.  Block (x, y) takes the two i0-planes x and n0 - 1 - x (together n1 + 1 rows
// under the symmetry, so every block has the same work) and its 4 waves rows i1 = lo + 4 y + w,
// stepping by 4 gridDim.y, where lo = i0 with the symmetry (rows i1 >= i0 only) and 0 without.
template <int KIND>
__device__ __forceinline__ void grid_rows_f32(float* __restrict__ A, const GridAxes& g, const KernelParams& kp,
                                              int qpr, int sym, int lane)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)blockIdx.y * 4 + (int)(threadIdx.x >> 6));
    const int nw = (int)gridDim.y * 4;
    const int n0 = g.n[0], n1 = g.n[1];
    for (int h = 0; h < 2; ++h) {
        const int i0 = h == 0 ? (int)blockIdx.x : n0 - 1 - (int)blockIdx.x;
        if (h == 1 && i0 <= (int)blockIdx.x) break;   // the middle plane of an odd n0: once
        const double x = (g.x0[0] + (double)i0 * g.h[0]) * kp.axs[0];
        for (int i1 = (sym ? i0 : 0) + wv; i1 < n1; i1 += nw) {
            const double y = (g.x0[1] + (double)i1 * g.h[1]) * kp.axs[1];
            const double xy = x * x + y * y;
            float* dst = A + ((long)i0 * n1 + i1) * g.n[2];
            float* dst2 = (sym && i0 != i1) ? A + ((long)i1 * n1 + i0) * g.n[2] : nullptr;
            grid_row_f32<KIND>(dst, dst2, g, kp, xy, qpr, lane);
        }
    }
}

// GENERAL: also the families without a closed form (kept out of the closed-form instance, whose
// register count they would raise).
template <bool GENERAL>
__global__ void __launch_bounds__(256) k_grid_eval_f32(float* __restrict__ A, GridAxes g, KernelParamsBatch kps,
                                                       int qpr, int sym, long bs)
{
    A = bshift(A, bs);
    const KernelParams& kp = kps.k[blockIdx.z];
    const int lane = threadIdx.x & 63;
    switch (grid_fast_kind(kp)) {
    case GF_M12: grid_rows_f32<GF_M12>(A, g, kp, qpr, sym, lane); break;
    case GF_M32: grid_rows_f32<GF_M32>(A, g, kp, qpr, sym, lane); break;
    case GF_M52: grid_rows_f32<GF_M52>(A, g, kp, qpr, sym, lane); break;
    case GF_SLATER1: grid_rows_f32<GF_SLATER1>(A, g, kp, qpr, sym, lane); break;
    case GF_GAUSS: grid_rows_f32<GF_GAUSS>(A, g, kp, qpr, sym, lane); break;
    default:
        if constexpr (GENERAL) grid_rows_f32<GF_GENERAL>(A, g, kp, qpr, sym, lane);
        break;
    }
}

// Uneven batches in one persistent launch: every work item is one plane pair (i0, n0 - 1 - i0)
// of one job's grid; the resident work-groups take items from a device counter until none is
// left (every group reaches the exit), each item in the order of the item list (jobs by
// descending size, so the largest planes start first).  A job's rows and values are those of
// k_grid_eval_f32 for the same grid.
__global__ void __launch_bounds__(256) k_grid_eval_f32_queue(const GridJob* __restrict__ jobs, int njobs,
                                                             const int* __restrict__ first_item, int nitems,
                                                             unsigned* __restrict__ counter)
{
    __shared__ int item_s;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (;;) {
        if (threadIdx.x == 0) item_s = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= nitems) return;
        // the job holding this item: first_item is increasing, first_item[njobs] == nitems
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first_item[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const GridJob& jb = jobs[lo];
        const int pair = item - first_item[lo];
        const GridAxes& g = jb.g;
        const KernelParams& kp = jb.kp;
        const int n0 = g.n[0], n1 = g.n[1];
        for (int h = 0; h < 2; ++h) {
            const int i0 = h == 0 ? pair : n0 - 1 - pair;
            if (h == 1 && i0 <= pair) break;
            const double x = (g.x0[0] + (double)i0 * g.h[0]) * kp.axs[0];
            for (int i1 = (jb.sym ? i0 : 0) + wv; i1 < n1; i1 += 4) {
                const double y = (g.x0[1] + (double)i1 * g.h[1]) * kp.axs[1];
                const double xy = x * x + y * y;
                float* dst = jb.A + ((long)i0 * n1 + i1) * g.n[2];
                float* dst2 = (jb.sym && i0 != i1) ? jb.A + ((long)i1 * n1 + i0) * g.n[2] : nullptr;
                switch (grid_fast_kind(kp)) {
                case GF_M12: grid_row_f32<GF_M12>(dst, dst2, g, kp, xy, jb.qpr, lane); break;
                case GF_M32: grid_row_f32<GF_M32>(dst, dst2, g, kp, xy, jb.qpr, lane); break;
                case GF_M52: grid_row_f32<GF_M52>(dst, dst2, g, kp, xy, jb.qpr, lane); break;
                case GF_SLATER1: grid_row_f32<GF_SLATER1>(dst, dst2, g, kp, xy, jb.qpr, lane); break;
                case GF_GAUSS: grid_row_f32<GF_GAUSS>(dst, dst2, g, kp, xy, jb.qpr, lane); break;
                default: grid_row_f32<GF_GENERAL>(dst, dst2, g, kp, xy, jb.qpr, lane); break;
                }
            }
        }
    }
}

// Launch shape of k_grid_eval_f32: ceil(n0/2) plane pairs, and about 8192 waves in all.
static dim3 grid_f32_shape(const GridAxes& g, int nb)
{
    const int pairs = (g.n[0] + 1) / 2;
    int sy = (2048 + pairs - 1) / pairs;
    const int cap = (g.n[1] + 3) / 4;
    if (sy > cap) sy = cap;
    if (sy < 1) sy = 1;
    return dim3((unsigned)pairs, (unsigned)sy, (unsigned)nb);
}

static bool grid_general(const KernelParams* kps, int nb)
{
    for (int b = 0; b < nb; ++b) {
        const KernelParams& k = kps[b];
        const bool fast = (k.family == FAM_MATERN && k.half >= 0 && k.half <= 2) ||
                          (k.family == FAM_SLATER && k.p == 1.0) || k.family == FAM_GAUSS;
        if (!fast) return true;
    }
    return false;
}

static int grid_symmetric(const GridAxes& g, const KernelParams* kps, int nb)
{
    if (g.n[0] != g.n[1] || g.x0[0] != g.x0[1] || g.h[0] != g.h[1]) return 0;
    for (int b = 0; b < nb; ++b)
        if (kps[b].axs[0] != kps[b].axs[1]) return 0;
    return 1;
}

static hipError_t launch_f32(float* A, const GridAxes& g, const KernelParams* kps, hipStream_t s, Bat bt)
{
    if (bt.nb < 1 || bt.nb > BATCH_MAX) return hipErrorInvalidValue;
    KernelParamsBatch kb{};
    for (int b = 0; b < bt.nb; ++b) kb.k[b] = kps[b];
    const int qpr = (g.n[2] + 3) / 4;
    const int sym = grid_symmetric(g, kps, bt.nb);
    const dim3 grid = grid_f32_shape(g, bt.nb);
    if (grid_general(kps, bt.nb))
        hipLaunchKernelGGL(k_grid_eval_f32<true>, grid, dim3(256), 0, s, A, g, kb, qpr, sym, bt.bs);
    else
        hipLaunchKernelGGL(k_grid_eval_f32<false>, grid, dim3(256), 0, s, A, g, kb, qpr, sym, bt.bs);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch(T* A, const GridAxes& g, const KernelParams* kps, hipStream_t s, Bat bt)
{
    if (bt.nb < 1 || bt.nb > BATCH_MAX) return hipErrorInvalidValue;
    KernelParamsBatch kb{};
    for (int b = 0; b < bt.nb; ++b) kb.k[b] = kps[b];
    int qpr = (g.n[2] + 3) / 4;
    long rows = (long)g.n[0] * g.n[1];
    long total = rows * qpr;
    long blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_grid_eval<T>, dim3((unsigned)blocks, 1, bt.nb), dim3(256), 0, s, A, g, kb, total, qpr,
                       bt.bs);
    return hipGetLastError();
}

template <typename T>
static void node_params(T* A, const GridAxes& g, const KernelParams* kps, Bat bt, GridEvalNode* nd)
{
    nd->A = A;
    nd->g = g;
    for (int b = 0; b < bt.nb; ++b) nd->kps.k[b] = kps[b];
    nd->qpr = (g.n[2] + 3) / 4;
    nd->total = (long)g.n[0] * g.n[1] * nd->qpr;
    nd->bs = bt.bs;
    nd->args[0] = &nd->A;
    nd->args[1] = &nd->g;
    nd->args[2] = &nd->kps;
    nd->args[3] = &nd->total;
    nd->args[4] = &nd->qpr;
    nd->args[5] = &nd->bs;
    nd->p.func = reinterpret_cast<void*>(&k_grid_eval<T>);
    nd->p.gridDim = dim3((unsigned)((nd->total + 255) / 256), 1, bt.nb);
    nd->p.blockDim = dim3(256);
    nd->p.sharedMemBytes = 0;
    nd->p.kernelParams = nd->args;
    nd->p.extra = nullptr;
}

void grid_eval_node_f32(float* A, const GridAxes& g, const KernelParams* kps, Bat bt, GridEvalNode* nd)
{
    nd->A = A;
    nd->g = g;
    for (int b = 0; b < bt.nb; ++b) nd->kps.k[b] = kps[b];
    nd->qpr = (g.n[2] + 3) / 4;
    nd->sym = grid_symmetric(g, kps, bt.nb);
    nd->bs = bt.bs;
    nd->args[0] = &nd->A;
    nd->args[1] = &nd->g;
    nd->args[2] = &nd->kps;
    nd->args[3] = &nd->qpr;
    nd->args[4] = &nd->sym;
    nd->args[5] = &nd->bs;
    nd->p.func = grid_general(kps, bt.nb) ? reinterpret_cast<void*>(&k_grid_eval_f32<true>)
                                          : reinterpret_cast<void*>(&k_grid_eval_f32<false>);
    nd->p.gridDim = grid_f32_shape(g, bt.nb);
    nd->p.blockDim = dim3(256);
    nd->p.sharedMemBytes = 0;
    nd->p.kernelParams = nd->args;
    nd->p.extra = nullptr;
}

void grid_eval_node_f64(double* A, const GridAxes& g, const KernelParams* kps, Bat bt, GridEvalNode* nd)
{
    node_params(A, g, kps, bt, nd);
}

GridJob grid_job_f32(float* A, const GridAxes& g, const KernelParams& kp)
{
    GridJob j{};
    j.A = A;
    j.g = g;
    j.kp = kp;
    j.qpr = (g.n[2] + 3) / 4;
    j.sym = grid_symmetric(g, &kp, 1);
    return j;
}

int grid_job_items(const GridJob& j) { return (j.g.n[0] + 1) / 2; }

hipError_t launch_grid_eval_f32_queue(const GridJob* jobs_dev, int njobs, const int* first_item_dev, int nitems,
                                      unsigned* counter_dev, hipStream_t s)
{
    if (njobs < 1 || nitems < 1) return hipErrorInvalidValue;
    // as many work-groups as stay resident (8 per CU), or one per item
    const int groups = nitems < 2048 ? nitems : 2048;
    hipLaunchKernelGGL(k_grid_eval_f32_queue, dim3(groups), dim3(256), 0, s, jobs_dev, njobs, first_item_dev, nitems,
                       counter_dev);
    return hipGetLastError();
}

// ---- radial tables ---------------------------------------------------------------------------
// For Matern orders without a closed form (K_nu by series or continued fraction per value) on
// grids whose axes share the
// spacing h, with first nodes in (h/2) Z and an isotropic metric, every squared radius is
// a (h/2)^2 m for an integer m = sum_k (c_k + 2 i_k)^2 (c_k = 2 x0_k / h, a the metric scale).
// The kernel is then evaluated once per value of m (a table of at most sum_k (n_k - 1)^2 + 1
// entries after dividing out the parity: all c_k even gives m = 4 m', all odd m = 8 m' + 3) and
// the grid gathers from it: 195,076 Bessel evaluations instead of 16.8 M at 256^3.  The table
// holds the FP64 values, rounded once to float for float storage.

// The route pays for a Matern order without a closed form (hundreds of FP64 operations per value);
// the spectral density and Slater p != 1 (one log / pow per value) are faster evaluated directly
// than gathered from a table.
static bool table_kind_host(const KernelParams& kp) { return kp.family == FAM_MATERN && kp.half < 0; }

long radial_table_cap(const int n[3])
{
    long t = 1;
    for (int k = 0; k < 3; ++k) t += (long)(n[k] - 1) * (n[k] - 1);
    return t;
}

bool radial_plan(const GridAxes& g, const KernelParams* kps, int nb, RadialGrid* rg)
{
    if (nb < 1) return false;
    for (int b = 0; b < nb; ++b) {
        const KernelParams& kp = kps[b];
        if (!table_kind_host(kp)) return false;
        if (kp.axs[1] != kp.axs[0] || kp.axs[2] != kp.axs[0]) return false;
        if (b > 0 && kp.axs[0] != kps[0].axs[0]) return false;
    }
    const double h = g.h[0];
    if (!(h > 0.0)) return false;
    int odd = 0;
    long mmax = 0;
    for (int k = 0; k < 3; ++k) {
        if (std::fabs(g.h[k] - h) > 1e-15 * h) return false;
        const double c = 2.0 * g.x0[k] / h;
        const double cr = std::rint(c);
        if (std::fabs(c - cr) > 1e-12 * std::fmax(1.0, std::fabs(c)) || std::fabs(cr) > (double)(1 << 20)) return false;
        rg->c[k] = (int)cr;
        odd += (rg->c[k] & 1);
        const long u0 = rg->c[k], u1 = rg->c[k] + 2L * (g.n[k] - 1);
        mmax += std::max(u0 * u0, u1 * u1);
    }
    rg->mode = (odd == 0) ? 4 : (odd == 3 ? 8 : 1);
    rg->T = (rg->mode == 4) ? mmax / 4 + 1 : (rg->mode == 8 ? (mmax - 3) / 8 + 1 : mmax + 1);
    if (rg->T > radial_table_cap(g.n)) return false;
    const double a = kps[0].axs[0];
    rg->q = a * a * 0.25 * h * h;
    return true;
}

__global__ void __launch_bounds__(256) k_radial_table(double* __restrict__ table, RadialGrid rg, KernelParamsBatch kps,
                                                      long bs)
{
    table = bshift(table, bs);
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rg.T) return;
    const long m = (rg.mode == 4) ? 4 * idx : (rg.mode == 8 ? 8 * idx + 3 : idx);
    table[idx] = cov_value(kps.k[blockIdx.z], sqrt(rg.q * (double)m));
}

// sym: the first two axes carry the same nodes, so row (i1, i0) equals row (i0, i1): threads of
// rows with i0 > i1 stop, the others store their values in both rows.
template <typename T>
__global__ void __launch_bounds__(256) k_grid_from_table(T* __restrict__ A, GridAxes g, RadialGrid rg,
                                                         const double* __restrict__ table, long total_quads,
                                                         int quads_per_row, int sym, long bs)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total_quads) return;
    A = bshift(A, bs);
    table = bshift(table, bs);
    long row;
    int i0, i1, i2;
    if (total_quads <= 0x7fffffffL) {
        const unsigned q32 = (unsigned)q, qpr = (unsigned)quads_per_row, n1 = (unsigned)g.n[1];
        const unsigned row32 = q32 / qpr;
        const unsigned i0u = row32 / n1;
        i2 = (int)(q32 - row32 * qpr) * 4;
        i1 = (int)(row32 - i0u * n1);
        i0 = (int)i0u;
        row = (long)row32;
    } else {
        row = q / quads_per_row;
        i2 = (int)(q - row * quads_per_row) * 4;
        i1 = (int)(row % g.n[1]);
        i0 = (int)(row / g.n[1]);
    }
    if (sym && i0 > i1) return;
    const long u0 = rg.c[0] + 2L * i0, u1 = rg.c[1] + 2L * i1;
    const long m01 = u0 * u0 + u1 * u1;
    T out[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const long u2 = rg.c[2] + 2L * (i2 + t < g.n[2] ? i2 + t : i2);
        const long m = m01 + u2 * u2;
        const long idx = (rg.mode == 4) ? (m >> 2) : (rg.mode == 8 ? (m - 3) >> 3 : m);
        out[t] = (T)table[idx];
    }
    const int copies = (sym && i0 != i1) ? 2 : 1;
    for (int cpy = 0; cpy < copies; ++cpy) {
        const long r = (cpy == 0) ? row : (long)i1 * g.n[1] + i0;
        T* dst = A + r * g.n[2] + i2;
        if (i2 + 4 <= g.n[2]) {
            if (sizeof(T) == 4 && (g.n[2] & 3) == 0) {
                *reinterpret_cast<float4*>(dst) =
                    make_float4((float)out[0], (float)out[1], (float)out[2], (float)out[3]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) dst[t] = out[t];
            }
        } else {
            for (int t = 0; t < 4 && i2 + t < g.n[2]; ++t) dst[t] = out[t];
        }
    }
}

hipError_t launch_grid_eval_radial(void* A, int esz, const GridAxes& g, const KernelParams* kps, const RadialGrid& rg,
                                   double* table, hipStream_t s, Bat bt)
{
    if (bt.nb < 1 || bt.nb > BATCH_MAX || (esz != 4 && esz != 8)) return hipErrorInvalidValue;
    KernelParamsBatch kb;
    for (int b = 0; b < bt.nb; ++b) kb.k[b] = kps[b];
    hipLaunchKernelGGL(k_radial_table, dim3((unsigned)((rg.T + 255) / 256), 1, bt.nb), dim3(256), 0, s, table, rg, kb,
                       bt.bs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int qpr = (g.n[2] + 3) / 4;
    const long total = (long)g.n[0] * g.n[1] * qpr;
    const int sym = (g.n[0] == g.n[1] && rg.c[0] == rg.c[1]) ? 1 : 0;
    const dim3 grid((unsigned)((total + 255) / 256), 1, bt.nb);
    if (esz == 4)
        hipLaunchKernelGGL(k_grid_from_table<float>, grid, dim3(256), 0, s, (float*)A, g, rg, (const double*)table,
                           total, qpr, sym, bt.bs);
    else
        hipLaunchKernelGGL(k_grid_from_table<double>, grid, dim3(256), 0, s, (double*)A, g, rg, (const double*)table,
                           total, qpr, sym, bt.bs);
    return hipGetLastError();
}

hipError_t launch_grid_eval_f32(float* A, const GridAxes& g, const KernelParams* kps, hipStream_t s, Bat bt)
{
    return launch_f32(A, g, kps, s, bt);
}

hipError_t launch_grid_eval_f64(double* A, const GridAxes& g, const KernelParams* kps, hipStream_t s, Bat bt)
{
    return launch(A, g, kps, s, bt);
}

}  // namespace tk
