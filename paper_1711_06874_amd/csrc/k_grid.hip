// a1: collocation tensor of a radial covariance function (Sec. 3.7 eq. (3.25)).
//
// A[i0,i1,i2] = sigma2 * k(||(x_i0, y_i1, z_i2)||), C-order.  Node coordinates and the radius
// are formed in double (x = x0 + i h, r = sqrt((x^2 + y^2) + z^2)) and the kernel is
// evaluated in double, then rounded once to the storage type (for float storage with a
// shorter exponential and square root whose ~1e-10 relative error is far below half a float
// ulp).  Each thread writes 4
// consecutive elements of one i2-row (one 16-byte store for float rows whose length is a
// multiple of 4); the grid is a flat 1-D launch over rows x ceil(n2/4) quads, so stores
// from a wave cover contiguous 1 KiB (float) / 2 KiB (double) spans.
#include "tk_kernels.h"

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
    node_params(A, g, kps, bt, nd);
}

void grid_eval_node_f64(double* A, const GridAxes& g, const KernelParams* kps, Bat bt, GridEvalNode* nd)
{
    node_params(A, g, kps, bt, nd);
}

hipError_t launch_grid_eval_f32(float* A, const GridAxes& g, const KernelParams* kps, hipStream_t s, Bat bt)
{
    return launch(A, g, kps, s, bt);
}

hipError_t launch_grid_eval_f64(double* A, const GridAxes& g, const KernelParams* kps, hipStream_t s, Bat bt)
{
    return launch(A, g, kps, s, bt);
}

}  // namespace tk
