// a8 (FFT form): the Kronecker-Toeplitz covariance matvec diagonalised by the 3-D DFT.
//
// Sec. 3.6 notes that a Toeplitz matrix times a vector costs O(n log n) by completing it to a
// circulant.  Every factor T(u)_{ij} = u[off + |i - j|] (i, j < m) embeds in the circulant of
// length L >= 2m - 1 (a power of two) whose first column is
//     c[t] = u[off + t] (0 <= t < m),  c[L - t] = u[off + t] (1 <= t < m),  0 elsewhere,
// so T(u) x = (C x_pad)[0:m] with C = F^-1 diag(F c) F.  The covariance
//     C = sum_abc G_abc T(U1[:,a]) (x) T(U2[:,b]) (x) T(U3[:,c])
// is then P (F^-1 (x) F^-1 (x) F^-1) diag(chat) (F (x) F (x) F) P^T with the Fourier-side
// generator
//     chat[f0][f1][f2] = sum_abc G_abc Uh1[f0][a] Uh2[f1][b] Uh3[f2][c],
//     Uh[f][a] = u_a[off] + 2 sum_{t=1}^{m-1} u_a[off + t] cos(2 pi f t / L)   (real, even c)
// which is again a Tucker tensor.  The matvec is five passes over the data:
//   P1  axis 2, forward, real input zero-padded, keeps f2 <= L2/2   (m0 m1 rows)
//   P2  axis 1, forward                                             (m0 x H2 fibres)
//   P3  axis 0, forward, times chat, inverse, keeps i0 < m0          (L1 x H2 fibres, in place)
//   P4  axis 1, inverse, keeps i1 < m1
//   P5  axis 2, inverse from the half spectrum (Hermitian), real part, keeps i2 < m2, 1/(L0 L1 L2)
// with H2 = L2/2 + 1.  chat is evaluated on the fly in P3 from Hs[f0][f1][c] = sum_ab
// G_abc Uh1[f0][a] Uh2[f1][b] and Uh3.
//
// Each work-group transforms F fibres of length L together in LDS (F L <= 8192 complex
// values, two ping-pong buffers): a mixed radix-8/4/2 Stockham autosort FFT, natural order in
// and out, one radix-R butterfly per thread per stage, twiddles exp(-/+ 2 pi i q / L) from a
// table computed once per matvec with double-precision sincospi (512-thread work-groups).  Global loads and stores are
// coalesced: along the fibre when it is contiguous, across neighbouring fibres otherwise.
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr int FFT_LDS_COMPLEX = 8192;
constexpr int FFT_THREADS = 512;
constexpr size_t FFT_LDS_MAX = 96 * 1024;

// LDS position of complex element x of a block: one spare slot after every 16 values, so the
// power-of-two strides of the Stockham stages do not pile onto a few banks.
__device__ __forceinline__ int pd(int x) { return x + (x >> 4); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ float2 cmul_mi(float2 a, bool inv) { return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }

__device__ __forceinline__ void dft2(float2* v)
{
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2* v, bool inv)
{
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = cmul_mi(csub(v[1], v[3]), inv);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

__device__ __forceinline__ void dft8(float2* v, bool inv)
{
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e, inv);
    dft4(o, inv);
    const float h = 0.70710678118654752f;
    // o[k] *= W8^k, W8 = exp(-/+ i pi / 4)
    o[1] = inv ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    o[2] = cmul_mi(o[2], inv);
    o[3] = inv ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    for (int k = 0; k < 4; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

// One Stockham stage of radix R = 2^LR over F fibres, in place: every thread reads all of its
// butterflies' inputs into registers (at most FFT_LDS_COMPLEX / FFT_THREADS values), the block
// synchronises, and the outputs are written to their new positions.  Ns = 2^lns.
template <int LR>
__device__ __forceinline__ void stockham_stage(float2* X, const float2* __restrict__ tw, int F, int logL, int lns,
                                               bool inv)
{
    constexpr int R = 1 << LR;
    constexpr int NB = (FFT_LDS_COMPLEX / FFT_THREADS) / R;     // butterflies per thread
    const int L = 1 << logL;
    const int Ns = 1 << lns;
    const int lq = logL - LR;
    const int Q = 1 << lq;
    const int nbf = F << lq;
    float2 v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int e = threadIdx.x + FFT_THREADS * b;
        if (e < nbf) {
            const int f = e >> lq, j = e & (Q - 1);
            const int k = j & (Ns - 1);
            const int sf = f * L;
            const int twstep = k << (logL - lns - LR);       // q = k r L / (Ns R)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = X[pd(sf + j + r * Q)];
                if (r > 0 && k > 0) {
                    float2 w = tw[(twstep * r) & (L - 1)];
                    if (inv) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[b][r] = x;
            }
            if (R == 8) dft8(v[b], inv);
            else if (R == 4) dft4(v[b], inv);
            else dft2(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int e = threadIdx.x + FFT_THREADS * b;
        if (e < nbf) {
            const int f = e >> lq, j = e & (Q - 1);
            const int k = j & (Ns - 1);
            const int df = f * L + ((j >> lns) << (lns + LR)) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) X[pd(df + (r << lns))] = v[b][r];
        }
    }
    __syncthreads();
}

// Stockham FFT, in place, of F fibres of length L = 2^logL at X[pd(f * L + k)] (natural order
// in and out); tw[q] = exp(-2 pi i q / L), q < L.
__device__ void fft_lds(float2* X, const float2* tw, int F, int logL, bool inv)
{
    int lns = 0, rem = logL;
    while (rem > 0) {
        const int lr = (rem >= 3) ? 3 : rem;          // radix 8, then 4 or 2
        if (lr == 3) stockham_stage<3>(X, tw, F, logL, lns, inv);
        else if (lr == 2) stockham_stage<2>(X, tw, F, logL, lns, inv);
        else stockham_stage<1>(X, tw, F, logL, lns, inv);
        lns += lr;
        rem -= lr;
    }
}

// R[f][f0] *= chat = sum_c Hs[f0][o][c] Uh3s[f][c] for f < nf (RB >= r2 registers per row).
template <int RB>
__device__ void times_chat(float2* R, int L, int nf, const float* __restrict__ Hs, int L1, long o,
                           const float* u3s, int r2)
{
    for (int f0 = threadIdx.x; f0 < L; f0 += blockDim.x) {
        const float* h = Hs + ((long)f0 * L1 + o) * r2;
        float hr[RB];
#pragma unroll
        for (int c = 0; c < RB; ++c) hr[c] = (c < r2) ? h[c] : 0.f;
        for (int f = 0; f < nf; ++f) {
            float chat = 0.f;
#pragma unroll
            for (int c = 0; c < RB; ++c)
                if (c < r2) chat += hr[c] * u3s[f * r2 + c];
            const float2 v = R[pd(f * L + f0)];
            R[pd(f * L + f0)] = make_float2(v.x * chat, v.y * chat);
        }
    }
}

__device__ void load_twiddles(float2* tw, const float2* __restrict__ gtw, int L)
{
    for (int q = threadIdx.x; q < L; q += blockDim.x) tw[q] = gtw[q];
}

}  // namespace

// Generic pass.  Fibre (o, i) of the pass: input element k (k < len_in) at
//   in + o * s_in_o + i * s_in_i + k * s_in_k   (float2, or float when in_real)
// and output element k (k < len_out) at out + o * s_out_o + i * s_out_i + k * s_out_k.
// Work-group: F fibres (o, i0 + f), f < F, i0 = blockIdx.x * F, o = blockIdx.y.
// mode 0: forward C2C / R2C;  mode 1: inverse C2C;  mode 2: inverse from a half spectrum
// (Hermitian extension of len_in = L/2 + 1 values), real output;  mode 3: forward, times
// chat, inverse (the P3 pass; fibres are (f1 = o, f2 = i)).
__global__ void __launch_bounds__(FFT_THREADS) k_fft_pass(FftPassArgs a)
{
    extern __shared__ __attribute__((aligned(16))) float2 fsm[];
    const int L = a.L, logL = a.logL, F = a.F;      // F: power of two <= FFT_THREADS
    float2* tw = fsm;
    float2* X = fsm + L;
    const long o = blockIdx.y;
    const int i0 = blockIdx.x * F;
    const int nf = (a.n_inner - i0 < F) ? (a.n_inner - i0) : F;
    const int tid = threadIdx.x;
    constexpr int NT = FFT_THREADS;
    load_twiddles(tw, a.tw, L);
    for (int e = tid; e < pd(F * L); e += NT) X[e] = make_float2(0.f, 0.f);
    __syncthreads();
    // ---- load (zero padded), natural order.  Contiguous fibres: threads walk k; strided
    // fibres: threads walk neighbouring fibres (f = tid % F), which are contiguous in memory.
    const int len_in = a.len_in;
    auto put = [&](int f, int k, float2 v) {
        X[pd(f * L + k)] = v;
        if (a.mode == 2 && k > 0 && k < (L >> 1)) X[pd(f * L + (L - k))] = make_float2(v.x, -v.y);
    };
    auto get = [&](long idx) -> float2 {
        if (a.in_real) return make_float2(((const float*)a.in)[idx], 0.f);
        return ((const float2*)a.in)[idx];
    };
    // every thread first issues all of its loads (up to QMAX), then scatters them into LDS
    constexpr int QMAX = FFT_LDS_COMPLEX / FFT_THREADS;
    const int total_in = nf * len_in;
    float2 buf[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int e = tid + NT * q;
        if (e < total_in) {
            int f, k;
            if (a.s_in_k == 1) { f = e / len_in; k = e - f * len_in; }
            else { f = e % nf; k = e / nf; }
            buf[q] = get(o * a.s_in_o + (long)(i0 + f) * a.s_in_i + (long)k * a.s_in_k);
        }
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int e = tid + NT * q;
        if (e < total_in) {
            int f, k;
            if (a.s_in_k == 1) { f = e / len_in; k = e - f * len_in; }
            else { f = e % nf; k = e / nf; }
            put(f, k, buf[q]);
        }
    }
    __syncthreads();
    fft_lds(X, tw, F, logL, a.mode == 1 || a.mode == 2);
    float2* R = X;
    if (a.mode == 3) {
        // times chat[f0][f1 = o][f2] = sum_c Hs[f0][f1][c] Uh3[f2][c]: each thread owns frequencies
        // f0 and reuses the Hs row for all fibres of the block
        float* u3s = reinterpret_cast<float*>(X + pd(F * L));      // F * r2 floats after the data
        for (int e = tid; e < nf * a.r2; e += NT) u3s[e] = a.Uh3[(long)i0 * a.r2 + e];
        __syncthreads();
        if (a.r2 <= 16) times_chat<16>(R, L, nf, a.Hs, a.L1, o, u3s, a.r2);
        else if (a.r2 <= 32) times_chat<32>(R, L, nf, a.Hs, a.L1, o, u3s, a.r2);
        else times_chat<48>(R, L, nf, a.Hs, a.L1, o, u3s, a.r2);
        __syncthreads();
        fft_lds(X, tw, F, logL, true);
    }
    // ---- store the first len_out entries
    const int len_out = a.len_out;
    auto put_out = [&](long idx, float2 v) {
        if (a.out_real) ((float*)a.out)[idx] = v.x * a.scale;
        else ((float2*)a.out)[idx] = make_float2(v.x * a.scale, v.y * a.scale);
    };
    const int total_out = nf * len_out;
    for (int e = tid; e < total_out; e += NT) {
        int f, k;
        if (a.s_out_k == 1) { f = e / len_out; k = e - f * len_out; }
        else { f = e % nf; k = e / nf; }
        put_out(o * a.s_out_o + (long)(i0 + f) * a.s_out_i + (long)k * a.s_out_k, R[pd(f * L + k)]);
    }
}

// tw[q] = exp(-2 pi i q / L) for q < L, from double-precision sincospi.
__global__ void k_twiddles(float2* tw, int L)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L) return;
    double sn, cs;
    sincospi(-2.0 * (double)q / (double)L, &sn, &cs);
    tw[q] = make_float2((float)cs, (float)sn);
}

hipError_t launch_twiddles(float2* tw, int L, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddles, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
    return hipGetLastError();
}

// Uh[f][a] = u_a[off] + 2 sum_{t=1}^{m-1} u_a[off + t] cos(2 pi f t / L) for f < nf, a < r
// (U: n x r row-major FP64; output nf x r FP64).  cos(2 pi q / L) comes from a per-block FP64
// table; the phase f t is reduced exactly modulo L (a power of two).
__global__ void __launch_bounds__(256) k_fourier_factor(const double* __restrict__ U, int r, int off, int m, int L,
                                                        int nf, double* __restrict__ Uh)
{
    extern __shared__ double ctab[];
    for (int q = threadIdx.x; q < L; q += blockDim.x) ctab[q] = cospi(2.0 * (double)q / (double)L);
    __syncthreads();
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)nf * r) return;
    const int f = (int)(e / r), a = (int)(e % r);
    const double* u = U + (long)off * r + a;
    double s = 0.0;
    int ph = 0;
    for (int t = 1; t < m; ++t) {
        ph = (ph + f) & (L - 1);
        s += u[(long)t * r] * ctab[ph];
    }
    Uh[e] = u[0] + 2.0 * s;
}

size_t fft_lds_bytes(int L, int F, int r2)
{
    size_t fl = (size_t)F * L;
    // twiddles, the data (padded), and F * r2 floats of scratch for the P3 pass
    return sizeof(float2) * ((size_t)L + fl + (fl >> 4)) + sizeof(float) * (size_t)F * r2;
}

int fft_fibres_per_block(int L, int r2)
{
    int F = FFT_LDS_COMPLEX / L;
    if (F > FFT_THREADS) F = FFT_THREADS;
    if (F < 1) F = 1;
    while (F > 1 && fft_lds_bytes(L, F, r2) > FFT_LDS_MAX) F >>= 1;
    return F;
}

hipError_t launch_fft_pass(const FftPassArgs& a, long n_outer, hipStream_t s)
{
    dim3 grid((unsigned)((a.n_inner + a.F - 1) / a.F), (unsigned)n_outer);
    hipLaunchKernelGGL(k_fft_pass, grid, dim3(FFT_THREADS), fft_lds_bytes(a.L, a.F, a.mode == 3 ? a.r2 : 0), s, a);
    return hipGetLastError();
}

hipError_t launch_fourier_factor(const double* U, int r, int off, int m, int L, int nf, double* Uh, hipStream_t s)
{
    long tot = (long)nf * r;
    hipLaunchKernelGGL(k_fourier_factor, dim3((unsigned)((tot + 255) / 256)), dim3(256), sizeof(double) * L, s, U, r,
                       off, m, L, nf, Uh);
    return hipGetLastError();
}

hipError_t fft_set_attributes()
{
    return hipFuncSetAttribute((const void*)k_fft_pass, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FFT_LDS_MAX);
}

}  // namespace tk
