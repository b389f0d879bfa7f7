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
constexpr int FFT_THREADS = 1024;
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
__device__ __forceinline__ void fft_lds(float2* X, const float2* tw, int F, int logL, bool inv)
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

// X[f][f0] *= chat[f0][f1 = o][f2 = i0 + f] = sum_c Hs[o][f0][c] Uh3[i0 + f][c] for f < nf.  Each thread
// owns frequencies f0 and keeps its Hs row (r2p <= 4 * RB4 floats, zero padded) in registers.
template <int RB4>
__device__ __forceinline__ void times_chat(float2* X, int L, int nf, const float* __restrict__ Hs, long o,
                                           const float* u3s, int r2p)
{
    const int n4 = r2p >> 2;
    for (int f0 = threadIdx.x; f0 < L; f0 += FFT_THREADS) {
        const float4* h = reinterpret_cast<const float4*>(Hs + ((long)o * L + f0) * r2p);
        float4 hr[RB4];
#pragma unroll
        for (int c = 0; c < RB4; ++c) hr[c] = (c < n4) ? h[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int f = 0; f < nf; ++f) {
            const float4* u = reinterpret_cast<const float4*>(u3s + f * r2p);
            float chat = 0.f;
#pragma unroll
            for (int c = 0; c < RB4; ++c) {
                if (c < n4) {
                    const float4 w = u[c];
                    chat += hr[c].x * w.x + hr[c].y * w.y + hr[c].z * w.z + hr[c].w * w.w;
                }
            }
            float2& v = X[pd(f * L + f0)];
            v = make_float2(v.x * chat, v.y * chat);
        }
    }
}

}  // namespace

// One pass over F fibres per work-group, fibre f = i0 + f_local (i0 = blockIdx.x * F), outer index
// o = blockIdx.y.  Element k of a fibre sits at
//   CONTIG:   base + o * s_o + f * s_i + k          (rows; P1 and P5)
//   !CONTIG:  base + o * s_o + f + k * s_k          (neighbouring fibres adjacent; P2, P3, P4)
// MODE 0: forward (real input when IN_REAL);  1: inverse;  2: inverse from the half spectrum
// (len_in = L/2 + 1, Hermitian extension), real output times scale;  3: forward, times chat,
// inverse (P3).  Inputs beyond len_in are zero; the first len_out outputs are stored.
template <int MODE, bool IN_REAL, bool CONTIG>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_pass(FftPassArgs a)
{
    extern __shared__ __attribute__((aligned(16))) float2 fsm[];
    constexpr int NT = FFT_THREADS;
    constexpr int QMAX = FFT_LDS_COMPLEX / FFT_THREADS;
    const int L = a.L, logL = a.logL, F = a.F, logF = a.logF;
    const int FL = F << logL;
    float2* tw = fsm;
    float2* X = fsm + L;
    const long o = blockIdx.y;
    const int i0 = blockIdx.x * F;
    const int nf = (a.n_inner - i0 < F) ? (a.n_inner - i0) : F;
    const int tid = threadIdx.x;
    const int len_in = a.len_in;
    // ---- every global load is issued first (zero for padding and for fibres past the end)
    float2 buf[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int e = tid + NT * q;
        const int f = CONTIG ? (e >> logL) : (e & (F - 1));
        const int k = CONTIG ? (e & (L - 1)) : (e >> logF);
        buf[q] = make_float2(0.f, 0.f);
        if (e < FL && f < nf && k < len_in) {
            const long idx = CONTIG ? o * a.s_in_o + (long)(i0 + f) * a.s_in_i + k
                                    : o * a.s_in_o + (i0 + f) + (long)k * a.s_in_k;
            if (IN_REAL) buf[q].x = static_cast<const float*>(a.in)[idx];
            else buf[q] = static_cast<const float2*>(a.in)[idx];
        }
    }
    for (int q = tid; q < L; q += NT) tw[q] = a.tw[q];
    float* u3s = reinterpret_cast<float*>(X + pd(FL));
    if (MODE == 3) {
        const int r2p = a.r2p;
        for (int e = tid; e < F * r2p; e += NT) u3s[e] = (e < nf * r2p) ? a.Uh3[(long)i0 * r2p + e] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int e = tid + NT * q;
        const int f = CONTIG ? (e >> logL) : (e & (F - 1));
        const int k = CONTIG ? (e & (L - 1)) : (e >> logF);
        if (e < FL) {
            if (MODE == 2) {
                // half spectrum: k <= L/2 given, L - k filled with the conjugate
                if (k < len_in) {
                    X[pd(f * L + k)] = buf[q];
                    if (k > 0 && k < (L >> 1)) X[pd(f * L + (L - k))] = make_float2(buf[q].x, -buf[q].y);
                }
            } else {
                X[pd(f * L + k)] = buf[q];
            }
        }
    }
    __syncthreads();
    fft_lds(X, tw, F, logL, MODE == 1 || MODE == 2);
    if (MODE == 3) {
        if (a.r2p <= 16) times_chat<4>(X, L, nf, a.Hs, o, u3s, a.r2p);
        else if (a.r2p <= 32) times_chat<8>(X, L, nf, a.Hs, o, u3s, a.r2p);
        else times_chat<12>(X, L, nf, a.Hs, o, u3s, a.r2p);
        __syncthreads();
        fft_lds(X, tw, F, logL, true);
    }
    // ---- store the first len_out entries of each fibre
    const int len_out = a.len_out;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        const int e = tid + NT * q;
        const int f = CONTIG ? (e >> logL) : (e & (F - 1));
        const int k = CONTIG ? (e & (L - 1)) : (e >> logF);
        if (e < FL && f < nf && k < len_out) {
            const float2 v = X[pd(f * L + k)];
            const long idx = CONTIG ? o * a.s_out_o + (long)(i0 + f) * a.s_out_i + k
                                    : o * a.s_out_o + (i0 + f) + (long)k * a.s_out_k;
            if (MODE == 2) static_cast<float*>(a.out)[idx] = v.x * a.scale;
            else static_cast<float2*>(a.out)[idx] = make_float2(v.x * a.scale, v.y * a.scale);
        }
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

size_t fft_lds_bytes(int L, int F, int r2p)
{
    const size_t fl = (size_t)F * L;
    // twiddles, the data (padded), and F * r2p floats of Uh3 rows for the P3 pass
    return sizeof(float2) * ((size_t)L + fl + (fl >> 4)) + sizeof(float) * (size_t)F * r2p;
}

int fft_fibres_per_block(int L, int r2p)
{
    int F = FFT_LDS_COMPLEX / L;
    if (F > FFT_THREADS) F = FFT_THREADS;
    if (F < 1) F = 1;
    while (F > 1 && fft_lds_bytes(L, F, r2p) > FFT_LDS_MAX) F >>= 1;
    return F;
}

namespace {
template <int MODE, bool IN_REAL, bool CONTIG>
hipError_t launch_pass_t(const FftPassArgs& a, long n_outer, size_t lds, hipStream_t s)
{
    dim3 grid((unsigned)((a.n_inner + a.F - 1) / a.F), (unsigned)n_outer);
    hipLaunchKernelGGL((k_fft_pass<MODE, IN_REAL, CONTIG>), grid, dim3(FFT_THREADS), lds, s, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fft_pass(const FftPassArgs& a, long n_outer, hipStream_t s)
{
    if (a.L < 2 || (1 << a.logL) != a.L || a.F < 1 || (1 << a.logF) != a.F || a.F * a.L > FFT_LDS_COMPLEX ||
        a.F > FFT_THREADS || n_outer < 1 || a.n_inner < 1 || a.len_in > a.L || a.len_out > a.L)
        return hipErrorInvalidValue;
    const bool contig_in = a.s_in_k == 1, contig_out = a.s_out_k == 1;
    if (contig_in != contig_out || (!contig_in && (a.s_in_i != 1 || a.s_out_i != 1))) return hipErrorInvalidValue;
    if (a.mode == 3 && (a.r2p < 4 || (a.r2p & 3) || a.r2p > 48)) return hipErrorInvalidValue;
    if (a.mode == 2 && a.len_in != a.L / 2 + 1) return hipErrorInvalidValue;
    const size_t lds = fft_lds_bytes(a.L, a.F, a.mode == 3 ? a.r2p : 0);
    if (lds > FFT_LDS_MAX) return hipErrorInvalidValue;
    if (a.mode == 0 && a.in_real && contig_in) return launch_pass_t<0, true, true>(a, n_outer, lds, s);
    if (a.mode == 0 && !a.in_real && !contig_in) return launch_pass_t<0, false, false>(a, n_outer, lds, s);
    if (a.mode == 1 && !a.in_real && !contig_in) return launch_pass_t<1, false, false>(a, n_outer, lds, s);
    if (a.mode == 2 && !a.in_real && contig_in) return launch_pass_t<2, false, true>(a, n_outer, lds, s);
    if (a.mode == 3 && !a.in_real && !contig_in) return launch_pass_t<3, false, false>(a, n_outer, lds, s);
    return hipErrorInvalidValue;
}

// Y[i][c] = c < cols ? (float)X[i * cols + c] : 0 for c < cols_pad.
__global__ void k_f64_to_f32_padded(const double* __restrict__ X, long rows, int cols, int cols_pad,
                                    float* __restrict__ Y)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols_pad) return;
    const long i = e / cols_pad;
    const int c = (int)(e - i * cols_pad);
    Y[e] = (c < cols) ? (float)X[i * cols + c] : 0.f;
}

hipError_t launch_f64_to_f32_padded(const double* X, long rows, int cols, int cols_pad, float* Y, hipStream_t s)
{
    const long tot = rows * cols_pad;
    hipLaunchKernelGGL(k_f64_to_f32_padded, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, rows, cols,
                       cols_pad, Y);
    return hipGetLastError();
}

// X[i][c] = 0 for cols <= c < cols_pad (rows of length cols_pad).
__global__ void k_zero_pad_cols(float* __restrict__ X, long rows, int cols, int cols_pad)
{
    const int w = cols_pad - cols;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * w) return;
    const long i = e / w;
    X[i * cols_pad + cols + (int)(e - i * w)] = 0.f;
}

hipError_t launch_zero_pad_cols(float* X, long rows, int cols, int cols_pad, hipStream_t s)
{
    if (cols_pad <= cols) return hipSuccess;
    const long tot = rows * (cols_pad - cols);
    hipLaunchKernelGGL(k_zero_pad_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, rows, cols,
                       cols_pad);
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
    const void* ks[] = {(const void*)k_fft_pass<0, true, true>, (const void*)k_fft_pass<0, false, false>,
                        (const void*)k_fft_pass<1, false, false>, (const void*)k_fft_pass<2, false, true>,
                        (const void*)k_fft_pass<3, false, false>};
    for (const void* k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FFT_LDS_MAX);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tk
