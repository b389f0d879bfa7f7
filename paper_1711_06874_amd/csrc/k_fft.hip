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
//   P5  axis 2, inverse from the half spectrum (Hermitian), real part, keeps i2 < m2, 1/(L0 L1 L2);
//       for the quadratic form z^T C z it also sums z . y as y is stored (z fetched with the input)
// with H2 = L2/2 + 1.  chat is evaluated on the fly in P3 from Hs[f0][f1][c] = sum_ab
// G_abc Uh1[f0][a] Uh2[f1][b] and Uh3.
//
// Each fibre is transformed by P = L / V lanes of one wavefront holding V values each (V = 8
// for 8 <= L <= 512, L / 64 above, L below 8), FW = 64 / P fibres per wavefront.  Lane p keeps
// the natural-order values X[p + P v] (v < V) in registers.  The FFT is a Stockham autosort
// of radix-8 stages (then 4 or 2): in stage s (Ns = 8^s) butterfly j = p + P b, b < V / R,
// takes the natural slots b + (V / R) r, multiplies by exp(-/+ 2 pi i (j mod Ns) r / (Ns R))
// and writes output r to position (j / Ns) Ns R + (j mod Ns) + r Ns.  The first stage thus reads
// the natural order straight from registers and the last one leaves it there; the stages in
// between exchange through the fibre's own LDS buffer with wavefront-level ordering only.
// Because m <= L / 2 for every axis of the embedding, forward transforms see zeros in the upper
// half and inverse transforms need only the lower half: both are pruned at compile time (the
// first radix-8 stage of a forward transform skips the additions of its four zero inputs).
//
// Passes with contiguous fibres (P1, P5) load and store the registers directly (coalesced
// along the fibre).  Strided passes (P2, P3, P4) stage a tile of F neighbouring fibres
// (F x 8 bytes per row) through LDS, read and written across fibres.  The transform length
// is a template parameter (2 <= L <= 2048), so all index arithmetic is compile-time.
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr int FFT_MAX_LOGL = 11;

// widest padded Uh3 row of the P3 pass is 48 floats
template <int LOGL>
struct Shape {
    static constexpr int L = 1 << LOGL;
    static constexpr int V = (L < 8) ? L : (L <= 512 ? 8 : L / 64);   // values per lane
    static constexpr int P = L / V;                                    // lanes per fibre
    static constexpr int FW = 64 / P;                                  // fibres per wavefront
    static constexpr int NW = (L <= 512) ? 16 : 8192 / L;              // wavefronts per work-group
    static constexpr int NT = 64 * NW;
    static constexpr int F = NW * FW;                                  // fibres per work-group
    static constexpr int LB = L + L / 8 + 1;                           // LDS stride between fibre buffers
    static constexpr int CS = (L + 15) / 16 * 16 + 4;                 // row stride of the multiplier table
    static constexpr int NS = (LOGL + 2) / 3;                          // stages
    static constexpr int QT = F * L / NT;                              // tile elements per thread
    // LDS of the P3 pass: the tile, the spectral multipliers and (when it fits) the Uh3 rows
    static constexpr size_t LDS_TILE = sizeof(float2) * (size_t)F * LB;
    static constexpr bool STAGE_U3 = LDS_TILE + sizeof(float) * (size_t)F * (CS + 48) <= 150 * 1024;
    static constexpr size_t LDS_CORE = LDS_TILE + sizeof(float) * (size_t)F * (CS + (STAGE_U3 ? 48 : 0));
    // the other passes keep the L twiddles in LDS after the tile (P3 holds its own in registers)
    static constexpr size_t LDS_PASS = LDS_TILE + sizeof(float2) * (size_t)L;
};

// log2 of the radix of stage s: 3 while at least 3 bits remain, then the rest
__host__ __device__ constexpr int stage_lr(int logl, int s) { return (logl - 3 * s >= 3) ? 3 : logl - 3 * s; }

// twiddles a lane needs in stages 1..S-1: sum over those stages of (V / R) (R - 1)
template <int LOGL>
__host__ __device__ constexpr int tw_offset(int S)
{
    int n = 0;
    for (int s = 1; s < S; ++s) {
        const int R = 1 << stage_lr(LOGL, s);
        n += (Shape<LOGL>::V / R) * (R - 1);
    }
    return n;
}
// In the P3 pass (two transforms per fibre, occupancy already set by its LDS) a lane keeps its
// twiddles in registers when there are at most 16 of them; the other passes load them per use.
template <int LOGL, bool WANT>
struct TwRegs {
    static constexpr int N = tw_offset<LOGL>(Shape<LOGL>::NS);
    static constexpr bool IN_REGS = WANT && N <= 16;
    float2 w[IN_REGS && N > 0 ? N : 1];
};

// LDS position of element k of a fibre buffer: one spare slot per 8 values
__device__ __forceinline__ int pos(int k) { return k + (k >> 3); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 cmul_mi(float2 a) { return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R])
{
    if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const float2 t2 = cadd(v[1], v[3]), t3 = cmul_mi<INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else {
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        dft<4, INV>(e);
        dft<4, INV>(o);
        const float h = 0.70710678118654752f;
        // o[k] *= exp(-/+ i pi k / 4)
        o[1] = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                   : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        o[2] = cmul_mi<INV>(o[2]);
        o[3] = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                   : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
}

// dft<8> of v[0..3] with v[4..7] = 0 (the first stage of a zero-padded forward transform):
// the additions with the zero inputs are left out.
template <bool INV>
__device__ __forceinline__ void dft8_half(float2 (&v)[8])
{
    const float2 e0 = cadd(v[0], v[2]), e2 = csub(v[0], v[2]);
    const float2 e1 = cadd(v[0], cmul_mi<INV>(v[2])), e3 = csub(v[0], cmul_mi<INV>(v[2]));
    float2 o0 = cadd(v[1], v[3]), o2 = csub(v[1], v[3]);
    float2 o1 = cadd(v[1], cmul_mi<INV>(v[3])), o3 = csub(v[1], cmul_mi<INV>(v[3]));
    const float h = 0.70710678118654752f;
    o1 = INV ? make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y)) : make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
    o2 = cmul_mi<INV>(o2);
    o3 = INV ? make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y)) : make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <int LOGL, int S, bool TWR>
__device__ __forceinline__ void load_twiddles_from(TwRegs<LOGL, TWR>& tr, int p, const float2* __restrict__ tw)
{
    if constexpr (S < Shape<LOGL>::NS) {
        constexpr int LR = stage_lr(LOGL, S), R = 1 << LR, B = Shape<LOGL>::V / R;
        constexpr int LNS = 3 * S, TWS = LOGL - LNS - LR;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = (p + Shape<LOGL>::P * b) & ((1 << LNS) - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) tr.w[tw_offset<LOGL>(S) + b * (R - 1) + (r - 1)] = tw[(k * r) << TWS];
        }
        load_twiddles_from<LOGL, S + 1, TWR>(tr, p, tw);
    }
}

// Stage S of the transform of the fibre whose buffer is fb, lane p of the fibre.
template <int LOGL, int S, bool INV, bool HALF_IN, bool TWR>
__device__ __forceinline__ void fft_stage(float2 (&x)[Shape<LOGL>::V], float2* fb, int p,
                                          const float2* __restrict__ tw, const TwRegs<LOGL, TWR>& tr)
{
    using Sh = Shape<LOGL>;
    constexpr int V = Sh::V, P = Sh::P;
    constexpr int LR = stage_lr(LOGL, S), R = 1 << LR, B = V / R;
    constexpr int LNS = 3 * S, NSZ = 1 << LNS;
    constexpr bool LAST = (S == Sh::NS - 1);
    constexpr int TWS = LOGL - LNS - LR;        // twiddle index step: L / (Ns R) = 2^TWS
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = p + P * b;
        const int k = j & (NSZ - 1);
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // stage 0 of a forward transform of zero-padded data: the upper half is zero
            if (HALF_IN && S == 0 && (b + B * r) >= V / 2) {
                u[r] = make_float2(0.f, 0.f);
                continue;
            }
            float2 v = x[b + B * r];
            if (S > 0 && r > 0) {
                float2 w;
                if constexpr (TwRegs<LOGL, TWR>::IN_REGS) w = tr.w[tw_offset<LOGL>(S) + b * (R - 1) + (r - 1)];
                else w = tw[(k * r) << TWS];
                if (INV) w.y = -w.y;
                v = cmul(v, w);
            }
            u[r] = v;
        }
        if constexpr (HALF_IN && S == 0 && R == 8) dft8_half<INV>(u);
        else dft<R, INV>(u);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[b + B * r] = u[r];
        } else {
            const int base = ((j >> LNS) << (LNS + LR)) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) fb[pos(base + r * NSZ)] = u[r];
        }
    }
    if (!LAST) {
        wave_sync();
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = fb[pos(p + P * v)];
        wave_sync();
    }
}

template <int LOGL, int S, bool INV, bool HALF_IN, bool TWR>
__device__ __forceinline__ void fft_stages(float2 (&x)[Shape<LOGL>::V], float2* fb, int p,
                                           const float2* __restrict__ tw, const TwRegs<LOGL, TWR>& tr)
{
    if constexpr (S < Shape<LOGL>::NS) {
        fft_stage<LOGL, S, INV, HALF_IN, TWR>(x, fb, p, tw, tr);
        fft_stages<LOGL, S + 1, INV, HALF_IN, TWR>(x, fb, p, tw, tr);
    }
}

// The twiddles exp(-2 pi i (j mod Ns) r / (Ns R)) of lane p in stages 1.. (forward sign).
template <int LOGL, bool TWR>
__device__ __forceinline__ void load_twiddles(TwRegs<LOGL, TWR>& tr, int p, const float2* __restrict__ tw)
{
    if constexpr (TwRegs<LOGL, TWR>::IN_REGS && TwRegs<LOGL, TWR>::N > 0) {
        load_twiddles_from<LOGL, 1, TWR>(tr, p, tw);
    }
}

// ct[ff][f0] (row stride CS) = chat[f0][o][i0 + ff] = sum_c Uh3[i0 + ff][c] Hs[o][f0][c] for the F
// fibres of the work-group: an (F x r2p) x (r2p x L) product on mfma_f32_16x16x4f32, 16 x 16
// output tiles shared out over the wavefronts (operand A: row lane % 16; B: column lane % 16;
// result v of a lane: row 4 (lane / 16) + v, column lane % 16).  The sum over c runs in groups
// of 16: lane group q = lane / 16 loads c = 16 g + 4 q .. + 3 of its row as one float4 and
// MFMA j of the group takes the j-th of them, so every operand of a tile is loaded by
// 16-byte loads issued together before the products.  The Uh3 rows of the work-group are
// staged in LDS (u3s, F x r2p) when they fit.
template <int LOGL>
__device__ __forceinline__ void chat_table(float* ct, float* u3s, long o, int i0, int nf, int r2p,
                                           const float* __restrict__ Hs, const float* __restrict__ Uh3)
{
    using Sh = Shape<LOGL>;
    constexpr int L = Sh::L, NT = Sh::NT, F = Sh::F, NW = Sh::NW, CS = Sh::CS;
    constexpr int TR = (F + 15) / 16, TC = (L + 15) / 16;
    constexpr int NG = 48 / 16;                 // groups of 16 in the widest row (r2p <= 48)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if constexpr (Sh::STAGE_U3) {
        for (int e = tid; e < F * r2p; e += NT) u3s[e] = (e < nf * r2p) ? Uh3[(long)i0 * r2p + e] : 0.f;
        __syncthreads();
    }
    const int lr = lane & 15, lq = lane >> 4;
    for (int t = wv; t < TR * TC; t += NW) {
        const int tr = t % TR, tc = t / TR;
        const int ff = 16 * tr + lr, f0 = 16 * tc + lr;
        const float* urow = Sh::STAGE_U3 ? u3s + (ff < F ? ff : 0) * r2p
                                         : Uh3 + (long)((ff < nf) ? i0 + ff : i0) * r2p;
        const float* hrow = Hs + ((long)o * L + (f0 < L ? f0 : 0)) * r2p;
        float4 av[NG], bv[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int c = 16 * g + 4 * lq;
            av[g] = (c < r2p && ff < F) ? *reinterpret_cast<const float4*>(urow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
            bv[g] = (c < r2p && f0 < L) ? *reinterpret_cast<const float4*>(hrow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (16 * g < r2p) {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].x, bv[g].x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].y, bv[g].y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].z, bv[g].z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].w, bv[g].w, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * tr + 4 * lq + v;
            if (row < F && f0 < L) ct[row * CS + f0] = acc[v];
        }
    }
}

// The same table when the Uh3 rows sit in LDS already (u3s, staged with the chunk's tile), in two
// steps so that the Hs operands can be requested before the barrier that publishes u3s:
// chat_hs_load issues this wavefront's Hs loads (its tiles t = wv, wv + NW, ...), chat_products
// takes the Uh3 operands from u3s and writes ct.  Same products in the same order as chat_table.
template <int LOGL>
struct ChatRegs {
    static constexpr int TPW = ((Shape<LOGL>::F + 15) / 16 * ((Shape<LOGL>::L + 15) / 16) + Shape<LOGL>::NW - 1) /
                               Shape<LOGL>::NW;    // tiles per wavefront
    float4 bv[TPW][3];
};

template <int LOGL>
__device__ __forceinline__ void chat_hs_load(ChatRegs<LOGL>& cr, long o, int r2p, const float* __restrict__ Hs)
{
    using Sh = Shape<LOGL>;
    constexpr int L = Sh::L, F = Sh::F, NW = Sh::NW;
    constexpr int TR = (F + 15) / 16, TC = (L + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int u = 0; u < ChatRegs<LOGL>::TPW; ++u) {
        const int t = wv + NW * u;
        const int tc = t / TR;
        const int f0 = 16 * tc + lr;
        const bool live = t < TR * TC && f0 < L;
        const float* hrow = Hs + ((long)o * L + (live ? f0 : 0)) * r2p;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const int c = 16 * g + 4 * lq;
            cr.bv[u][g] = (live && c < r2p) ? *reinterpret_cast<const float4*>(hrow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

template <int LOGL>
__device__ __forceinline__ void chat_products(float* ct, const float* u3s, const ChatRegs<LOGL>& cr, int r2p)
{
    using Sh = Shape<LOGL>;
    constexpr int L = Sh::L, F = Sh::F, NW = Sh::NW, CS = Sh::CS;
    constexpr int TR = (F + 15) / 16, TC = (L + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int u = 0; u < ChatRegs<LOGL>::TPW; ++u) {
        const int t = wv + NW * u;
        if (t >= TR * TC) break;
        const int tr = t % TR, tc = t / TR;
        const int ff = 16 * tr + lr, f0 = 16 * tc + lr;
        const float* urow = u3s + (ff < F ? ff : 0) * r2p;
        float4 av[3];
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const int c = 16 * g + 4 * lq;
            av[g] = (c < r2p && ff < F) ? *reinterpret_cast<const float4*>(urow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            if (16 * g < r2p) {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].x, cr.bv[u][g].x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].y, cr.bv[u][g].y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].z, cr.bv[u][g].z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].w, cr.bv[u][g].w, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * tr + 4 * lq + v;
            if (row < F && f0 < L) ct[row * CS + f0] = acc[v];
        }
    }
}

// Pass kinds
enum { PK_R2C = 0, PK_FWD = 1, PK_CORE = 2, PK_INV = 3, PK_C2R = 4 };

// Chunk c of a pass: F fibres (i0 = (c mod nbx) F, ...) of outer index o = c / nbx.  In the P3
// pass the work-groups of one XCD (work-group ids are dealt to the 8 XCDs in turn) walk the
// outer planes o = xcd (mod 8), so that each plane's transformed core is read into one L2.
struct Chunk {
    long o;
    int i0;
};

template <int F>
__device__ __forceinline__ bool chunk_at(long j, int nbx, long n_outer, bool xcd_planes, Chunk* ch)
{
    const long G = gridDim.x;
    long c;
    if (xcd_planes) {
        const long x = blockIdx.x & 7, slot = blockIdx.x >> 3, nslot = G >> 3;
        const long q = slot + j * nslot;                       // index within the XCD's planes
        const long plane = (q / nbx) * 8 + x;
        if (plane >= n_outer) return false;
        c = plane * nbx + q % nbx;
    } else {
        c = blockIdx.x + j * G;
        if (c >= (long)nbx * n_outer) return false;
    }
    ch->o = c / nbx;
    ch->i0 = (int)(c % nbx) * F;
    return true;
}

template <int LOGL, int PK>
__global__ void __launch_bounds__(Shape<LOGL>::NT) k_fft_pass(FftPassArgs a)
{
    using Sh = Shape<LOGL>;
    constexpr int L = Sh::L, V = Sh::V, P = Sh::P, F = Sh::F, NT = Sh::NT, LB = Sh::LB;
    constexpr bool CONTIG = (PK == PK_R2C || PK == PK_C2R);
    extern __shared__ __attribute__((aligned(16))) float2 fsm[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int q = lane / P, p = lane - q * P;          // fibre within the wavefront, lane within the fibre
    const int f = wv * Sh::FW + q;                     // fibre within the chunk
    // contiguous passes pair the rows: n_inner rows make (n_inner + 1) / 2 fibres
    const int nfib = CONTIG ? (a.n_inner + 1) / 2 : a.n_inner;
    const int nbx = (nfib + F - 1) / F;
    const bool xcd_planes = (PK == PK_CORE) && (a.n_outer % 8 == 0) && (gridDim.x % 8 == 0);
    float2* fb = fsm + f * LB;
    TwRegs<LOGL, PK == PK_CORE> tr;
    load_twiddles<LOGL, PK == PK_CORE>(tr, p, a.tw);
    // passes other than P3 read their twiddles from an LDS copy of the table (written before the
    // first barrier of the chunk loop; contiguous passes, which have none before their first
    // transform, wait here); P3 keeps them in registers, or reads the global table for long L
    const float2* twp = a.tw;
    if constexpr (PK != PK_CORE) {
        float2* tws = fsm + (size_t)F * LB;
        for (int qq = tid; qq < L; qq += NT) tws[qq] = a.tw[qq];
        if constexpr (CONTIG) __syncthreads();
        twp = tws;
    }

    // ---- loads of one chunk into registers: rows of the pair (contiguous) or the tile (strided)
    constexpr int KIN = (PK == PK_INV) ? L : L / 2;    // forward passes: only the lower half is non-zero
    constexpr int VIN = (PK == PK_INV) ? V : V / 2;
    constexpr int NREG = CONTIG ? V : Sh::QT;
    float2 pre[NREG];
    // mode 2 with dot_part: the z values of the next chunk's outputs (rows ra, rb), fetched with it
    constexpr int VZ = (PK == PK_C2R) ? V / 2 : 1;
    float zpa[VZ], zpb[VZ];
    // P3 with staged Uh3 rows (when at most two multiplier tiles fall to a wavefront): the next
    // chunk's rows (F x r2p, r2p <= 48), fetched with its tile
    constexpr bool STAGED = (PK == PK_CORE) && Sh::STAGE_U3 && ChatRegs<LOGL>::TPW <= 2;
    constexpr int UPT = STAGED ? (F * 48 + NT - 1) / NT : 1;
    float upre[UPT];
    auto fetch = [&](const Chunk& ch) {
        const int nf = (nfib - ch.i0 < F) ? (nfib - ch.i0) : F;
        if constexpr (STAGED) {
#pragma unroll
            for (int j = 0; j < UPT; ++j) {
                const int e = tid + NT * j;
                upre[j] = (e < nf * a.r2p) ? a.Uh3[(long)ch.i0 * a.r2p + e] : 0.f;
            }
        }
        if constexpr (CONTIG) {
            const long ra = 2L * (ch.i0 + f), rb = ra + 1;
            const bool la = f < nf && ra < a.n_inner, lb = f < nf && rb < a.n_inner;
            if constexpr (PK == PK_C2R) {
                if (a.dot_part) {
                    const float* zz = a.dot_z + ch.o * a.s_out_o;
#pragma unroll
                    for (int v = 0; v < VZ; ++v) {
                        const int k = p + P * v;
                        zpa[v] = (la && k < a.len_out) ? zz[ra * a.s_out_i + k] : 0.f;
                        zpb[v] = (lb && k < a.len_out) ? zz[rb * a.s_out_i + k] : 0.f;
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k = p + P * v;
                pre[v] = make_float2(0.f, 0.f);
                if constexpr (PK == PK_R2C) {
                    const float* in = static_cast<const float*>(a.in) + ch.o * a.s_in_o;
                    if (v < V / 2 && k < a.len_in) {
                        if (la) pre[v].x = in[ra * a.s_in_i + k];
                        if (lb) pre[v].y = in[rb * a.s_in_i + k];
                    }
                } else {
                    // half spectra k <= L / 2 given; above it the conjugate of L - k.  Z = Xa + i Xb.
                    const float2* in = static_cast<const float2*>(a.in) + ch.o * a.s_in_o;
                    const int kk = (k <= L / 2) ? k : L - k;
                    const float sg = (k <= L / 2) ? 1.f : -1.f;
                    float2 xa = make_float2(0.f, 0.f), xb = make_float2(0.f, 0.f);
                    if (la) xa = in[ra * a.s_in_i + kk];
                    if (lb) xb = in[rb * a.s_in_i + kk];
                    pre[v] = make_float2(xa.x - sg * xb.y, sg * xa.y + xb.x);
                }
            }
        } else {
            const float2* in = static_cast<const float2*>(a.in);
            const long base = ch.o * a.s_in_o + ch.i0;
#pragma unroll
            for (int t = 0; t < Sh::QT; ++t) {
                const int e = tid + NT * t;
                const int ff = e & (F - 1), k = e / F;
                pre[t] = make_float2(0.f, 0.f);
                if (k < KIN && ff < nf && k < a.len_in) pre[t] = in[base + ff + (long)k * a.s_in_k];
            }
        }
    };

    double dsum = 0.0;                                 // mode 2 with dot_part: z . y over this block's outputs
    Chunk ch;
    if (!chunk_at<F>(0, nbx, a.n_outer, xcd_planes, &ch)) {
        if (PK == PK_C2R && a.dot_part && tid == 0) a.dot_part[blockIdx.x] = 0.0;
        return;
    }
    fetch(ch);
    for (long j = 0;; ++j) {
        const Chunk cur = ch;
        const int i0 = cur.i0;
        const long o = cur.o;
        const int nf = (nfib - i0 < F) ? (nfib - i0) : F;
        float2 x[V];
        float zca[VZ], zcb[VZ];
        bool more;
        if constexpr (CONTIG) {
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = pre[v];
            if constexpr (PK == PK_C2R) {
#pragma unroll
                for (int v = 0; v < VZ; ++v) {
                    zca[v] = zpa[v];
                    zcb[v] = zpb[v];
                }
            }
            // the next chunk's loads are in flight while this one is transformed
            more = chunk_at<F>(j + 1, nbx, a.n_outer, xcd_planes, &ch);
            if (more) fetch(ch);
        } else {
            ChatRegs<LOGL> cr;
            // the Hs operands of this chunk's multiplier table are requested first; they arrive
            // while the tile and the Uh3 rows are written to LDS
            if constexpr (STAGED) chat_hs_load<LOGL>(cr, o, a.r2p, a.Hs);
            __syncthreads();          // the previous chunk has finished reading the tile
#pragma unroll
            for (int t = 0; t < Sh::QT; ++t) {
                const int e = tid + NT * t;
                const int ff = e & (F - 1), k = e / F;
                if (k < KIN) fsm[ff * LB + pos(k)] = pre[t];
            }
            float* const ctab = reinterpret_cast<float*>(fsm + F * LB);
            float* const u3s = ctab + F * Sh::CS;
            if constexpr (STAGED) {
#pragma unroll
                for (int jj = 0; jj < UPT; ++jj) {
                    const int e = tid + NT * jj;
                    if (e < F * 48) u3s[e] = upre[jj];
                }
            }
            // the next chunk's loads are in flight while this one is transformed
            more = chunk_at<F>(j + 1, nbx, a.n_outer, xcd_planes, &ch);
            if (more) fetch(ch);
            if constexpr (STAGED) {
                __syncthreads();      // tile and Uh3 rows published
                chat_products<LOGL>(ctab, u3s, cr, a.r2p);
            } else if constexpr (PK == PK_CORE) {
                chat_table<LOGL>(ctab, u3s, o, i0, nf, a.r2p, a.Hs, a.Uh3);
            }
            __syncthreads();
#pragma unroll
            for (int v = 0; v < VIN; ++v) x[v] = fb[pos(p + P * v)];
#pragma unroll
            for (int v = VIN; v < V; ++v) x[v] = make_float2(0.f, 0.f);
        }

        // ------------------------------------------------------------ transform(s)
        if constexpr (PK == PK_R2C || PK == PK_FWD) {
            fft_stages<LOGL, 0, false, true>(x, fb, p, twp, tr);
        } else if constexpr (PK == PK_CORE) {
            fft_stages<LOGL, 0, false, true>(x, fb, p, twp, tr);
            const float* ct = reinterpret_cast<const float*>(fsm + F * LB) + f * Sh::CS;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float c = ct[p + P * v];
                x[v] = make_float2(x[v].x * c, x[v].y * c);
            }
            fft_stages<LOGL, 0, true, false>(x, fb, p, twp, tr);
        } else {
            fft_stages<LOGL, 0, true, false>(x, fb, p, twp, tr);
        }

        // ------------------------------------------------------------ store
        if constexpr (CONTIG) {
            const long ra = 2L * (i0 + f), rb = ra + 1;
            const bool la = f < nf && ra < a.n_inner, lb = f < nf && rb < a.n_inner;
            if constexpr (PK == PK_R2C) {
                // Xa[k] = (Z[k] + conj Z[L-k]) / 2, Xb[k] = (Z[k] - conj Z[L-k]) / (2i), k <= L / 2
#pragma unroll
                for (int v = 0; v < V; ++v) fb[pos(p + P * v)] = x[v];
                wave_sync();
                float2* out = static_cast<float2*>(a.out) + o * a.s_out_o;
#pragma unroll
                for (int v = 0; v <= V / 2 && v < V; ++v) {
                    const int k = p + P * v;
                    if (k <= L / 2 && k < a.len_out) {
                        const float2 zm = fb[pos((L - k) & (L - 1))];
                        const float2 z = x[v];
                        if (la) out[ra * a.s_out_i + k] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
                        if (lb) out[rb * a.s_out_i + k] = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
                    }
                }
                wave_sync();          // the buffer is rewritten by the next chunk's first stage
            } else {
                float* out = static_cast<float*>(a.out) + o * a.s_out_o;
#pragma unroll
                for (int v = 0; v < V / 2; ++v) {
                    const int k = p + P * v;
                    if (k < a.len_out) {
                        const float ya = x[v].x * a.scale, yb = x[v].y * a.scale;
                        if (!a.no_store) {
                            if (la) out[ra * a.s_out_i + k] = ya;
                            if (lb) out[rb * a.s_out_i + k] = yb;
                        }
                        if (a.dot_part) {
                            if (la) dsum += (double)ya * (double)zca[v];
                            if (lb) dsum += (double)yb * (double)zcb[v];
                        }
                    }
                }
            }
        } else {
            // forward passes keep all L outputs; inverse ones the lower half
            constexpr int VOUT = (PK == PK_FWD) ? V : V / 2;
            constexpr int KOUT = (PK == PK_FWD) ? L : L / 2;
#pragma unroll
            for (int v = 0; v < VOUT; ++v) fb[pos(p + P * v)] = x[v];
            __syncthreads();
            float2* out = static_cast<float2*>(a.out);
            const long base = o * a.s_out_o + i0;
#pragma unroll
            for (int t = 0; t < Sh::QT; ++t) {
                const int e = tid + NT * t;
                const int ff = e & (F - 1), k = e / F;
                if (k < KOUT && ff < nf && k < a.len_out) {
                    const float2 v = fsm[ff * LB + pos(k)];
                    out[base + ff + (long)k * a.s_out_k] = make_float2(v.x * a.scale, v.y * a.scale);
                }
            }
        }
        if (!more) break;
    }
    if constexpr (PK == PK_C2R) {
        if (a.dot_part) {
            // fixed-order reduction: each wavefront by butterflies, then the wavefronts in order
            __syncthreads();
            double* red = reinterpret_cast<double*>(fsm);
            dsum = wave_sum(dsum);
            if (lane == 0) red[wv] = dsum;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
                for (int w = 0; w < Sh::NW; ++w) t += red[w];
                a.dot_part[blockIdx.x] = t;
            }
        }
    }
}

}  // namespace

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
// (U: n x r row-major FP64; output nf x r FP64), for the three axes in one launch (grid y).
// cos(2 pi q / L) comes from a per-block FP64 table; the phase f t is reduced exactly modulo L
// (a power of two).  Eight lanes share one output, lane g summing t = 1 + g + 8 j in order
// (four loads issued together); the eight partial sums are combined by butterfly shuffles,
// which give every lane of the eight the same bits (each addition is commutative).
constexpr int FF_SEG = 8;
constexpr int FF_OUT = 256 / FF_SEG;          // outputs per work-group

__global__ void __launch_bounds__(256) k_fourier_factor(FourierAxes fa)
{
    extern __shared__ double ctab[];
    const FourierAxis& ax = fa.ax[blockIdx.y];
    const int r = ax.r, m = ax.m, L = ax.L;
    if ((long)blockIdx.x * FF_OUT >= (long)ax.nf * r) return;           // uniform over the block
    for (int q = threadIdx.x; q < L; q += blockDim.x) ctab[q] = cospi(2.0 * (double)q / (double)L);
    __syncthreads();
    const int g = threadIdx.x & (FF_SEG - 1);
    const long e = (long)blockIdx.x * FF_OUT + (threadIdx.x / FF_SEG);
    const bool live = e < (long)ax.nf * r;
    const long ee = live ? e : 0;
    const int f = (int)(ee / r), a = (int)(ee % r);
    const double* u = ax.U + (long)ax.off * r + a;
    double s = 0.0;
    int t = 1 + g;
    for (; t + 3 * FF_SEG < m; t += 4 * FF_SEG) {
        const double u0 = u[(long)t * r], u1 = u[(long)(t + FF_SEG) * r];
        const double u2 = u[(long)(t + 2 * FF_SEG) * r], u3 = u[(long)(t + 3 * FF_SEG) * r];
        s += u0 * ctab[(f * t) & (L - 1)];
        s += u1 * ctab[(f * (t + FF_SEG)) & (L - 1)];
        s += u2 * ctab[(f * (t + 2 * FF_SEG)) & (L - 1)];
        s += u3 * ctab[(f * (t + 3 * FF_SEG)) & (L - 1)];
    }
    for (; t < m; t += FF_SEG) s += u[(long)t * r] * ctab[(f * t) & (L - 1)];
#pragma unroll
    for (int d = 1; d < FF_SEG; d <<= 1) s += __shfl_xor(s, d, FF_SEG);
    if (live && g == 0) ax.Uh[e] = u[0] + 2.0 * s;
}

// Hs[f1][f0][c] = sum_b Uh1[f1][b] M1[f0][b][c] (FP64 sums stored as FP32) for c < r2, and 0 for
// r2 <= c < r2p: the Fourier-side core contracted with the axis-1 factor, one row of r2p values
// per (f1, f0).  A work-group owns 256 / r2p consecutive f0 and HS_F1 consecutive f1; thread
// (f0, c) keeps M1[f0][:][c] in registers, the Uh1 rows of its f1 block sit in LDS, and each f1
// writes one contiguous run of the f0 block's rows.
constexpr int HS_F1 = 32;
constexpr int HS_RMAX = 48;

__global__ void __launch_bounds__(256) k_spectral_core(const double* __restrict__ Uh1, const double* __restrict__ M1,
                                                       int L0, int L1, int r1, int r2, int r2p, float* __restrict__ Hs)
{
    __shared__ double us[HS_F1][HS_RMAX];
    const int nf0 = 256 / r2p;
    const int c = threadIdx.x % r2p, fl = threadIdx.x / r2p;
    const int f0 = blockIdx.x * nf0 + fl;
    const int f1b = blockIdx.y * HS_F1;
    const bool row = fl < nf0 && f0 < L0;
    const bool live = row && c < r2;
    double mr[HS_RMAX];
#pragma unroll
    for (int b = 0; b < HS_RMAX; ++b) mr[b] = (live && b < r1) ? M1[((long)f0 * r1 + b) * r2 + c] : 0.0;
    for (int e = threadIdx.x; e < HS_F1 * r1; e += blockDim.x) {
        const int j = e / r1, b = e - j * r1;
        us[j][b] = (f1b + j < L1) ? Uh1[(long)(f1b + j) * r1 + b] : 0.0;
    }
    __syncthreads();
    if (!row) return;
    const int nj = (L1 - f1b < HS_F1) ? (L1 - f1b) : HS_F1;
    for (int j = 0; j < nj; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < HS_RMAX; ++b)
            if (b < r1) acc += us[j][b] * mr[b];
        Hs[((long)(f1b + j) * L0 + f0) * r2p + c] = live ? (float)acc : 0.f;
    }
}

hipError_t launch_spectral_core(const double* Uh1, const double* M1, int L0, int L1, int r1, int r2, int r2p,
                                float* Hs, hipStream_t s)
{
    if (r1 < 1 || r1 > HS_RMAX || r2 < 1 || r2p < r2 || r2p > 256 || L0 < 1 || L1 < 1) return hipErrorInvalidValue;
    const int nf0 = 256 / r2p;
    const dim3 grid((unsigned)((L0 + nf0 - 1) / nf0), (unsigned)((L1 + HS_F1 - 1) / HS_F1));
    hipLaunchKernelGGL(k_spectral_core, grid, dim3(256), 0, s, Uh1, M1, L0, L1, r1, r2, r2p, Hs);
    return hipGetLastError();
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

hipError_t launch_fourier_factors(const FourierAxes& fa, hipStream_t s)
{
    long blocks = 1;
    int lmax = 2;
    for (int k = 0; k < 3; ++k) {
        const FourierAxis& x = fa.ax[k];
        if (!x.U || !x.Uh || x.r < 1 || x.m < 1 || x.nf < 1 || x.L < 2 || (x.L & (x.L - 1)) || x.L > 2048 || x.m > x.L ||
            (long)x.nf * x.L > (1L << 30))
            return hipErrorInvalidValue;
        blocks = std::max(blocks, ((long)x.nf * x.r + FF_OUT - 1) / FF_OUT);
        lmax = std::max(lmax, x.L);
    }
    hipLaunchKernelGGL(k_fourier_factor, dim3((unsigned)blocks, 3), dim3(256), sizeof(double) * lmax, s, fa);
    return hipGetLastError();
}

namespace {
// resident work-groups per CU of each pass (from the occupancy calculator) and the CU count,
// filled when the attributes are set; the passes run persistent grids of that size
int g_resident[FFT_MAX_LOGL + 1][5];
int g_cus = 0;

template <int LOGL>
hipError_t launch_len(FftPassArgs a, int kind, long n_outer, hipStream_t s, unsigned* blocks)
{
    using Sh = Shape<LOGL>;
    const int nfib = (kind == PK_R2C || kind == PK_C2R) ? (a.n_inner + 1) / 2 : a.n_inner;
    const long chunks = (long)((nfib + Sh::F - 1) / Sh::F) * n_outer;
    const int per_cu = g_resident[LOGL][kind] > 0 ? g_resident[LOGL][kind] : 1;
    long slots = (long)(g_cus > 0 ? g_cus : 256) * per_cu;
    if (a.dot_part && slots > a.dot_cap) slots = a.dot_cap;
    const dim3 grid((unsigned)(chunks < slots ? chunks : slots));
    if (blocks) *blocks = grid.x;
    a.n_outer = n_outer;
    const size_t lds = (kind == PK_CORE) ? Sh::LDS_CORE : Sh::LDS_PASS;
    switch (kind) {
    case PK_R2C: hipLaunchKernelGGL((k_fft_pass<LOGL, PK_R2C>), grid, dim3(Sh::NT), lds, s, a); break;
    case PK_FWD: hipLaunchKernelGGL((k_fft_pass<LOGL, PK_FWD>), grid, dim3(Sh::NT), lds, s, a); break;
    case PK_INV: hipLaunchKernelGGL((k_fft_pass<LOGL, PK_INV>), grid, dim3(Sh::NT), lds, s, a); break;
    case PK_C2R: hipLaunchKernelGGL((k_fft_pass<LOGL, PK_C2R>), grid, dim3(Sh::NT), lds, s, a); break;
    default: hipLaunchKernelGGL((k_fft_pass<LOGL, PK_CORE>), grid, dim3(Sh::NT), lds, s, a);
    }
    return hipGetLastError();
}

template <int LOGL>
hipError_t set_attrs_len()
{
    using Sh = Shape<LOGL>;
    const int lds = (int)Sh::LDS_PASS;
    const int lds_core = (int)Sh::LDS_CORE;
    const void* ks[] = {(const void*)k_fft_pass<LOGL, PK_R2C>, (const void*)k_fft_pass<LOGL, PK_FWD>,
                        (const void*)k_fft_pass<LOGL, PK_CORE>, (const void*)k_fft_pass<LOGL, PK_INV>,
                        (const void*)k_fft_pass<LOGL, PK_C2R>};
    for (int i = 0; i < 5; ++i) {
        const int bytes = (i == PK_CORE) ? lds_core : lds;
        hipError_t e = hipFuncSetAttribute(ks[i], hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
        int nb = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ks[i], Sh::NT, (size_t)bytes);
        if (e != hipSuccess) return e;
        g_resident[LOGL][i] = nb > 0 ? nb : 1;
    }
    return hipSuccess;
}

template <int LOGL>
hipError_t set_attrs_upto()
{
    hipError_t e = set_attrs_len<LOGL>();
    if constexpr (LOGL > 1) {
        if (e == hipSuccess) e = set_attrs_upto<LOGL - 1>();
    }
    return e;
}
}  // namespace

hipError_t launch_fft_pass(const FftPassArgs& a, long n_outer, hipStream_t s, unsigned* blocks)
{
    const int L = a.L;
    if (a.logL < 1 || a.logL > FFT_MAX_LOGL || L != (1 << a.logL) || n_outer < 1 || a.n_inner < 1 ||
        a.len_in < 1 || a.len_out < 1 || !a.in || !a.tw)
        return hipErrorInvalidValue;
    if (a.dot_part && (a.mode != 2 || !a.dot_z || a.dot_cap < 1)) return hipErrorInvalidValue;
    if (a.no_store ? (a.mode != 2 || !a.dot_part) : !a.out) return hipErrorInvalidValue;
    const bool contig = a.s_in_k == 1 && a.s_out_k == 1;
    const bool strided = a.s_in_i == 1 && a.s_out_i == 1 && !contig;
    int kind;
    if (a.mode == 0 && a.in_real && contig && a.len_in <= L / 2 && a.len_out <= L / 2 + 1) kind = PK_R2C;
    else if (a.mode == 0 && !a.in_real && strided && a.len_in <= L / 2 && a.len_out <= L) kind = PK_FWD;
    else if (a.mode == 3 && !a.in_real && strided && a.len_in <= L / 2 && a.len_out <= L / 2 && a.Hs && a.Uh3 &&
             a.r2p >= 4 && a.r2p <= 48 && (a.r2p & 3) == 0)
        kind = PK_CORE;
    else if (a.mode == 1 && !a.in_real && strided && a.len_in <= L && a.len_out <= L / 2) kind = PK_INV;
    else if (a.mode == 2 && !a.in_real && contig && a.len_in == L / 2 + 1 && a.len_out <= L / 2) kind = PK_C2R;
    else return hipErrorInvalidValue;
    switch (a.logL) {
    case 1: return launch_len<1>(a, kind, n_outer, s, blocks);
    case 2: return launch_len<2>(a, kind, n_outer, s, blocks);
    case 3: return launch_len<3>(a, kind, n_outer, s, blocks);
    case 4: return launch_len<4>(a, kind, n_outer, s, blocks);
    case 5: return launch_len<5>(a, kind, n_outer, s, blocks);
    case 6: return launch_len<6>(a, kind, n_outer, s, blocks);
    case 7: return launch_len<7>(a, kind, n_outer, s, blocks);
    case 8: return launch_len<8>(a, kind, n_outer, s, blocks);
    case 9: return launch_len<9>(a, kind, n_outer, s, blocks);
    case 10: return launch_len<10>(a, kind, n_outer, s, blocks);
    default: return launch_len<11>(a, kind, n_outer, s, blocks);
    }
}

hipError_t fft_set_attributes()
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    g_cus = cus;
    return set_attrs_upto<FFT_MAX_LOGL>();
}

}  // namespace tk
