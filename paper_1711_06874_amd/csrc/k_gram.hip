// a2: mode-k Gram matrices G_k = A_(k) A_(k)^T of the HOSVD (Sec. 3.2).
//
// X = A_(k) is n_k x K with K = N / n_k.  Element X[row][Kg] of each unfolding, for the
// C-order n0 x n1 x n2 tensor A:
//   mode 0: A[row*n1*n2 + Kg]                          (rows contiguous, "NT")
//   mode 1: A[(Kg/n2)*n1*n2 + row*n2 + Kg%n2]          (n2-long contiguous pieces)
//   mode 2: A[Kg*n2 + row]                             (columns contiguous, "TN")
// The n_k x n_k result is cut into 64 x 64 tiles; only tiles (ti <= tj) are computed.  The K
// range is split into S equal chunks; work-group (pair, split) accumulates its chunk on MFMA
// and writes a float (or double) 64 x 64 partial.  A second kernel adds the S partials of
// every entry in split order in FP64 and writes both G[i][j] and G[j][i] (diagonal tiles are
// mirrored from their upper half), so the result is deterministic and exactly symmetric.
//
// Large FP32 grids (every n_k a multiple of 32 and, by default, the mode's n_k >= 256; from 128
// on when the autotuner finds it faster) take k_gram_big:
// 128 x 128 tiles, each wave a 64 x 64 block (four independent 32 x 32 MFMA accumulators), K
// chunks of 32 loaded as float4 and staged in LDS, and the splits of K given to the XCDs so
// that all tile pairs of one split run on one XCD (its L2 holds the split's row panels once).
//
// Precision variants:
//   double : mfma_f64_16x16x4f64, FP64 accumulation and FP64 partials
//   float  : mfma_f32_32x32x2f32, FP32 accumulation
//   bf16x3 : float tiles split into bf16 (hi, lo); hi*hi + hi*lo + lo*hi on
//            mfma_f32_32x32x16_bf16 with FP32 accumulation
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr int BM = 64;      // output tile edge
constexpr int NT = 256;     // threads per work-group (4 waves, 2 x 2 of 32 x 32 blocks)

template <int MODE>
struct Unfold {
    long n1n2;
    int n1, n2;
    __device__ __forceinline__ long addr(int row, long Kg) const
    {
        if (MODE == 0) return (long)row * n1n2 + Kg;
        if (MODE == 1) { long i0 = Kg / n2; return i0 * n1n2 + (long)row * n2 + (Kg - i0 * n2); }
        return Kg * n2 + row;
    }
    __device__ __forceinline__ long rowstride() const { return MODE == 0 ? n1n2 : (long)n2; }
};

// Column cursor of modes 0 and 1, where every load of a thread reads one column Kg (rows vary)
// and Kg advances by BK per chunk: the column's base address without a division per chunk
// (mode 1: Kg = q n2 + r, base = q n1 n2 + r).
template <int MODE>
struct KCursor {
    long q;
    int r;
    __device__ __forceinline__ void init(const Unfold<MODE>& u, long Kg)
    {
        if (MODE == 1) { q = Kg / u.n2; r = (int)(Kg - q * u.n2); }
        else { q = Kg; r = 0; }
    }
    __device__ __forceinline__ long base(const Unfold<MODE>& u) const { return MODE == 1 ? q * u.n1n2 + r : q; }
    __device__ __forceinline__ void advance(const Unfold<MODE>& u, int step)
    {
        if (MODE == 1) {
            r += step;
            while (r >= u.n2) { r -= u.n2; ++q; }
        } else {
            q += step;
        }
    }
};

// Map a tile-pair index to (ti, tj) with ti <= tj, row-major over the upper triangle.
__device__ __forceinline__ void pair_of(int pidx, int T, int& ti, int& tj)
{
    int i = 0, base = 0;
    while (base + (T - i) <= pidx) { base += T - i; ++i; }
    ti = i;
    tj = i + (pidx - base);
}

// ----------------------------------------------------------------------------------------
// FP32 / FP64 tiles: LDS holds the chunk as [BK][BM + 1] (k-major), loaded with coalesced
// global reads (along K for modes 0/1, along rows for mode 2).
// ----------------------------------------------------------------------------------------
template <int MODE, typename T, int BK>
__global__ void __launch_bounds__(NT) k_gram_tiles(const T* __restrict__ A, Unfold<MODE> u, int nrow,
                                                   long K, long kchunk, int T_tiles, int nsplit,
                                                   T* __restrict__ partials, long bs)
{
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BM + 1];
    A = bshift(A, bs);
    partials = bshift(partials, bs);
    const int tid = threadIdx.x;
    // split-major order: the work-groups resident together share one K range, so each row tile
    // of that range is fetched from memory once and re-read by its other pairs from cache
    const int npairs = T_tiles * (T_tiles + 1) / 2;
    const int split = blockIdx.x / npairs;
    const int pidx = blockIdx.x - split * npairs;
    int ti, tj;
    pair_of(pidx, T_tiles, ti, tj);
    const bool diag = (ti == tj);
    const int r0a = ti * BM, r0b = tj * BM;
    const long kbeg = (long)split * kchunk;
    const long kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    // per-thread load coordinates
    constexpr int PER = BM * BK / NT;   // elements per thread per tile
    int lk, lm, mstep, kstep;
    if (MODE == 2) { lm = tid % BM; lk = tid / BM; mstep = 0; kstep = NT / BM; }
    else           { lk = tid % BK; lm = tid / BK; mstep = NT / BK; kstep = 0; }

    typedef typename std::conditional<sizeof(T) == 8, f64x4, f32x16>::type acc_t;
    acc_t acc[sizeof(T) == 8 ? 4 : 1];
#pragma unroll
    for (int q = 0; q < (sizeof(T) == 8 ? 4 : 1); ++q)
        for (int v = 0; v < (sizeof(T) == 8 ? 4 : 16); ++v) acc[q][v] = 0;

    T ra[PER], rb[PER];
    KCursor<MODE> cur;
    if (MODE != 2) cur.init(u, kbeg + lk);
    const long rs = u.rowstride();
    auto gload = [&](long k0) {
        const long cb = (MODE != 2) ? cur.base(u) : 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int m = lm + e * mstep, kk = lk + e * kstep;
            long Kg = k0 + kk;
            bool kin = Kg < kend;
            int rowa = r0a + m, rowb = r0b + m;
            const long aa = (MODE != 2) ? cb + (long)rowa * rs : u.addr(rowa, Kg);
            const long ab = (MODE != 2) ? cb + (long)rowb * rs : u.addr(rowb, Kg);
            ra[e] = (kin && rowa < nrow) ? A[aa] : (T)0;
            if (!diag) rb[e] = (kin && rowb < nrow) ? A[ab] : (T)0;
        }
        if (MODE != 2) cur.advance(u, BK);
    };
    auto sstore = [&]() {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int m = lm + e * mstep, kk = lk + e * kstep;
            As[kk][m] = ra[e];
            if (!diag) Bs[kk][m] = rb[e];
        }
    };

    gload(kbeg);
    for (long k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (k0 + BK < kend) gload(k0 + BK);     // prefetch the next chunk into registers
        T (*Bp)[BM + 1] = diag ? As : Bs;
        if constexpr (sizeof(T) == 8) {
            // 2 x 2 blocks of 16 x 16 per wave, k-steps of 4
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                int kr = ks + (lane >> 4);
                double a0 = As[kr][wm + (lane & 15)], a1 = As[kr][wm + 16 + (lane & 15)];
                double b0 = Bp[kr][wn + (lane & 15)], b1 = Bp[kr][wn + 16 + (lane & 15)];
                acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
                acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < BK; ks += 2) {
                int kr = ks + (lane >> 5);
                float a = As[kr][wm + (lane & 31)];
                float b = Bp[kr][wn + (lane & 31)];
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[0], 0, 0, 0);
            }
        }
    }

    // write the 64 x 64 partial (row-major) of this (pair, split)
    T* P = partials + ((long)pidx * nsplit + split) * (BM * BM);
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int i = wm + 16 * bi + 4 * v + (lane >> 4);
                    int j = wn + 16 * bj + (lane & 15);
                    P[i * BM + j] = acc[bi * 2 + bj][v];
                }
    } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int i = wm + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
            int j = wn + (lane & 31);
            P[i * BM + j] = acc[0][v];
        }
    }
}

// ----------------------------------------------------------------------------------------
// FP32, large tiles.  Work-group = 4 waves (2 x 2), output tile BG x BG, each wave a 64 x 64
// block of four mfma_f32_32x32x2f32 accumulators.  Within a K chunk of 32, MFMA step j (0..15)
// takes k = j on lanes 0-31 and k = 16 + j on lanes 32-63 (any fixed assignment of the chunk's
// k values to the steps sums the same products).  LDS layout: modes 0/1 (unfoldings contiguous
// along K) [m][k] with row stride 36 floats, read as float4 runs of k; mode 2 (contiguous along
// the rows) [k][m] with row stride 132, read one float per lane.  Both strides keep the float4
// stores and the operand reads free of bank conflicts.
// ----------------------------------------------------------------------------------------
constexpr int BG = 128;
constexpr int BKG = 32;

// LDS of one large-tile work-group: the two tiles, sized for the widest mode layout
constexpr int BIG_LDS = (BG * (BKG + 4) > BKG * (BG + 4)) ? BG * (BKG + 4) : BKG * (BG + 4);

// Work-group b of one mode's large-tile Gram (npairs x nsplit work-groups; A and partials already
// moved to the batched problem).
template <int MODE>
__device__ __forceinline__ void gram_big_body(float* __restrict__ As, float* __restrict__ Bs,
                                              const float* __restrict__ A, const Unfold<MODE>& u, int nrow, long K,
                                              long kchunk, int T_tiles, int npairs, int nsplit,
                                              float* __restrict__ partials, int b)
{
    constexpr int SL = (MODE == 2) ? BG + 4 : BKG + 4;   // LDS row stride (floats)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // blocks b with equal b mod 8 share an XCD: the npairs tile pairs of split
    // (b mod 8) + 8 floor(b / (8 npairs)) are consecutive blocks of one XCD
    const int xcd = b & 7, l = b >> 3;
    const int grp = l / npairs;
    const int pidx = l - grp * npairs;
    const int split = xcd + 8 * grp;
    int ti, tj;
    pair_of(pidx, T_tiles, ti, tj);
    const bool diag = (ti == tj);
    const int r0a = ti * BG, r0b = tj * BG;
    const long kbeg = (long)split * kchunk;
    const long kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

    f32x16 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[bi][bj][v] = 0.f;

    // global -> register staging: 4 runs of 4 floats per tile per thread (native vector type:
    // the HIP float4 class kept these arrays in scratch memory)
    f32x4 ra[4], rb[4];
    // modes 0/1: thread (rr = tid / 8, c4 = tid % 8) loads rows rr + 32 e, k = 4 c4 .. 4 c4 + 3
    // mode 2:    thread (c32 = tid % 32, kq = tid / 32) loads rows 4 c32 .. 4 c32 + 3, k = kq + 8 e
    const int rr = tid >> 3, c4 = tid & 7;
    const int c32 = tid & 31, kq = tid >> 5;
    long q1 = 0;   // mode 1: the chunk's i0 block and offset within it (K = q1 n2 + o1)
    int o1 = 0;
    if (MODE == 1) { q1 = kbeg / u.n2; o1 = (int)(kbeg - q1 * u.n2); }
    const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
    auto gload = [&](long k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (MODE == 2) {
                const long base = (k0 + kq + 8 * e) * (long)u.n2;
                const int ra_ = r0a + 4 * c32, rb_ = r0b + 4 * c32;
                ra[e] = ra_ < nrow ? *reinterpret_cast<const f32x4*>(A + base + ra_) : z4;
                if (!diag) rb[e] = rb_ < nrow ? *reinterpret_cast<const f32x4*>(A + base + rb_) : z4;
            } else {
                const int rowa = r0a + rr + 32 * e, rowb = r0b + rr + 32 * e;
                const long kb = (MODE == 0) ? k0 + 4 * c4 : q1 * u.n1n2 + o1 + 4 * c4;
                const long rs = u.rowstride();
                ra[e] = rowa < nrow ? *reinterpret_cast<const f32x4*>(A + kb + (long)rowa * rs) : z4;
                if (!diag) rb[e] = rowb < nrow ? *reinterpret_cast<const f32x4*>(A + kb + (long)rowb * rs) : z4;
            }
        }
        if (MODE == 1) {
            o1 += BKG;
            if (o1 >= u.n2) { o1 -= u.n2; ++q1; }
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int off = (MODE == 2) ? (kq + 8 * e) * SL + 4 * c32 : (rr + 32 * e) * SL + 4 * c4;
            *reinterpret_cast<f32x4*>(&As[off]) = ra[e];
            if (!diag) *reinterpret_cast<f32x4*>(&Bs[off]) = rb[e];
        }
    };

    // The K loop, in three copies by the wave's role (chosen once, outside the loop, so the loop
    // body has no branches): ROLE 0 forms all four 32 x 32 blocks; in diagonal tiles the
    // reduction reads only the upper half, so waves 0 and 3 (diagonal 64 x 64 blocks) leave out
    // block (1, 0) (ROLE 1) and wave 2 (rows 64-127 x columns 0-63) forms nothing (ROLE 2).
    // Every wave stages its share of the tiles and meets the same barriers; the skipped
    // accumulators stay zero in the partial.
    auto kloop = [&](auto rolec) {
        constexpr int ROLE = decltype(rolec)::value;
        if (kbeg < kend) gload(kbeg);
        for (long k0 = kbeg; k0 < kend; k0 += BKG) {
            __syncthreads();
            sstore();
            __syncthreads();
            if (k0 + BKG < kend) gload(k0 + BKG);     // the next chunk, in flight during the products
            if constexpr (ROLE < 2) {
                const float* Bp = diag ? As : Bs;
                const int li = lane & 31, h = lane >> 5;
                if (MODE == 2) {
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const int kr = (16 * h + j) * SL;
                        const float a0 = As[kr + wm + li], a1 = As[kr + wm + 32 + li];
                        const float b0 = Bp[kr + wn + li], b1 = Bp[kr + wn + 32 + li];
                        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
                        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
                        if constexpr (ROLE == 0)
                            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
                        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kc = 16 * h + 4 * q;
                        const f32x4 av0 = *reinterpret_cast<const f32x4*>(&As[(wm + li) * SL + kc]);
                        const f32x4 av1 = *reinterpret_cast<const f32x4*>(&As[(wm + 32 + li) * SL + kc]);
                        const f32x4 bv0 = *reinterpret_cast<const f32x4*>(&Bp[(wn + li) * SL + kc]);
                        const f32x4 bv1 = *reinterpret_cast<const f32x4*>(&Bp[(wn + 32 + li) * SL + kc]);
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0[t], bv0[t], acc[0][0], 0, 0, 0);
                            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0[t], bv1[t], acc[0][1], 0, 0, 0);
                            if constexpr (ROLE == 0)
                                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1[t], bv0[t], acc[1][0], 0, 0, 0);
                            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1[t], bv1[t], acc[1][1], 0, 0, 0);
                        }
                    }
                }
            }
        }
    };
    const int role = !diag ? 0 : (wave == 2 ? 2 : (wave == 1 ? 0 : 1));
    if (role == 0) kloop(std::integral_constant<int, 0>{});
    else if (role == 1) kloop(std::integral_constant<int, 1>{});
    else kloop(std::integral_constant<int, 2>{});

    // the BG x BG partial (row-major) of this (pair, split)
    float* P = partials + ((long)pidx * nsplit + split) * (BG * BG);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = wm + 32 * bi + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
                const int j = wn + 32 * bj + (lane & 31);
                P[i * BG + j] = acc[bi][bj][v];
            }
}

template <int MODE>
__global__ void __launch_bounds__(NT) k_gram_big(const float* __restrict__ A, Unfold<MODE> u, int nrow, long K,
                                                 long kchunk, int T_tiles, int npairs,
                                                 float* __restrict__ partials, long bs)
{
    __shared__ __attribute__((aligned(16))) float As[BIG_LDS];
    __shared__ __attribute__((aligned(16))) float Bs[BIG_LDS];
    gram_big_body<MODE>(As, Bs, bshift(A, bs), u, nrow, K, kchunk, T_tiles, npairs, (int)(gridDim.x / npairs),
                        bshift(partials, bs), (int)blockIdx.x);
}

// The three mode Grams of one tensor in one launch: work-groups [first[m], first[m + 1]) are
// those of mode m (each range a multiple of 8, so a work-group keeps the XCD it has in the
// launch of its mode alone, and every partial is the same).
struct Gram3Args {
    Unfold<0> u0;
    Unfold<1> u1;
    Unfold<2> u2;
    int nrow[3], T_tiles[3], npairs[3], nsplit[3], first[4];
    long K[3], kchunk[3];
    float* partials[3];
};

__global__ void __launch_bounds__(NT) k_gram_big3(const float* __restrict__ A, Gram3Args g, long bs)
{
    __shared__ __attribute__((aligned(16))) float As[BIG_LDS];
    __shared__ __attribute__((aligned(16))) float Bs[BIG_LDS];
    A = bshift(A, bs);
    const int b = (int)blockIdx.x;
    if (b < g.first[1])
        gram_big_body<0>(As, Bs, A, g.u0, g.nrow[0], g.K[0], g.kchunk[0], g.T_tiles[0], g.npairs[0], g.nsplit[0],
                         bshift(g.partials[0], bs), b);
    else if (b < g.first[2])
        gram_big_body<1>(As, Bs, A, g.u1, g.nrow[1], g.K[1], g.kchunk[1], g.T_tiles[1], g.npairs[1], g.nsplit[1],
                         bshift(g.partials[1], bs), b - g.first[1]);
    else
        gram_big_body<2>(As, Bs, A, g.u2, g.nrow[2], g.K[2], g.kchunk[2], g.T_tiles[2], g.npairs[2], g.nsplit[2],
                         bshift(g.partials[2], bs), b - g.first[2]);
}

// ----------------------------------------------------------------------------------------
// BF16x3 tiles.  LDS holds [BM][BK + 8] bf16 hi and lo parts (row-major, so that each lane
// reads its 8 consecutive k values with one 16-byte load).
// ----------------------------------------------------------------------------------------
template <int MODE, int BK>
__global__ void __launch_bounds__(NT) k_gram_tiles_bf16x3(const float* __restrict__ A, Unfold<MODE> u,
                                                          int nrow, long K, long kchunk, int T_tiles,
                                                          int nsplit, float* __restrict__ partials, long bs)
{
    constexpr int LD = BK + 8;
    __shared__ __attribute__((aligned(16))) __bf16 Ah[BM][LD], Al[BM][LD], Bh[BM][LD], Bl[BM][LD];
    A = bshift(A, bs);
    partials = bshift(partials, bs);
    const int tid = threadIdx.x;
    // split-major order: the work-groups resident together share one K range, so each row tile
    // of that range is fetched from memory once and re-read by its other pairs from cache
    const int npairs = T_tiles * (T_tiles + 1) / 2;
    const int split = blockIdx.x / npairs;
    const int pidx = blockIdx.x - split * npairs;
    int ti, tj;
    pair_of(pidx, T_tiles, ti, tj);
    const bool diag = (ti == tj);
    const int r0a = ti * BM, r0b = tj * BM;
    const long kbeg = (long)split * kchunk;
    const long kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    constexpr int PER = BM * BK / NT;
    int lk, lm, mstep, kstep;
    if (MODE == 2) { lm = tid % BM; lk = tid / BM; mstep = 0; kstep = NT / BM; }
    else           { lk = tid % BK; lm = tid / BK; mstep = NT / BK; kstep = 0; }

    f32x16 acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    float ra[PER], rb[PER];
    KCursor<MODE> cur;
    if (MODE != 2) cur.init(u, kbeg + lk);
    const long rs = u.rowstride();
    auto gload = [&](long k0) {
        const long cb = (MODE != 2) ? cur.base(u) : 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int m = lm + e * mstep, kk = lk + e * kstep;
            long Kg = k0 + kk;
            bool kin = Kg < kend;
            int rowa = r0a + m, rowb = r0b + m;
            const long aa = (MODE != 2) ? cb + (long)rowa * rs : u.addr(rowa, Kg);
            const long ab = (MODE != 2) ? cb + (long)rowb * rs : u.addr(rowb, Kg);
            ra[e] = (kin && rowa < nrow) ? A[aa] : 0.f;
            if (!diag) rb[e] = (kin && rowb < nrow) ? A[ab] : 0.f;
        }
        if (MODE != 2) cur.advance(u, BK);
    };
    auto sstore = [&]() {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int m = lm + e * mstep, kk = lk + e * kstep;
            __bf16 h, l;
            split_bf16(ra[e], h, l);
            Ah[m][kk] = h; Al[m][kk] = l;
            if (!diag) { split_bf16(rb[e], h, l); Bh[m][kk] = h; Bl[m][kk] = l; }
        }
    };

    gload(kbeg);
    for (long k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (k0 + BK < kend) gload(k0 + BK);
        __bf16 (*BhP)[LD] = diag ? Ah : Bh;
        __bf16 (*BlP)[LD] = diag ? Al : Bl;
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            int kc = ks + 8 * (lane >> 5);
            int ra_ = wm + (lane & 31), rb_ = wn + (lane & 31);
            bf16x8 ah = *reinterpret_cast<const bf16x8*>(&Ah[ra_][kc]);
            bf16x8 al = *reinterpret_cast<const bf16x8*>(&Al[ra_][kc]);
            bf16x8 bh = *reinterpret_cast<const bf16x8*>(&BhP[rb_][kc]);
            bf16x8 bl = *reinterpret_cast<const bf16x8*>(&BlP[rb_][kc]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
        }
    }
    float* P = partials + ((long)pidx * nsplit + split) * (BM * BM);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        int i = wm + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
        int j = wn + (lane & 31);
        P[i * BM + j] = acc[v];
    }
}

// G[ti*TB + ii][tj*TB + jj] = sum_s P[pair][s][ii][jj] in FP64 (TB: the tile edge); mirrored.  Each entry is
// summed by 4 threads (thread g takes splits g, g + 4, g + 8, ... in order) and the four
// sums are added in the fixed order g = 0, 1, 2, 3, so the result does not depend on timing.
template <typename T, int TB>
__device__ __forceinline__ void gram_reduce_body(const T* __restrict__ partials, int T_tiles, int nsplit, int nrow,
                                                 double* __restrict__ G, int pidx, int bx)
{
    __shared__ double part[4][64];
    int ti, tj;
    pair_of(pidx, T_tiles, ti, tj);
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int e = bx * 64 + lane;                     // entry within the tile
    const T* P = partials + (long)pidx * nsplit * (TB * TB) + e;
    double s = 0.0;
    for (int q = g; q < nsplit; q += 4) s += (double)P[(long)q * (TB * TB)];
    part[g][lane] = s;
    __syncthreads();
    if (g != 0) return;
    const int ii = e / TB, jj = e % TB;
    if (ti == tj && ii > jj) return;                  // diagonal tiles: upper half only
    const int gi = ti * TB + ii, gj = tj * TB + jj;
    if (gi >= nrow || gj >= nrow) return;
    const double v = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    G[(long)gi * nrow + gj] = v;
    G[(long)gj * nrow + gi] = v;
}

template <typename T, int TB>
__global__ void __launch_bounds__(256) k_gram_reduce(const T* __restrict__ partials, int T_tiles,
                                                     int nsplit, int nrow, double* __restrict__ G, long bs)
{
    gram_reduce_body<T, TB>(bshift(partials, bs), T_tiles, nsplit, nrow, bshift(G, bs), (int)blockIdx.y,
                            (int)blockIdx.x);
}

// The reductions of the three modes of k_gram_big3 in one launch: blockIdx.y runs over the tile
// pairs of mode 0, then 1, then 2.
__global__ void __launch_bounds__(256) k_gram_reduce3(Gram3Args g, double* __restrict__ G0, double* __restrict__ G1,
                                                      double* __restrict__ G2, long bs)
{
    const int y = (int)blockIdx.y;
    const int m = (y < g.npairs[0]) ? 0 : (y < g.npairs[0] + g.npairs[1] ? 1 : 2);
    const int pidx = y - (m > 0 ? g.npairs[0] : 0) - (m > 1 ? g.npairs[1] : 0);
    double* G = (m == 0) ? G0 : (m == 1 ? G1 : G2);
    gram_reduce_body<float, BG>(bshift((const float*)g.partials[m], bs), g.T_tiles[m], g.nsplit[m], g.nrow[m],
                                bshift(G, bs), pidx, (int)blockIdx.x);
}

struct GramPlan {
    int nrow, T_tiles, npairs, nsplit;
    long K, kchunk;
};

GramPlan make_plan(const int n[3], int mode, int BK, int nsplit_req = 0)
{
    GramPlan p;
    long N = (long)n[0] * n[1] * n[2];
    p.nrow = n[mode];
    p.K = N / n[mode];
    p.T_tiles = (p.nrow + BM - 1) / BM;
    p.npairs = p.T_tiles * (p.T_tiles + 1) / 2;
    long want = (2048 + p.npairs - 1) / p.npairs;               // ~2048 work-groups
    if (want > (p.K + 63) / 64) want = (p.K + 63) / 64;          // but at least 64 of K each
    long maxsplit = (p.K + BK - 1) / BK;
    if (nsplit_req > 0) want = nsplit_req;                      // a tuned split count
    long s = want < maxsplit ? want : maxsplit;
    if (s < 1) s = 1;
    long kc = (p.K + s - 1) / s;
    kc = (kc + BK - 1) / BK * BK;
    p.kchunk = kc;
    p.nsplit = (int)((p.K + kc - 1) / kc);
    return p;
}

constexpr int BK_F32 = 32, BK_F64 = 16, BK_BF = 32;

int bk_for(int prec) { return prec == 0 ? BK_F64 : (prec == 1 ? BK_F32 : BK_BF); }

// The large-tile kernel can take FP32 modes with n_mode >= 128 when every extent is a multiple
// of 32 (float4 runs and whole K chunks inside one i0 block of the mode-1 unfolding); it is the
// default from n_mode >= 256 on.  A split request ("code") of GRAM_BIG + s asks for the
// large-tile kernel with s splits, 0 < s < GRAM_BIG for the 64-tile kernel, 0 for the default.
bool big_eligible(const int n[3], int mode, int prec)
{
    return prec == 1 && n[mode] >= 128 && n[0] % 32 == 0 && n[1] % 32 == 0 && n[2] % 32 == 0;
}

bool use_big(const int n[3], int mode, int prec, int code)
{
    if (!big_eligible(n, mode, prec)) return false;
    if (code >= GRAM_BIG) return true;
    if (code > 0) return false;
    return n[mode] >= 256;
}

int split_of(int code) { return code >= GRAM_BIG ? code - GRAM_BIG : code; }

// Large-tile split count for about `per_cu` resident work-groups on each of the 256 CUs (164
// VGPRs per lane: three waves per SIMD, so three work-groups per CU at most), rounded down to a
// multiple of 8 (the XCD grouping), at least 8.
int big_splits(int npairs, int per_cu)
{
    const int s = (256 * per_cu / npairs) / 8 * 8;
    return s > 8 ? s : 8;
}

// Large-tile plan: nsplit a multiple of 8 (default: three work-groups per CU, capped so that the
// partials hold at most a quarter of the tensor's elements; a requested split count is rounded up
// to a multiple of 8).
GramPlan make_plan_big(const int n[3], int mode, int nsplit_req = 0)
{
    GramPlan p;
    long N = (long)n[0] * n[1] * n[2];
    p.nrow = n[mode];
    p.K = N / n[mode];
    p.T_tiles = (p.nrow + BG - 1) / BG;
    p.npairs = p.T_tiles * (p.T_tiles + 1) / 2;
    long s = nsplit_req;
    if (s <= 0) {
        // three work-groups per CU, but no more split partials than a quarter of the tensor
        // (their write and read-back in the reduction would cost more than the extra parallelism)
        s = big_splits(p.npairs, 3);
        const long cap = (N / (4L * p.npairs * BG * BG)) / 8 * 8;
        if (s > cap) s = cap > 8 ? cap : 8;
    }
    s = (s + 7) / 8 * 8;
    const long maxs = (p.K + BKG - 1) / BKG;
    if (s > (maxs + 7) / 8 * 8) s = (maxs + 7) / 8 * 8;
    long kc = (p.K + s - 1) / s;
    kc = (kc + BKG - 1) / BKG * BKG;
    p.kchunk = kc;
    p.nsplit = (int)s;   // trailing splits past K (if any) add zeros
    return p;
}

}  // namespace

int gram_default_splits(const int n[3], int mode, int prec)
{
    if (use_big(n, mode, prec, 0)) return GRAM_BIG + make_plan_big(n, mode).nsplit;
    return make_plan(n, mode, bk_for(prec)).nsplit;
}

size_t gram_work_bytes(const int n[3], int mode, int prec, int code)
{
    if (use_big(n, mode, prec, code)) {
        GramPlan p = make_plan_big(n, mode, split_of(code));
        return (size_t)p.npairs * p.nsplit * BG * BG * 4;
    }
    GramPlan p = make_plan(n, mode, bk_for(prec), split_of(code));
    size_t elt = (prec == 0) ? 8 : 4;
    return (size_t)p.npairs * p.nsplit * BM * BM * elt;
}

int gram_split_candidates(const int n[3], int mode, int prec, int out[GRAM_MAX_CANDIDATES])
{
    // out[0] the default; then, within the default's workspace, about 3, 2 and 1 work-groups per
    // CU of the large-tile kernel (where it can run) and the 64-tile kernel at its default split,
    // half and a quarter of it
    const int def = gram_default_splits(n, mode, prec);
    const size_t wmax = gram_work_bytes(n, mode, prec, def);
    int c = 0;
    out[c++] = def;
    auto add = [&](int code) {
        for (int i = 0; i < c; ++i)
            if (out[i] == code) return;
        if (c < GRAM_MAX_CANDIDATES && gram_work_bytes(n, mode, prec, code) <= wmax) out[c++] = code;
    };
    if (big_eligible(n, mode, prec)) {
        const GramPlan p = make_plan_big(n, mode);
        for (int per = 3; per >= 1; --per) add(GRAM_BIG + make_plan_big(n, mode, big_splits(p.npairs, per)).nsplit);
    }
    const int s0 = make_plan(n, mode, bk_for(prec)).nsplit;
    for (int d = 1; d <= 4; d *= 2) add(s0 / d > 1 ? s0 / d : 1);
    return c;
}

template <int MODE>
static hipError_t launch_mode(const void* A, const int n[3], int prec, double* G, void* work, hipStream_t s,
                              Bat bt, int nsplit)
{
    Unfold<MODE> u;
    u.n1n2 = (long)n[1] * n[2];
    u.n1 = n[1];
    u.n2 = n[2];
    if (use_big(n, MODE, prec, nsplit)) {
        GramPlan p = make_plan_big(n, MODE, split_of(nsplit));
        dim3 grid((unsigned)(p.npairs * p.nsplit), 1, bt.nb);
        hipLaunchKernelGGL(k_gram_big<MODE>, grid, dim3(NT), 0, s, (const float*)A, u, p.nrow, p.K, p.kchunk,
                           p.T_tiles, p.npairs, (float*)work, bt.bs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        dim3 rgrid(BG * BG / 64, p.npairs, bt.nb);
        hipLaunchKernelGGL((k_gram_reduce<float, BG>), rgrid, dim3(256), 0, s, (const float*)work, p.T_tiles,
                           p.nsplit, p.nrow, G, bt.bs);
        return hipGetLastError();
    }
    GramPlan p = make_plan(n, MODE, bk_for(prec), split_of(nsplit));
    dim3 grid((unsigned)(p.npairs * p.nsplit), 1, bt.nb);
    if (prec == 0) {
        hipLaunchKernelGGL((k_gram_tiles<MODE, double, BK_F64>), grid, dim3(NT), 0, s, (const double*)A, u,
                           p.nrow, p.K, p.kchunk, p.T_tiles, p.nsplit, (double*)work, bt.bs);
    } else if (prec == 1) {
        hipLaunchKernelGGL((k_gram_tiles<MODE, float, BK_F32>), grid, dim3(NT), 0, s, (const float*)A, u,
                           p.nrow, p.K, p.kchunk, p.T_tiles, p.nsplit, (float*)work, bt.bs);
    } else {
        hipLaunchKernelGGL((k_gram_tiles_bf16x3<MODE, BK_BF>), grid, dim3(NT), 0, s, (const float*)A, u,
                           p.nrow, p.K, p.kchunk, p.T_tiles, p.nsplit, (float*)work, bt.bs);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 rgrid(BM * BM / 64, p.npairs, bt.nb);
    if (prec == 0)
        hipLaunchKernelGGL((k_gram_reduce<double, BM>), rgrid, dim3(256), 0, s, (const double*)work, p.T_tiles,
                           p.nsplit, p.nrow, G, bt.bs);
    else
        hipLaunchKernelGGL((k_gram_reduce<float, BM>), rgrid, dim3(256), 0, s, (const float*)work, p.T_tiles,
                           p.nsplit, p.nrow, G, bt.bs);
    return hipGetLastError();
}

bool gram3_eligible(const int n[3], int prec, const int codes[3])
{
    for (int k = 0; k < 3; ++k)
        if (!use_big(n, k, prec, codes[k])) return false;
    return true;
}

size_t gram3_work_bytes(const int n[3], int prec, const int codes[3])
{
    size_t t = 0;
    for (int k = 0; k < 3; ++k) t += (gram_work_bytes(n, k, prec, codes[k]) + 255) / 256 * 256;
    return t;
}

hipError_t launch_gram3(const void* A, const int n[3], int prec, double* G, long sG, void* work, hipStream_t s,
                        Bat bt, const int codes[3])
{
    if (bt.nb < 1 || !gram3_eligible(n, prec, codes)) return hipErrorInvalidValue;
    Gram3Args g;
    g.u0.n1n2 = g.u1.n1n2 = g.u2.n1n2 = (long)n[1] * n[2];
    g.u0.n1 = g.u1.n1 = g.u2.n1 = n[1];
    g.u0.n2 = g.u1.n2 = g.u2.n2 = n[2];
    char* wp = (char*)work;
    g.first[0] = 0;
    int npairs_total = 0;
    for (int k = 0; k < 3; ++k) {
        const GramPlan p = make_plan_big(n, k, split_of(codes[k]));
        g.nrow[k] = p.nrow;
        g.T_tiles[k] = p.T_tiles;
        g.npairs[k] = p.npairs;
        g.nsplit[k] = p.nsplit;
        g.K[k] = p.K;
        g.kchunk[k] = p.kchunk;
        g.partials[k] = (float*)wp;
        wp += ((size_t)p.npairs * p.nsplit * BG * BG * 4 + 255) / 256 * 256;
        g.first[k + 1] = g.first[k] + p.npairs * p.nsplit;
        npairs_total += p.npairs;
    }
    hipLaunchKernelGGL(k_gram_big3, dim3((unsigned)g.first[3], 1, bt.nb), dim3(NT), 0, s, (const float*)A, g, bt.bs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce3, dim3(BG * BG / 64, npairs_total, bt.nb), dim3(256), 0, s, g, G, G + sG,
                       G + 2 * sG, bt.bs);
    return hipGetLastError();
}

hipError_t launch_gram(const void* A, const int n[3], int mode, int prec, double* G, void* work,
                       hipStream_t s, Bat bt, int nsplit)
{
    if (bt.nb < 1) return hipErrorInvalidValue;
    if (mode == 0) return launch_mode<0>(A, n, prec, G, work, s, bt, nsplit);
    if (mode == 1) return launch_mode<1>(A, n, prec, G, work, s, bt, nsplit);
    return launch_mode<2>(A, n, prec, G, work, s, bt, nsplit);
}

}  // namespace tk
