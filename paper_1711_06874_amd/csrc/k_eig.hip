// a3: leading eigenpairs of the symmetric positive semidefinite Gram matrices of the HOSVD
// and of the HOOI single-hole tensors (Sec. 3.2), in FP64.
//
// Method: block subspace (orthogonal) iteration with Rayleigh-Ritz.  With a working block of
// p >= r + 8 columns, every iteration multiplies the block by G and re-orthonormalises it
// with Householder QR; the Gram spectra of these kernel tensors fall by orders of magnitude
// per index, so the block converges in a few iterations (warm starts from the previous HOOI
// factor need fewer).  The projected p x p matrix Q^T G Q is diagonalised by two-sided Jacobi
// with the parallel (round-robin) ordering, its eigenpairs are sorted in descending order,
// U = Q V, and each column is signed so that its entry of largest magnitude is positive
// (entries within 1e-10 relative of the maximum tie, the lowest index wins).  When p == n
// the block is the identity and the whole matrix is diagonalised by Jacobi directly.
//
// Kernels: k_eig_init (start block; a warm block of exactly p columns is read in place by the
// first product instead), k_cholqr_reg (Cholesky QR of the span-only blocks of the float eps
// path, with a Householder fallback), k_hqr_reg (rows in registers, n <= 1024 and p <= 32; it can
// also write an FP32 copy of the factor) and k_hqr (one work-group per problem, Householder QR with the
// n x p block resident in LDS when it fits, producing the explicit Q in place), k_jacobi_w /
// k_jacobi (one work-group per problem, p x p in LDS), k_signfix; the products G Q, Q^T Y and
// Q V use the batched small-product kernel.
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr size_t QR_LDS_BYTES = 144 * 1024;

// Counter-based uniform in [-1, 1) from (problem, row, column): a 64-bit integer mix
// (splitmix64 finaliser).  Only used to seed the iteration; any full-rank start works.
__device__ __forceinline__ double start_value(unsigned long long key)
{
    unsigned long long z = key + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 4503599627370496.0) - 1.0;   // 2^52
}

__global__ void k_eig_init(EigBatch b)
{
    b.warm = bshift(b.warm, b.bs);
    b.Q = bshift(b.Q, b.bs);
    int prob = blockIdx.y;
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long tot = (long)b.n * b.p;
    if (idx >= tot) return;
    int i = (int)(idx / b.p), j = (int)(idx % b.p);
    double v;
    if (b.p == b.n) v = (i == j) ? 1.0 : 0.0;
    else if (j < b.rw && b.warm) v = b.warm[prob * b.sW + (long)i * b.ldw + j];
    else v = start_value(((unsigned long long)prob << 40) ^ ((unsigned long long)i << 20) ^ (unsigned long long)j);
    b.Q[prob * (long)tot + idx] = v;
}

// Householder QR of the n x p matrix In (row-major, ld p) of problem blockIdx.x; writes the
// explicit orthonormal factor (n x p) to Out.  W is the working copy (LDS if it fits).
//
// Per column j three barrier-separated phases, with no integer division in any loop:
//   A: finish column j-1 (scale its reflector below the diagonal, store beta on it) and form
//      ||W[j+1:, j]||^2;
//   B: every thread derives (tau, scale, beta) of column j from the reduction, and the groups
//      form w_c = v^T W[j:, c] for c > j from the *unscaled* column (w_c = W[j][c] + scale *
//      sum_{i>j} W[i][j] W[i][c]), so column j is not touched in this phase;
//   C: W[i][c] -= tau v_i w_c for i >= j, c > j (one column per thread, rows strided).
// The explicit Q is then formed in place from the last reflector to the first.
__global__ void __launch_bounds__(256) k_hqr(const double* __restrict__ In, double* __restrict__ Out,
                                             int n, int p, int in_lds, long bs)
{
    In = bshift(In, bs);
    Out = bshift(Out, bs);
    extern __shared__ double smem[];
    __shared__ double red[4];
    __shared__ double wsum[64];
    __shared__ double tau_s[64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long off = (long)blockIdx.x * n * p;
    double* W = in_lds ? smem : (Out + off);
    for (int e = tid; e < n * p; e += 256) W[e] = In[off + e];
    __syncthreads();

    double prev_scale = 0.0, prev_beta = 0.0, prev_tau = 0.0;
    for (int j = 0; j < p; ++j) {
        // ---- phase A
        if (j > 0) {
            if (prev_tau != 0.0)
                for (int i = j + tid; i < n; i += 256) W[i * p + (j - 1)] *= prev_scale;
            if (tid == 0) W[(j - 1) * p + (j - 1)] = prev_beta;
        }
        double s = 0.0;
        for (int i = j + 1 + tid; i < n; i += 256) { double x = W[i * p + j]; s += x * x; }
        s = wave_sum(s);
        if (lane == 0) red[wv] = s;
        __syncthreads();
        // ---- phase B
        const double xn2 = (red[0] + red[1]) + (red[2] + red[3]);
        const double alpha = W[j * p + j];
        double t = 0.0, scale = 0.0, beta = alpha;
        if (xn2 > 0.0) {
            double nrm = sqrt(alpha * alpha + xn2);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            t = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (tid == 0) tau_s[j] = t;
        const int nc = p - j - 1;
        int G = 64;
        while (G > 1 && G * nc > 256) G >>= 1;
        if (t != 0.0 && nc > 0) {
            const int gid = tid / G, gl = tid & (G - 1);
            double acc = 0.0;
            if (gid < nc) {
                const int c = j + 1 + gid;
                for (int i = j + 1 + gl; i < n; i += G) acc += W[i * p + j] * W[i * p + c];
            }
            for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (gid < nc && gl == 0) wsum[gid] = W[j * p + j + 1 + gid] + scale * acc;
        }
        __syncthreads();
        // ---- phase C
        if (t != 0.0 && nc > 0) {
            const int per = 256 / nc;             // threads per column
            const int cc = tid % nc, r0 = tid / nc;
            if (r0 < per) {
                const int c = j + 1 + cc;
                const double tw = t * wsum[cc];
                if (r0 == 0) W[j * p + c] -= tw;
                for (int i = j + 1 + r0; i < n; i += per) W[i * p + c] -= tw * scale * W[i * p + j];
            }
        }
        __syncthreads();
        prev_scale = scale;
        prev_beta = beta;
        prev_tau = t;
    }
    // finish the last column
    if (prev_tau != 0.0)
        for (int i = p + tid; i < n; i += 256) W[i * p + (p - 1)] *= prev_scale;
    if (tid == 0) W[(p - 1) * p + (p - 1)] = prev_beta;
    __syncthreads();

    // ---- explicit Q, built in place from the last reflector to the first
    for (int j = p - 1; j >= 0; --j) {
        const double t = tau_s[j];
        const int nc = p - j - 1;
        if (nc > 0 && t != 0.0) {
            int G = 64;
            while (G > 1 && G * nc > 256) G >>= 1;
            const int gid = tid / G, gl = tid & (G - 1);
            double acc = 0.0;
            if (gid < nc) {
                const int c = j + 1 + gid;
                for (int i = j + 1 + gl; i < n; i += G) acc += W[i * p + j] * W[i * p + c];
            }
            for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (gid < nc && gl == 0) wsum[gid] = W[j * p + j + 1 + gid] + acc;
            __syncthreads();
            const int per = 256 / nc;
            const int cc = tid % nc, r0 = tid / nc;
            if (r0 < per) {
                const int c = j + 1 + cc;
                const double tw = t * wsum[cc];
                if (r0 == 0) W[j * p + c] -= tw;
                for (int i = j + 1 + r0; i < n; i += per) W[i * p + c] -= tw * W[i * p + j];
            }
            __syncthreads();
        }
        // column j of Q: -tau v below, 1 - tau on the diagonal, 0 above
        for (int i = tid; i < n; i += 256) {
            double x;
            if (i < j) x = 0.0;
            else if (i == j) x = 1.0 - t;
            else x = -t * W[i * p + j];
            W[i * p + j] = x;
        }
        __syncthreads();
    }
    if (in_lds)
        for (int e = tid; e < n * p; e += 256) Out[off + e] = W[e];
}

// Two-sided Jacobi on the p x p symmetric H of problem blockIdx.x (row-major; symmetrised),
// parallel round-robin ordering.  Outputs the r leading eigenvalues (descending, stable) and
// the matching eigenvector columns Vs (p x r, row-major).
__global__ void __launch_bounds__(256) k_jacobi(const double* __restrict__ Hin, int p, int r,
                                                double* __restrict__ Vs, double* __restrict__ lam,
                                                long sLam, int max_sweeps, double tol, long bs)
{
    Hin = bshift(Hin, bs);
    Vs = bshift(Vs, bs);
    lam = bshift(lam, bs);
    __shared__ double H[EIG_PMAX][EIG_PMAX + 1];
    __shared__ double V[EIG_PMAX][EIG_PMAX + 1];
    __shared__ double cs[EIG_PMAX / 2][2];
    __shared__ int pq[EIG_PMAX / 2][2];
    __shared__ double red[4];
    __shared__ int flag;
    __shared__ double prev_off_s;
    __shared__ int rank_of[EIG_PMAX];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double* Hp = Hin + (long)blockIdx.x * p * p;
    for (int e = tid; e < p * p; e += 256) {
        int i = e / p, j = e % p;
        H[i][j] = 0.5 * (Hp[i * p + j] + Hp[j * p + i]);
        V[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int m = p + (p & 1);
    // Frobenius norm for the stopping test
    double s = 0.0;
    for (int e = tid; e < p * p; e += 256) { double x = H[e / p][e % p]; s += x * x; }
    s = wave_sum(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    const double fro = sqrt((red[0] + red[1]) + (red[2] + red[3]));
    // off(H) stalls near p u ||H||_F in floating point: never ask for less
    tol = fmax(tol, (double)p * 2.220446049250313e-16);
    if (tid == 0) prev_off_s = INFINITY;
    __syncthreads();

    for (int sweep = 0; sweep < max_sweeps && p > 1; ++sweep) {
        // off-diagonal norm
        double o = 0.0;
        if ((tid & 63) < p)
            for (int i = tid >> 6; i < p; i += 4)
                if (i != (tid & 63)) o += H[i][tid & 63] * H[i][tid & 63];
        o = wave_sum(o);
        if (lane == 0) red[wv] = o;
        __syncthreads();
        if (tid == 0) {
            const double off = sqrt((red[0] + red[1]) + (red[2] + red[3]));
            // converged, or stagnating at the rounding floor (see k_jacobi_w)
            flag = (off <= tol * fro || (off <= 1e-12 * fro && off > 0.5 * prev_off_s)) ? 1 : 0;
            prev_off_s = off;
        }
        __syncthreads();
        if (flag) break;
        for (int step = 0; step < m - 1; ++step) {
            if (tid < m / 2) {
                int k = tid, a, bb;
                if (k == 0) { a = m - 1; bb = step; }
                else { a = (step + k) % (m - 1); bb = (step - k + (m - 1)) % (m - 1); }
                if (a > bb) { int t = a; a = bb; bb = t; }
                double c = 1.0, sn = 0.0;
                if (bb < p) {
                    double apq = H[a][bb];
                    if (apq != 0.0) {
                        double tau = (H[bb][bb] - H[a][a]) / (2.0 * apq);
                        double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                                : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                    }
                }
                pq[k][0] = a; pq[k][1] = bb; cs[k][0] = c; cs[k][1] = sn;
            }
            __syncthreads();
            // rows: H <- J^T H ; V <- V J (columns of V).  Thread (k0 = tid/64, j = tid%64)
            // handles column j of pairs k0, k0 + 4, ...
            const int np = m / 2;
            const int jj = tid & 63, k0 = tid >> 6;
            if (jj < p) {
                for (int k = k0; k < np; k += 4) {
                    int a = pq[k][0], bb = pq[k][1];
                    double sn = cs[k][1];
                    if (bb >= p || sn == 0.0) continue;
                    double c = cs[k][0];
                    double x = H[a][jj], y = H[bb][jj];
                    H[a][jj] = c * x - sn * y;
                    H[bb][jj] = sn * x + c * y;
                    double vx = V[jj][a], vy = V[jj][bb];
                    V[jj][a] = c * vx - sn * vy;
                    V[jj][bb] = sn * vx + c * vy;
                }
            }
            __syncthreads();
            // columns: H <- H J  (thread handles row jj)
            if (jj < p) {
                for (int k = k0; k < np; k += 4) {
                    int a = pq[k][0], bb = pq[k][1];
                    double sn = cs[k][1];
                    if (bb >= p || sn == 0.0) continue;
                    double c = cs[k][0];
                    double x = H[jj][a], y = H[jj][bb];
                    H[jj][a] = c * x - sn * y;
                    H[jj][bb] = sn * x + c * y;
                }
            }
            __syncthreads();
        }
    }
    // stable descending ranks
    if (tid < p) {
        double d = H[tid][tid];
        int rk = 0;
        for (int i = 0; i < p; ++i) {
            double e = H[i][i];
            if (e > d || (e == d && i < tid)) ++rk;
        }
        rank_of[tid] = rk;
    }
    __syncthreads();
    double* Vo = Vs + (long)blockIdx.x * p * r;
    for (int e = tid; e < p * p; e += 256) {
        int i = e / p, j = e % p;      // V[i][j]: component i of eigenvector j
        int rk = rank_of[j];
        if (rk < r) Vo[i * r + rk] = V[i][j];
    }
    if (tid < p && rank_of[tid] < r) lam[(long)blockIdx.x * sLam + rank_of[tid]] = H[tid][tid];
}


// ---------------------------------------------------------------------------------------------
// S[c] = sum_i x_i w_i[c] for C0 <= c < PM over the RPT rows of every thread (x[q]: the
// multiplier of the thread's row q, 0 for rows that take no part).  T holds PM x NT doubles (the
// thread's rows are summed before the LDS transpose).  Everything but the row index is
// compile-time.
template <int PM, int NT, int RPT, int C0>
__device__ __forceinline__ void block_col_sums(double* T, double* S, const double (&w)[RPT][PM], const double (&x)[RPT])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int c = C0; c < PM; ++c) {
        double v = x[0] * w[0][c];
#pragma unroll
        for (int q = 1; q < RPT; ++q) v += x[q] * w[q][c];
        T[c * NT + t] = v;
    }
    __syncthreads();
    constexpr int NC = PM - C0;
    constexpr int G = (NC * 64 <= NT) ? 64 : (NC * 32 <= NT ? 32 : (NC * 16 <= NT ? 16 : (NC * 8 <= NT ? 8 : (NC * 4 <= NT ? 4 : (NC * 2 <= NT ? 2 : 1)))));
    const int ci = t / G, g = t & (G - 1);
    double acc = 0.0;
    if (ci < NC) {
        // four independent partial sums keep the dependent chain short
        const double* row = T + (C0 + ci) * NT;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        constexpr int NK = NT / G;
#pragma unroll
        for (int q = 0; q + 3 < NK; q += 4) {
            a0 += row[g + q * G];
            a1 += row[g + (q + 1) * G];
            a2 += row[g + (q + 2) * G];
            a3 += row[g + (q + 3) * G];
        }
#pragma unroll
        for (int q = NK - NK % 4; q < NK; ++q) a0 += row[g + q * G];
        acc = (a0 + a1) + (a2 + a3);
    }
#pragma unroll
    for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (ci < NC && g == 0) S[C0 + ci] = acc;
    __syncthreads();
}

// Householder step for column J (rows in registers, columns >= p are zero and stay zero).  Row q
// of thread i is row i + q NT of the block; row J (J < p <= PM <= 32 < NT) is row 0 of thread J.
template <int PM, int NT, int RPT, int J>
__device__ __forceinline__ void qr_forward(double (&w)[RPT][PM], double* T, double* S, double (*rowjb)[PM],
                                           double* taus, int n, int p)
{
    if constexpr (J < PM) {
        if (J >= p) return;
        const int i = threadIdx.x;
        double* rowj = rowjb[J & 1];
        if (i == J) {
#pragma unroll
            for (int c = 0; c < PM; ++c) rowj[c] = w[0][c];
        }
        double x[RPT], xs[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = i + q * NT;
            x[q] = w[q][J];
            xs[q] = (row < n && row > J) ? x[q] : 0.0;
        }
        block_col_sums<PM, NT, RPT, J>(T, S, w, xs);
        const double xn2 = S[J];
        const double alpha = rowj[J];
        double t = 0.0, scale = 0.0, beta = alpha;
        if (xn2 > 0.0) {
            const double nrm = sqrt(alpha * alpha + xn2);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            t = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (i == 0) taus[J] = t;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = i + q * NT;
            const double v = (row == J) ? 1.0 : ((row < n && row > J) ? x[q] * scale : 0.0);
            const double tv = t * v;
#pragma unroll
            for (int c = J + 1; c < PM; ++c) w[q][c] -= tv * (rowj[c] + scale * S[c]);
            // column J: beta on the diagonal, the scaled reflector below it
            w[q][J] = (row == J) ? beta : ((row > J) ? x[q] * scale : x[q]);
        }
        qr_forward<PM, NT, RPT, J + 1>(w, T, S, rowjb, taus, n, p);
    }
}

// Explicit Q, column J (from the last reflector to the first, in place).
template <int PM, int NT, int RPT, int J>
__device__ __forceinline__ void qr_backward(double (&w)[RPT][PM], double* T, double* S, const double* taus, int n,
                                            int p)
{
    if constexpr (J >= 0) {
        if (J < p) {
            const int i = threadIdx.x;
            double v[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int row = i + q * NT;
                v[q] = (row == J) ? 1.0 : ((row < n && row > J) ? w[q][J] : 0.0);
            }
            const double t = taus[J];
            if constexpr (J + 1 < PM) {
                if (J + 1 < p) {
                    block_col_sums<PM, NT, RPT, J + 1>(T, S, w, v);
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        const double tv = t * v[q];
#pragma unroll
                        for (int c = J + 1; c < PM; ++c) w[q][c] -= tv * S[c];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int row = i + q * NT;
                w[q][J] = (row < J) ? 0.0 : ((row == J) ? 1.0 - t : -t * v[q]);
            }
        }
        qr_backward<PM, NT, RPT, J - 1>(w, T, S, taus, n, p);
    }
}

// ---------------------------------------------------------------------------------------------
// Householder QR with the rows of the n x p block held in registers, RPT rows per thread
// (n <= RPT NT, p <= PM, columns p..PM-1 carried as zeros).  Per column one block reduction
// gives both the squared norm below the diagonal and the products of that part of the column
// with every later column:  S[c] = sum_{i > j} W[i][j] W[i][c],  so with
// scale = 1 / (alpha - beta) the reflector v = (1, scale W[j+1:, j]) satisfies
// v^T W[j:, c] = W[j][c] + scale S[c].  The reduction goes through an LDS transpose T[c][i]
// (two barriers).  The column loop is unrolled at compile time, so every register index is
// static.  The explicit Q is then accumulated backwards in the same registers.
template <int PM, int NT, int RPT>
__device__ __forceinline__ void hqr_rows(double (&w)[RPT][PM], double* T, double* S, double (*rowjb)[PM],
                                         double* taus, int n, int p)
{
    qr_forward<PM, NT, RPT, 0>(w, T, S, rowjb, taus, n, p);
    // thread 0 wrote the last tau after the last barrier of the forward pass, and the backward
    // pass reads it first
    __syncthreads();
    qr_backward<PM, NT, RPT, PM - 1>(w, T, S, taus, n, p);
}

template <int PM, int NT, int RPT>
__device__ __forceinline__ void load_rows(double (&w)[RPT][PM], const double* __restrict__ In, long off, int n,
                                          int p)
{
    const int i = threadIdx.x;
    if (p == PM) {
        // no padding columns: one block of loads per row
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = i + q * NT;
            const double* src = In + off + (long)(row < n ? row : 0) * PM;
#pragma unroll
            for (int c = 0; c < PM; ++c) w[q][c] = src[c];
            if (row >= n) {
#pragma unroll
                for (int c = 0; c < PM; ++c) w[q][c] = 0.0;
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = i + q * NT;
#pragma unroll
        for (int c = 0; c < PM; ++c) w[q][c] = (row < n && c < p) ? In[off + (long)row * p + c] : 0.0;
    }
}

// The same without a branch per column: every load reads an in-bounds element (row and column
// clamped) and the padding is selected to zero afterwards.
template <int PM, int NT, int RPT>
__device__ __forceinline__ void load_rows_clamped(double (&w)[RPT][PM], const double* __restrict__ In, long off,
                                                  int n, int p)
{
    const int i = threadIdx.x;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = i + q * NT;
        const double* src = In + off + (long)min(row, n - 1) * p;
        const bool ok = row < n;
#pragma unroll
        for (int c = 0; c < PM; ++c) {
            const double v = src[min(c, p - 1)];
            w[q][c] = (ok && c < p) ? v : 0.0;
        }
    }
}

template <int PM, int NT, int RPT>
__device__ __forceinline__ void store_rows(const double (&w)[RPT][PM], double* __restrict__ Out,
                                           float* __restrict__ Out32, long off, int n, int p)
{
    const int i = threadIdx.x;
    if (p == PM) {
        // no padding columns: one block of stores per row (a branch per column makes the
        // compiler wait for every store before the next)
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = i + q * NT;
            if (row < n) {
                double* dst = Out + off + (long)row * PM;
#pragma unroll
                for (int c = 0; c < PM; ++c) dst[c] = w[q][c];
                if (Out32) {
                    float* d32 = Out32 + off + (long)row * PM;
#pragma unroll
                    for (int c = 0; c < PM; ++c) d32[c] = (float)w[q][c];
                }
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = i + q * NT;
        if (row < n) {
#pragma unroll
            for (int c = 0; c < PM; ++c)
                if (c < p) Out[off + (long)row * p + c] = w[q][c];
            if (Out32) {
#pragma unroll
                for (int c = 0; c < PM; ++c)
                    if (c < p) Out32[off + (long)row * p + c] = (float)w[q][c];
            }
        }
    }
}

template <int PM, int NT, int RPT>
__global__ void __launch_bounds__(NT) k_hqr_reg(const double* __restrict__ In, double* __restrict__ Out,
                                                float* __restrict__ Out32, int n, int p, long bs)
{
    In = bshift(In, bs);
    Out = bshift(Out, bs);
    if (Out32) Out32 = bshift(Out32, bs);
    extern __shared__ double T[];
    __shared__ double S[PM];
    __shared__ double rowjb[2][PM];     // row j, double-buffered by column parity
    __shared__ double taus[PM];
    const long off = (long)blockIdx.x * n * p;
    double w[RPT][PM];
    load_rows<PM, NT, RPT>(w, In, off, n, p);
    hqr_rows<PM, NT, RPT>(w, T, S, rowjb, taus, n, p);
    store_rows<PM, NT, RPT>(w, Out, Out32, off, n, p);
}

// ---------------------------------------------------------------------------------------------
// Cholesky QR of the same register-resident block, for orthonormalisations that only need the
// span (the float eps path).  One pass: W = Y^T Y, W = L D L^T, Q = Y L^-T D^-1/2 (the R of
// Y = Q R is D^1/2 L^T, so Q is the thin QR factor with a positive diagonal in R).  A second
// pass on Q restores orthogonality to the rounding level when the first one was conditioned
// worse than the one-pass bound.
//   Gram: every wavefront stages 64 of the rows in LDS and accumulates the 16 x 16 tiles of the
//   lower triangle of W (one tile for p <= 16, three for p <= 32) over them on FP64 MFMA; the
//   per-wavefront tiles are summed in LDS by all threads.
//   LDL^T: wavefront 0, lane i holding row i of W; at step j row j is broadcast lane by lane
//   (readlane), so the step has no LDS round trip.
//   Apply: each thread solves z L^T = y for its rows with L^T read from LDS, then scales by
//   D^-1/2.
// The pivots decide, through s_j = d_j / W_jj (the squared sine of column j against the span of
// the columns before it).  First pass: a pivot with s_j < floor is raised to floor W_jj: such a
// column lies in the span of the earlier ones to rounding (a power step of a subspace whose
// trailing directions are below the Gram's rounding level gives such columns), and the pass
// leaves what remains of it, orthogonal to the earlier columns up to that rounding, with a small
// norm.  All s_j >= one_pass: done; otherwise a second pass.  Second pass: all s_j >= accept2
// (and W_jj > 0): its result is the factor.  Columns below that are, after the first pass,
// rounding noise inside the span of the others: they are replaced by fixed pseudo-random
// columns (an arbitrary completion of the span, as the Householder QR would make one) and a
// third pass orthonormalises the block, again requiring all s_j >= accept2.  If it does not
// pass, the block is reloaded and the Householder QR above runs instead.  Every pass multiplies
// by an invertible triangle, so the span of the columns that carry information is Y's.
template <int PM>
__device__ __forceinline__ int stage_index(int row, int c)
{
    // p = 32: the halves of odd rows are swapped, so that the four rows one MFMA operand read
    // touches do not fall on the same LDS banks
    if constexpr (PM == 32) return row * 32 + (c ^ ((row & 1) << 4));
    else return row * PM + c;
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / d to about one ulp without the IEEE division sequence: hardware reciprocal and two Newton
// steps (d > 0)
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

template <int PM, int NT, int RPT>
__global__ void __launch_bounds__(NT) k_cholqr_reg(const double* __restrict__ In, double* __restrict__ Out,
                                                   float* __restrict__ Out32, int n, int p, double floor,
                                                   double one_pass, double accept2, long bs)
{
    constexpr int NW = NT / 64;
    constexpr int NTILE = PM <= 16 ? 1 : 3;     // (0,0), (1,0), (1,1)
    In = bshift(In, bs);
    Out = bshift(Out, bs);
    if (Out32) Out32 = bshift(Out32, bs);
    extern __shared__ double T[];               // NT x PM doubles: staging, then tile partials
    __shared__ double Ws[PM][PM + 1];           // W, lower triangle and mirror
    __shared__ double LT[PM][PM + 1];           // LT[k][j] = L[j][k], j > k
    __shared__ double rsd[PM];                  // d_j^-1/2
    __shared__ unsigned decision_s[2];          // decision, columns to replace
    __shared__ double S[PM];
    __shared__ double rowjb[2][PM];
    __shared__ double taus[PM];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long off = (long)blockIdx.x * n * p;
    double y[RPT][PM];
    load_rows<PM, NT, RPT>(y, In, off, n, p);
    double* stg = T + wv * 64 * PM;
    bool householder = false;

    // decisions: 0 done, 1 solve and take another pass, 2 Householder, 3 replace the columns in
    // decision_s[1] (numerically inside the span of the others) and take another pass
    for (int pass = 0; pass < 3; ++pass) {
        // ---- Gram of the NT RPT rows on MFMA, per wavefront over its own rows
        f64x4 acc[NTILE];
#pragma unroll
        for (int t = 0; t < NTILE; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
#pragma unroll
            for (int c = 0; c < PM; c += 2)
                *reinterpret_cast<double2*>(stg + stage_index<PM>(lane, c)) = double2{y[q][c], y[q][c + 1]};
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int ks = 0; ks < 64; ks += 4) {
                const int row = ks + (lane >> 4), c0 = lane & 15;
                const double a0 = (c0 < PM) ? stg[stage_index<PM>(row, c0 < PM ? c0 : 0)] : 0.0;
                if constexpr (NTILE == 1) {
                    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, acc[0], 0, 0, 0);
                } else {
                    const int c1 = 16 + c0;
                    const double a1 = (c1 < PM) ? stg[stage_index<PM>(row, c1 < PM ? c1 : 0)] : 0.0;
                    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a0, acc[1], 0, 0, 0);
                    acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, acc[2], 0, 0, 0);
                }
            }
            // the next round's staging (or the partials below) overwrite rows just read
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // tile t, entry (i, j) (i = 4 v + lane / 16, j = lane % 16) of this wavefront
#pragma unroll
        for (int t = 0; t < NTILE; ++t) {
            stg[t * 256 + (0 + (lane >> 4)) * 16 + (lane & 15)] = acc[t][0];
            stg[t * 256 + (4 + (lane >> 4)) * 16 + (lane & 15)] = acc[t][1];
            stg[t * 256 + (8 + (lane >> 4)) * 16 + (lane & 15)] = acc[t][2];
            stg[t * 256 + (12 + (lane >> 4)) * 16 + (lane & 15)] = acc[t][3];
        }
        __syncthreads();
        for (int e = tid; e < PM * PM; e += NT) {
            const int i = e / PM, j = e - (e / PM) * PM;
            if (i < j) continue;
            const int t = (i < 16) ? 0 : (j < 16 ? 1 : 2);
            const int x = (i & 15) * 16 + (j & 15);
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < NW; ++u) v += T[u * 64 * PM + t * 256 + x];
            if (i >= p) v = (i == j) ? 1.0 : 0.0;     // padding columns: identity block
            Ws[i][j] = v;
            Ws[j][i] = v;
        }
        __syncthreads();
        // ---- LDL^T in wavefront 0: lane i holds row i; lane j tests and floors its own pivot
        if (wv == 0) {
            double wr[PM];
#pragma unroll
            for (int c = 0; c < PM; ++c) wr[c] = (lane < PM) ? Ws[lane < PM ? lane : 0][c] : 0.0;
            const double w0 = (lane < PM) ? Ws[lane < PM ? lane : 0][lane < PM ? lane : 0] : 1.0;
            // pivot tests without divisions: d >= t W_jj (false for NaN)
            bool weak = false, bad = false;
            double mydiag = 1.0;
#pragma unroll
            for (int j = 0; j < PM; ++j) {
                // lane j's candidate pivot (the other lanes' values are not used)
                const double draw = wr[j];
                const double cand = (pass > 0 || draw >= floor * w0) ? draw : floor * w0;
                if (lane == j) {
                    // a zero column (W_jj = 0) is weak too: the second pass replaces it
                    weak = !(draw >= one_pass * w0) || !(w0 > 0.0);
                    bad = !(draw >= accept2 * w0) || !(w0 > 0.0);
                    mydiag = cand;
                }
                const double djj = read_lane(cand, j);
                const double inv = djj > 0.0 ? recip(djj) : 0.0;
                // lanes <= j take l = 0 and keep their row (no branch; rows <= j are final)
                const double l = (lane > j) ? wr[j] * inv : 0.0;
#pragma unroll
                for (int k = j + 1; k < PM; ++k) wr[k] = fma(-l, read_lane(wr[k], j), wr[k]);
                wr[j] = (lane > j) ? l : wr[j];
                __builtin_amdgcn_sched_barrier(0);     // one step's broadcasts live at a time
            }
            const unsigned long long weak_m = __ballot(weak && lane < PM);
            const unsigned long long bad_m = __ballot(bad && lane < PM);
            if (lane < PM) {
#pragma unroll
                for (int k = 0; k < PM; ++k)
                    if (k < lane) LT[k][lane] = wr[k];
                rsd[lane] = mydiag > 0.0 ? 1.0 / sqrt(mydiag) : 0.0;
            }
            if (lane == 0) {
                unsigned v;
                if (pass == 0) v = weak_m ? 1u : 0u;
                else if (pass == 1) v = bad_m ? 3u : 0u;
                else v = bad_m ? 2u : 0u;
                decision_s[0] = v;
                decision_s[1] = (unsigned)bad_m;
            }
        }
        __syncthreads();
        const unsigned decision = decision_s[0];
        if (decision == 2) {
            householder = true;
            break;
        }
        if (decision == 3) {
            // complete the span with fixed pseudo-random columns in place of the dependent ones
            const unsigned repl = decision_s[1];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int row = tid + q * NT;
#pragma unroll
                for (int c = 0; c < PM; ++c)
                    if ((repl >> c) & 1u)
                        y[q][c] = row < n ? start_value(((unsigned long long)blockIdx.x << 40) ^
                                                        ((unsigned long long)row << 20) ^ (unsigned long long)c)
                                          : 0.0;
            }
            __syncthreads();
            continue;
        }
        // ---- z L^T = y, then z D^-1/2; row k + 1 of L^T is loaded while row k is applied (where
        // the registers allow)
        if constexpr (RPT * PM > 24) {
#pragma unroll
            for (int k = 0; k < PM; ++k) {
#pragma unroll
                for (int j = k + 1; j < PM; ++j) {
                    const double l = LT[k][j];
#pragma unroll
                    for (int q = 0; q < RPT; ++q) y[q][j] = fma(-y[q][k], l, y[q][j]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            double cur[PM];
#pragma unroll
            for (int j = 1; j < PM; ++j) cur[j] = LT[0][j];
#pragma unroll
            for (int k = 0; k < PM; ++k) {
                double nxt[PM];
#pragma unroll
                for (int j = k + 2; j < PM; ++j) nxt[j] = LT[k + 1][j];
#pragma unroll
                for (int j = k + 1; j < PM; ++j) {
#pragma unroll
                    for (int q = 0; q < RPT; ++q) y[q][j] = fma(-y[q][k], cur[j], y[q][j]);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int j = k + 2; j < PM; ++j) cur[j] = nxt[j];
            }
        }
#pragma unroll
        for (int j = 0; j < PM; ++j) {
            const double sc = rsd[j];
#pragma unroll
            for (int q = 0; q < RPT; ++q) y[q][j] *= sc;
        }
        // (unconditional, so that the solve and its loads share one block) a further pass
        // restages these rows and rewrites Ws / LT / rsd
        __syncthreads();
        if (decision == 0) break;
    }
    if (householder) {
        load_rows<PM, NT, RPT>(y, In, off, n, p);
        hqr_rows<PM, NT, RPT>(y, T, S, rowjb, taus, n, p);
    }
    store_rows<PM, NT, RPT>(y, Out, Out32, off, n, p);
}

// ---------------------------------------------------------------------------------------------
// Two-sided Jacobi on a p x p symmetric matrix (p <= JW_PMAX) by one work-group, parallel
// round-robin ordering.  In every step each 2 x 2 block (P, Q) of the pair partition is replaced
// by J_P^T B J_Q (upper blocks, mirrored), the diagonal blocks by the closed form
// (a_pp - t a_pq, a_qq + t a_pq, 0), and the rows of V by V J.  Stops when
// off(H) <= max(tol, p u) ||H||_F or after max_sweeps sweeps.
constexpr int JW_PMAX = 32;
constexpr int JW_NP = JW_PMAX / 2;                          // pairs per step
constexpr int JW_NBLK = JW_NP * (JW_NP + 1) / 2;            // 2 x 2 blocks (P <= Q)
// Sum over the NTJ threads of a work-group (one wavefront, or four through LDS), the same value in
// every thread.
template <int NTJ>
__device__ __forceinline__ double jw_sum(double v, double* red)
{
    v = wave_sum(v);
    if constexpr (NTJ == 64) {
        return v;
    } else {
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        return (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Rotation of the pair (a, b) of the symmetric matrix H (row stride JW_PMAX + 1): t = tan of the
// smaller angle that annihilates h_ab, c = cos, s = sin; (1, 0, 0) when h_ab = 0 or b is the
// padding index.  The quotients use the hardware reciprocal and reciprocal square root with
// Newton steps (about one ulp).
__device__ __forceinline__ void jw_rotation(const double (*H)[JW_PMAX + 1], int a, int b, int p, double& c,
                                            double& sn, double& t)
{
    c = 1.0; sn = 0.0; t = 0.0;
    if (b >= p) return;
    const double apq = H[a][b];
    if (apq == 0.0) return;
    const double d = H[b][b] - H[a][a];
    const double den = fabs(d) + sqrt(d * d + 4.0 * apq * apq);
    t = 2.0 * apq * recip(den);
    if (d < 0.0) t = -t;
    const double x = 1.0 + t * t;
    double rs = __builtin_amdgcn_rsq(x);
    rs = rs * fma(-0.5 * x * rs, rs, 1.5);
    rs = rs * fma(-0.5 * x * rs, rs, 1.5);
    c = rs;
    sn = t * c;
}

// NTJ threads (64: one wavefront; 256: the 2 x 2 blocks and the rows of V spread over four).
// H is double-buffered: a step reads the rotations' entries and its blocks from one copy and
// writes every entry of its blocks to the other, so each thread forms the rotations it needs
// itself and a step takes one barrier.
template <int NTJ>
__global__ void __launch_bounds__(NTJ) k_jacobi_w(const double* __restrict__ Hin, long sH, int p, int r,
                                                  double* __restrict__ Vs, long sV, int ldv, double* __restrict__ lam,
                                                  long sLam, int max_sweeps, double tol, long bs)
{
    constexpr int JW_BPL = (JW_NBLK + NTJ - 1) / NTJ;      // blocks per thread
    constexpr int JW_VG = NTJ / 32;                        // thread groups over the rows of V
    constexpr int JW_VPL = (JW_NP + JW_VG - 1) / JW_VG;    // V pairs per thread
    __shared__ double red[4];
    Hin = bshift(Hin, bs);
    Vs = bshift(Vs, bs);
    lam = bshift(lam, bs);
    __shared__ double Hb[2][JW_PMAX][JW_PMAX + 1];
    __shared__ double V[JW_PMAX][JW_PMAX + 1];
    __shared__ unsigned char pairs[JW_PMAX - 1][JW_NP][2];   // round-robin pairs (a < b) of every step
    __shared__ unsigned char blk[JW_NBLK][2];
    __shared__ int rank_of[JW_PMAX];
    const int lane = threadIdx.x;     // thread index (not only within a wavefront)
    const double* Hp = Hin + (long)blockIdx.x * sH;
    for (int e = lane; e < p * p; e += NTJ) {
        const int i = e / p, j = e - (e / p) * p;
        Hb[0][i][j] = 0.5 * (Hp[(long)i * p + j] + Hp[(long)j * p + i]);
        V[i][j] = (i == j) ? 1.0 : 0.0;
    }
    const int m = p + (p & 1);
    const int np = m / 2;
    const int nblk = np * (np + 1) / 2;
    for (int e = lane; e < (m - 1) * np; e += NTJ) {
        const int step = e / np, k = e - (e / np) * np;
        int a, bb;
        if (k == 0) { a = m - 1; bb = step; }
        else { a = (step + k) % (m - 1); bb = (step - k + (m - 1)) % (m - 1); }
        if (a > bb) { const int q = a; a = bb; bb = q; }
        pairs[step][k][0] = (unsigned char)a;
        pairs[step][k][1] = (unsigned char)bb;
    }
    if (lane == 0) {
        int e = 0;
        for (int P = 0; P < np; ++P)
            for (int Q = P; Q < np; ++Q, ++e) { blk[e][0] = (unsigned char)P; blk[e][1] = (unsigned char)Q; }
    }
    __syncthreads();
    int cur = 0;
    double f = 0.0;
    for (int e = lane; e < p * p; e += NTJ) {
        const double x = Hb[0][e / p][e - (e / p) * p];
        f += x * x;
    }
    const double fro = sqrt(jw_sum<NTJ>(f, red));
    tol = fmax(tol, (double)p * 2.220446049250313e-16);
    double prev_off = INFINITY;

    for (int sweep = 0; sweep < max_sweeps && p > 1; ++sweep) {
        double o = 0.0;
        for (int e = lane; e < p * p; e += NTJ) {
            const int i = e / p, j = e - (e / p) * p;
            if (i != j) o += Hb[cur][i][j] * Hb[cur][i][j];
        }
        const double off = sqrt(jw_sum<NTJ>(o, red));
        if (off <= tol * fro) break;
        // at the rounding floor (eigenvalues below u ||H|| keep off(H) near p u ||H||): a sweep
        // that no longer halves off(H) once it is below 1e-12 ||H|| changes nothing that matters
        if (off <= 1e-12 * fro && off > 0.5 * prev_off) break;
        prev_off = off;
        for (int step = 0; step < m - 1; ++step) {
            const double (*Hc)[JW_PMAX + 1] = Hb[cur];
            double (*Hn)[JW_PMAX + 1] = Hb[cur ^ 1];
            // ---- 2 x 2 blocks (P <= Q): rotations and entries from Hc, every entry to Hn
#pragma unroll
            for (int u = 0; u < JW_BPL; ++u) {
                const int e = lane + NTJ * u;
                if (e >= nblk) continue;
                const int P = blk[e][0], Q = blk[e][1];
                const int ia = pairs[step][P][0], ib = pairs[step][P][1];
                const int ja = pairs[step][Q][0], jb = pairs[step][Q][1];
                const bool rb = ib < p, cb = jb < p;
                double cP, sP, tP;
                jw_rotation(Hc, ia, ib, p, cP, sP, tP);
                const double x00 = Hc[ia][ja];
                const double x01 = cb ? Hc[ia][jb] : 0.0;
                const double x10 = rb ? Hc[ib][ja] : 0.0;
                const double x11 = (rb && cb) ? Hc[ib][jb] : 0.0;
                if (P == Q) {
                    if (rb) {
                        // closed form on the diagonal block: (a_pp - t a_pq, a_qq + t a_pq, 0)
                        const bool rot = tP != 0.0;
                        Hn[ia][ia] = rot ? x00 - tP * x01 : x00;
                        Hn[ib][ib] = rot ? x11 + tP * x01 : x11;
                        Hn[ia][ib] = rot ? 0.0 : x01;
                        Hn[ib][ia] = rot ? 0.0 : x01;
                    } else {
                        Hn[ia][ia] = x00;
                    }
                } else {
                    double cQ, sQ, tQ;
                    jw_rotation(Hc, ja, jb, p, cQ, sQ, tQ);
                    // rows: J_P^T [x0; x1]; columns: [y.0 y.1] J_Q
                    const double y00 = cP * x00 - sP * x10, y10 = sP * x00 + cP * x10;
                    const double y01 = cP * x01 - sP * x11, y11 = sP * x01 + cP * x11;
                    const double z00 = cQ * y00 - sQ * y01, z01 = sQ * y00 + cQ * y01;
                    const double z10 = cQ * y10 - sQ * y11, z11 = sQ * y10 + cQ * y11;
                    Hn[ia][ja] = z00; Hn[ja][ia] = z00;
                    if (cb) { Hn[ia][jb] = z01; Hn[jb][ia] = z01; }
                    if (rb) { Hn[ib][ja] = z10; Hn[ja][ib] = z10; }
                    if (rb && cb) { Hn[ib][jb] = z11; Hn[jb][ib] = z11; }
                }
            }
            // ---- rows of V (row = lane % 32, pairs of one parity): each entry has one owner
            const int vrow = lane & 31, vhalf = lane >> 5;
#pragma unroll
            for (int u = 0; u < JW_VPL; ++u) {
                const int kk = vhalf + JW_VG * u;
                if (kk >= np || vrow >= p) continue;
                const int va = pairs[step][kk][0], vb = pairs[step][kk][1];
                if (vb >= p) continue;
                double c, sn, t;
                jw_rotation(Hc, va, vb, p, c, sn, t);
                const double vx = V[vrow][va], vy = V[vrow][vb];
                V[vrow][va] = c * vx - sn * vy;
                V[vrow][vb] = sn * vx + c * vy;
            }
            cur ^= 1;
            __syncthreads();
        }
    }
    const double (*H)[JW_PMAX + 1] = Hb[cur];
    // stable descending ranks
    if (lane < p) {
        const double d = H[lane][lane];
        int rk = 0;
        for (int i = 0; i < p; ++i) {
            const double e = H[i][i];
            if (e > d || (e == d && i < lane)) ++rk;
        }
        rank_of[lane] = rk;
    }
    __syncthreads();
    double* Vo = Vs + (long)blockIdx.x * sV;
    for (int e = lane; e < p * p; e += NTJ) {
        const int i = e / p, j = e - (e / p) * p;
        const int rk = rank_of[j];
        if (rk < r) Vo[(long)i * ldv + rk] = V[i][j];
    }
    if (lane < p && rank_of[lane] < r) lam[(long)blockIdx.x * sLam + rank_of[lane]] = H[lane][lane];
}

// Sign rule on the n x r factor of problem blockIdx.y, column blockIdx.x.
__global__ void __launch_bounds__(256) k_signfix(double* __restrict__ U, long sU, int ldu, int n, long bs)
{
    U = bshift(U, bs);
    __shared__ double red[4];
    __shared__ int redi[4];
    __shared__ double amax_s;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double* u = U + blockIdx.y * sU + blockIdx.x;
    double m = 0.0;
    for (int i = tid; i < n; i += 256) m = fmax(m, fabs(u[(long)i * ldu]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (tid == 0) amax_s = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    const double thr = amax_s * (1.0 - 1e-10);
    int lead = 0x7fffffff;
    for (int i = tid; i < n; i += 256)
        if (fabs(u[(long)i * ldu]) >= thr && i < lead) lead = i;
    for (int o = 32; o > 0; o >>= 1) lead = min(lead, __shfl_xor(lead, o, 64));
    if (lane == 0) redi[wv] = lead;
    __syncthreads();
    int L = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
    // every thread reads the leading entry before any thread negates it
    const bool flip = L < n && u[(long)L * ldu] < 0.0;
    __syncthreads();
    if (flip)
        for (int i = tid; i < n; i += 256) u[(long)i * ldu] = -u[(long)i * ldu];
}

// Sign rule on column blockIdx.x of U (n rows, ld ldu); the same flip is applied to column
// blockIdx.x of V (nv rows, ld ldv).
__global__ void __launch_bounds__(256) k_signfix_pair(double* __restrict__ U, int ldu, int n, double* __restrict__ V,
                                                      int ldv, int nv, long bs)
{
    U = bshift(U, bs);
    V = bshift(V, bs);
    __shared__ double red[4];
    __shared__ int redi[4];
    __shared__ double amax_s;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double* u = U + blockIdx.x;
    double m = 0.0;
    for (int i = tid; i < n; i += 256) m = fmax(m, fabs(u[(long)i * ldu]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (tid == 0) amax_s = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    const double thr = amax_s * (1.0 - 1e-10);
    int lead = 0x7fffffff;
    for (int i = tid; i < n; i += 256)
        if (fabs(u[(long)i * ldu]) >= thr && i < lead) lead = i;
    for (int o = 32; o > 0; o >>= 1) lead = min(lead, __shfl_xor(lead, o, 64));
    if (lane == 0) redi[wv] = lead;
    __syncthreads();
    const int L = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
    // every thread reads the leading entry before any thread negates it
    const bool flip = L < n && u[(long)L * ldu] < 0.0;
    __syncthreads();
    if (flip) {
        for (int i = tid; i < n; i += 256) u[(long)i * ldu] = -u[(long)i * ldu];
        for (int i = tid; i < nv; i += 256) V[(long)i * ldv + blockIdx.x] = -V[(long)i * ldv + blockIdx.x];
    }
}

// Convergence test of the Ritz pairs (lam_j, u_j), j < r, of each problem:
// rho_j = ||G u_j - lam_j u_j||_2 against max(tau lam_j, cfloor sqrt(n) u ||G||_F), u the FP64
// unit roundoff.  The first term asks converged vectors of the large eigenvalues; below
// cfloor sqrt(n) u ||G||_F / tau the test falls back to the rounding level of the product
// G u itself, which no further iteration can go below.  flags[problem] = 1 when every column
// passes (a NaN fails).
// Two kernels.  k_eig_resid_part: work-group (problem, rb) takes rows rb*64 .. rb*64+63 of
// G u (lane = row; the four waves split k into quarters, added in wave order), and writes
// per column the sum over its rows of (G u - lam u)^2 and, in slot EIG_CHECK_COLS, its part of
// ||G||_F^2 (G symmetric, so lane i reads column i of row k: coalesced).  k_eig_resid_flags
// adds the parts in row-block order and applies the test, so the outcome does not depend on
// scheduling.
constexpr int RES_CB = 8;
__global__ void __launch_bounds__(256) k_eig_resid_part(const double* __restrict__ G, long sG, int n,
                                                        const double* __restrict__ U, long sU, int ldu, int r,
                                                        const double* __restrict__ lam, long sL,
                                                        double* __restrict__ part, long bs)
{
    G = bshift(G, bs);
    U = bshift(U, bs);
    lam = bshift(lam, bs);
    part = bshift(part, bs);
    __shared__ double red[4][64][RES_CB + 1];
    __shared__ double gred[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rb = blockIdx.y;
    const double* g = G + blockIdx.x * sG;
    const double* u = U + blockIdx.x * sU;
    const double* l = lam + blockIdx.x * sL;
    double* pp = part + (long)blockIdx.x * EIG_CHECK_DOUBLES + (long)rb * (EIG_CHECK_COLS + 1);
    const int i = rb * 64 + lane;
    const bool live = i < n;
    const int kq = (n + 3) / 4;
    const int k0 = wv * kq, k1 = min(n, k0 + kq);
    double gs = 0.0;
    for (int c0 = 0; c0 < r; c0 += RES_CB) {
        double y[RES_CB];
#pragma unroll
        for (int j = 0; j < RES_CB; ++j) y[j] = 0.0;
        for (int k = k0; k < k1; ++k) {
            const double gv = live ? g[(long)k * n + i] : 0.0;
            if (c0 == 0) gs = fma(gv, gv, gs);
            const double* uk = u + (long)k * ldu + c0;
#pragma unroll
            for (int j = 0; j < RES_CB; ++j) y[j] = fma(gv, (c0 + j < r) ? uk[j] : 0.0, y[j]);
        }
#pragma unroll
        for (int j = 0; j < RES_CB; ++j) red[wv][lane][j] = y[j];
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int j = 0; j < RES_CB; ++j) {
                const double yy = ((red[0][lane][j] + red[1][lane][j]) + red[2][lane][j]) + red[3][lane][j];
                const int c = c0 + j;
                const double d = (live && c < r) ? yy - l[c] * u[(long)i * ldu + c] : 0.0;
                const double sq = wave_sum(d * d);
                if (lane == 0 && c < r) pp[c] = sq;
            }
        }
        __syncthreads();
    }
    gs = wave_sum(gs);
    if (lane == 0) gred[wv] = gs;
    __syncthreads();
    if (tid == 0) pp[EIG_CHECK_COLS] = (gred[0] + gred[1]) + (gred[2] + gred[3]);
}

__global__ void __launch_bounds__(64) k_eig_resid_flags(const double* __restrict__ part, int n, int r,
                                                        const double* __restrict__ lam, long sL, double tau,
                                                        double cfloor, int* __restrict__ flags, long bs)
{
    part = bshift(part, bs);
    lam = bshift(lam, bs);
    flags = bshift(flags, bs);
    const int lane = threadIdx.x;
    const int nrb = (n + 63) / 64;
    const double* pp = part + (long)blockIdx.x * EIG_CHECK_DOUBLES;
    const double* l = lam + blockIdx.x * sL;
    double g2 = 0.0;
    for (int rb = 0; rb < nrb; ++rb) g2 += pp[(long)rb * (EIG_CHECK_COLS + 1) + EIG_CHECK_COLS];
    const double floor_level = cfloor * sqrt((double)n) * 2.220446049250313e-16 * sqrt(g2);
    int ok = 1;
    for (int c = lane; c < r; c += 64) {
        double s2 = 0.0;
        for (int rb = 0; rb < nrb; ++rb) s2 += pp[(long)rb * (EIG_CHECK_COLS + 1) + c];
        const double rho = sqrt(s2);
        if (!(rho <= fmax(tau * l[c], floor_level))) ok = 0;
    }
    for (int o = 32; o > 0; o >>= 1) ok = min(ok, __shfl_xor(ok, o, 64));
    if (lane == 0) flags[blockIdx.x] = ok;
}

__global__ void k_trace(const double* __restrict__ G, long sG, int n, double* __restrict__ out, long sOut, long bs)
{
    G = bshift(G, bs);
    out = bshift(out, bs);
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const double* g = G + blockIdx.x * sG;
    double s = 0.0;
    for (int i = tid; i < n; i += 256) s += g[(long)i * n + i];
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) out[blockIdx.x * sOut] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

// out32 (optional, register kernels only): an FP32 copy of the factor, same layout.
// chol.floor > 0 (register sizes only): Cholesky QR with these thresholds and the Householder
// fallback; the factor then spans the same space, with R's diagonal positive where the Cholesky
// route is taken.
static hipError_t qr_launch(const double* in, double* out, int count, int n, int p, hipStream_t s, Bat bt,
                            float* out32 = nullptr, CholQr chol = CholQr{})
{
    const dim3 grid(count, 1, bt.nb);
    if (n <= 1024 && p <= 32) {
        const int nt = n <= 256 ? 256 : 512;     // rows per thread: 1 up to 512 rows, 2 above
        const bool two = n > 512;
        const int pm = (p + 7) / 8 * 8;
        const size_t lds = sizeof(double) * (size_t)pm * nt;
        // Cholesky QR up to 256 rows (one per thread), and up to 512 for p <= 24: the larger
        // register blocks spill
        const bool use_chol = chol.floor > 0.0 && (n <= 256 || (n <= 512 && pm <= 24));
#define TK_QR_LAUNCH3(K, PM, NT, RPT, ...)                                                                     \
    hipLaunchKernelGGL((K<PM, NT, RPT>), grid, dim3(NT), lds, s, in, out, out32, n, p, ##__VA_ARGS__, bt.bs)
#define TK_CHOL_LAUNCH(PM, NT) TK_QR_LAUNCH3(k_cholqr_reg, PM, NT, 1, chol.floor, chol.one_pass, chol.accept2)
#define TK_QR_LAUNCH(PM)                                                                                         \
    do {                                                                                                        \
        if (nt == 256) TK_QR_LAUNCH3(k_hqr_reg, PM, 256, 1);                                                    \
        else if (!two) TK_QR_LAUNCH3(k_hqr_reg, PM, 512, 1);                                                    \
        else TK_QR_LAUNCH3(k_hqr_reg, PM, 512, 2);                                                              \
    } while (0)
        if (use_chol) {
            switch (pm) {
            case 8: if (nt == 256) TK_CHOL_LAUNCH(8, 256); else TK_CHOL_LAUNCH(8, 512); break;
            case 16: if (nt == 256) TK_CHOL_LAUNCH(16, 256); else TK_CHOL_LAUNCH(16, 512); break;
            case 24: if (nt == 256) TK_CHOL_LAUNCH(24, 256); else TK_CHOL_LAUNCH(24, 512); break;
            default: TK_CHOL_LAUNCH(32, 256);
            }
        } else {
            switch (pm) {
            case 8: TK_QR_LAUNCH(8); break;
            case 16: TK_QR_LAUNCH(16); break;
            case 24: TK_QR_LAUNCH(24); break;
            default: TK_QR_LAUNCH(32);
            }
        }
#undef TK_QR_LAUNCH
#undef TK_CHOL_LAUNCH
#undef TK_QR_LAUNCH3
        return hipGetLastError();
    }
    if (out32) return hipErrorInvalidValue;
    size_t bytes = (size_t)n * p * sizeof(double);
    int in_lds = bytes <= QR_LDS_BYTES ? 1 : 0;
    hipLaunchKernelGGL(k_hqr, grid, dim3(256), in_lds ? bytes : 0, s, in, out, n, p, in_lds, bt.bs);
    return hipGetLastError();
}

// Jacobi on `count` p x p matrices (stride sH) -> leading r eigenvectors (stride sV, ld ldv)
// tol: the stopping threshold on off(H) / ||H||_F (0: 1e-15)
static hipError_t jacobi_launch(const double* H, long sH, int count, int p, int r, double* V, long sV, int ldv,
                                double* lam, long sL, hipStream_t s, Bat bt, double tol = 0.0)
{
    const dim3 grid(count, 1, bt.nb);
    if (!(tol > 0.0)) tol = 1e-15;
    if (p <= JW_PMAX) {
        hipLaunchKernelGGL(k_jacobi_w<256>, grid, dim3(256), 0, s, H, sH, p, r, V, sV, ldv, lam, sL, 60, tol, bt.bs);
        return hipGetLastError();
    }
    if (sH != (long)p * p || sV != (long)p * r || ldv != r) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi, grid, dim3(256), 0, s, H, p, r, V, lam, sL, 60, tol, bt.bs);
    return hipGetLastError();
}

hipError_t launch_signfix_pair(double* U, int ldu, int n, double* V, int ldv, int nv, int r, hipStream_t s, Bat bt)
{
    hipLaunchKernelGGL(k_signfix_pair, dim3(r, 1, bt.nb), dim3(256), 0, s, U, ldu, n, V, ldv, nv, bt.bs);
    return hipGetLastError();
}

hipError_t eig_set_attributes()
{
    hipError_t e = hipFuncSetAttribute((const void*)k_hqr, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)QR_LDS_BYTES);
    if (e != hipSuccess) return e;
    // dynamic LDS of the register QR above 64 KB: PM x 512 doubles
    const void* ks[] = {(const void*)k_hqr_reg<24, 512, 1>, (const void*)k_hqr_reg<32, 512, 1>,
                        (const void*)k_hqr_reg<24, 512, 2>, (const void*)k_hqr_reg<32, 512, 2>,
                        (const void*)k_cholqr_reg<24, 512, 1>};
    const int bytes[] = {(int)(sizeof(double) * 24 * 512), (int)(sizeof(double) * 32 * 512),
                         (int)(sizeof(double) * 24 * 512), (int)(sizeof(double) * 32 * 512),
                         (int)(sizeof(double) * 24 * 512)};
    for (int i = 0; i < 5; ++i)
        if ((e = hipFuncSetAttribute(ks[i], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[i])) != hipSuccess)
            return e;
    return hipSuccess;
}

static hipError_t eig_body(const EigBatch& b, int iters, hipStream_t s, bool& wrote32)
{
    hipError_t e;
    const int n = b.n, p = b.p, r = b.r;
    const long np_ = (long)n * p;
    Bat bt;
    bt.nb = b.nb > 1 ? b.nb : 1;
    bt.bs = b.bs;
    if (b.trace) {
        hipLaunchKernelGGL(k_trace, dim3(b.count, 1, bt.nb), dim3(256), 0, s, b.G, b.sG, n, b.trace, b.sTrace, bt.bs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (p == n && p <= JW_PMAX) {
        // the block is the identity: diagonalise G itself
        if ((e = jacobi_launch(b.G, b.count > 1 ? b.sG : 0, b.count, p, r, b.U, b.sU, b.ldu, b.lam, b.sL, s, bt,
                               b.jacobi_tol)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_signfix, dim3(r, b.count, bt.nb), dim3(256), 0, s, b.U, b.sU, b.ldu, n, bt.bs);
        return hipGetLastError();
    }
    // start block: a warm block of exactly p columns is read in place by the first product
    const bool warm_direct = b.warm && b.rw == p && p < n && iters > 0;
    if (!warm_direct) {
        hipLaunchKernelGGL(k_eig_init, dim3((unsigned)((np_ + 255) / 256), b.count, bt.nb), dim3(256), 0, s, b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    GemmArgs gq{};   // Y = G Q
    gq.M = n; gq.N = p; gq.K = n; gq.batch = b.count;
    gq.A = b.G; gq.sAb = b.sG; gq.sAm = n; gq.sAk = 1;
    gq.B = b.Q; gq.sBb = np_; gq.sBk = p; gq.sBn = 1;
    gq.C = b.Y; gq.sCb = np_; gq.sCm = p; gq.sCn = 1;
    gq.alpha = 1.0; gq.beta = 0.0;
    gq.nb = bt.nb; gq.bs = bt.bs;
    if (p < n) {
        const bool start_orthonormal = b.warm && b.rw == p;   // previous factor, no extra columns
        // a span-only iteration needs no orthonormal start: G times the random block spans the
        // same space as G times its orthonormalisation, and every iteration ends with a QR
        const bool skip_start_qr = b.span_only && !b.warm && iters > 0;
        if (!start_orthonormal && !skip_start_qr && (e = qr_launch(b.Q, b.Q, b.count, n, p, s, bt)) != hipSuccess)
            return e;
        // span-only with a compact U: the last QR writes the factor itself
        const bool direct = b.span_only && p == r && iters > 0 && b.ldu == p && (b.count == 1 || b.sU == np_);
        // the FP32 copy comes out of the last QR when it writes the factor in place
        const bool direct32 = direct && b.U32 && p <= 32 && n <= 1024;   // U32 strided like U (n p)
        for (int it = 0; it < iters; ++it) {
            GemmArgs g = gq;
            if (it == 0 && warm_direct) { g.B = b.warm; g.sBb = b.sW; g.sBk = b.ldw; g.sBn = 1; }
            if ((e = launch_gemm<double, double, double>(g, s)) != hipSuccess) return e;
            const bool last = direct && it == iters - 1;
            // span-only: Cholesky QR once the block is a power step of an orthonormal one (G times
            // a random block has all its columns close to the leading eigenvector)
            const CholQr chol = (b.span_only && (b.warm || it > 0)) ? b.cholqr : CholQr{};
            if ((e = qr_launch(b.Y, last ? b.U : b.Q, b.count, n, p, s, bt, last && direct32 ? b.U32 : nullptr,
                               chol)) != hipSuccess)
                return e;
        }
        if (direct) {
            wrote32 = direct32;
            return hipSuccess;
        }
    }
    if (b.span_only) {
        // the block spans G^iters W: hand it over as the factor (ld p == r)
        if (!(p == r && p < n && iters > 0)) return hipErrorInvalidValue;
        if (b.ldu == p && (b.count == 1 || b.sU == np_))
            return launch_copy_f64(b.Q, b.U, b.count * np_, s, bt);
        if (b.ldu == p) {
            for (long c = 0; c < b.count; ++c)
                if ((e = launch_copy_f64(b.Q + c * np_, b.U + c * b.sU, np_, s, bt)) != hipSuccess) return e;
            return hipSuccess;
        }
        if (bt.nb > 1) return hipErrorInvalidValue;
        for (long c = 0; c < b.count; ++c)
            if ((e = hipMemcpy2DAsync(b.U + c * b.sU, sizeof(double) * b.ldu, b.Q + c * np_, sizeof(double) * p,
                                      sizeof(double) * p, n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
                return e;
        return hipSuccess;
    }
    if ((e = launch_gemm<double, double, double>(gq, s)) != hipSuccess) return e;
    GemmArgs hq{};   // H = Q^T Y  (p x p)
    hq.M = p; hq.N = p; hq.K = n; hq.batch = b.count;
    hq.A = b.Q; hq.sAb = np_; hq.sAm = 1; hq.sAk = p;
    hq.B = b.Y; hq.sBb = np_; hq.sBk = p; hq.sBn = 1;
    hq.C = b.H; hq.sCb = (long)p * p; hq.sCm = p; hq.sCn = 1;
    hq.alpha = 1.0; hq.beta = 0.0;
    hq.nb = bt.nb; hq.bs = bt.bs;
    if ((e = launch_gemm<double, double, double>(hq, s)) != hipSuccess) return e;
    if ((e = jacobi_launch(b.H, (long)p * p, b.count, p, r, b.Vs, (long)p * r, r, b.lam, b.sL, s, bt)) != hipSuccess)
        return e;
    GemmArgs uq{};   // U = Q Vs  (n x r)
    uq.M = n; uq.N = r; uq.K = p; uq.batch = b.count;
    uq.A = b.Q; uq.sAb = np_; uq.sAm = p; uq.sAk = 1;
    uq.B = b.Vs; uq.sBb = (long)p * r; uq.sBk = r; uq.sBn = 1;
    uq.C = b.U; uq.sCb = b.sU; uq.sCm = b.ldu; uq.sCn = 1;
    uq.alpha = 1.0; uq.beta = 0.0;
    uq.nb = bt.nb; uq.bs = bt.bs;
    if ((e = launch_gemm<double, double, double>(uq, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_signfix, dim3(r, b.count, bt.nb), dim3(256), 0, s, b.U, b.sU, b.ldu, n, bt.bs);
    return hipGetLastError();
}

hipError_t launch_qr(const double* in, double* out, int count, int n, int p, hipStream_t s)
{
    if (n < 1 || p < 1 || p > n || p > EIG_PMAX) return hipErrorInvalidValue;
    return qr_launch(in, out, count, n, p, s, Bat());
}

// Column c of the fine factor at node j: the coarse column, read as a function on the uniform
// coarse nodes x0c + i hc, linearly interpolated at x0f + j hf (the same interval).
__global__ void __launch_bounds__(256) k_interp_factor(const double* __restrict__ Uc, int nc, double x0c, double hc,
                                                       double* __restrict__ Uf, int nf, double x0f, double hf, int r)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)nf * r) return;
    const int j = (int)(e / r), c = (int)(e - (long)j * r);
    const double t = ((x0f + j * hf) - x0c) / hc;
    int i = (int)floor(t);
    i = i < 0 ? 0 : (i > nc - 2 ? nc - 2 : i);
    const double w = t - i;
    Uf[e] = (1.0 - w) * Uc[(long)i * r + c] + w * Uc[(long)(i + 1) * r + c];
}

hipError_t launch_interp_factor(const double* Uc, int nc, double x0c, double hc, double* Uf, int nf, double x0f,
                                double hf, int r, hipStream_t s)
{
    if (nc < 2 || nf < 1 || r < 1) return hipErrorInvalidValue;
    const long tot = (long)nf * r;
    hipLaunchKernelGGL(k_interp_factor, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Uc, nc, x0c, hc, Uf,
                       nf, x0f, hf, r);
    return hipGetLastError();
}

hipError_t launch_eig_check(const EigBatch& b, double tau, double cfloor, int* flags, double* part, hipStream_t s)
{
    if (b.n < 1 || b.n > EIG_CHECK_NMAX || b.r < 1 || b.r > EIG_CHECK_COLS) return hipErrorInvalidValue;
    const int nb = b.nb > 1 ? b.nb : 1;
    const int nrb = (b.n + 63) / 64;
    hipLaunchKernelGGL(k_eig_resid_part, dim3(b.count, nrb, nb), dim3(256), 0, s, b.G, b.sG, b.n, b.U, b.sU, b.ldu,
                       b.r, b.lam, b.sL, part, b.bs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eig_resid_flags, dim3(b.count, 1, nb), dim3(64), 0, s, (const double*)part, b.n, b.r, b.lam,
                       b.sL, tau, cfloor, flags, b.bs);
    return hipGetLastError();
}

hipError_t launch_eig(const EigBatch& b, int iters, hipStream_t s)
{
    bool wrote32 = false;
    hipError_t e = eig_body(b, iters, s, wrote32);
    if (e != hipSuccess || !b.U32 || wrote32) return e;
    // FP32 copy of the factor where no kernel of the path wrote it
    if (b.ldu != b.r || (b.count > 1 && b.sU != (long)b.n * b.r)) return hipErrorInvalidValue;
    Bat bt;
    bt.nb = b.nb > 1 ? b.nb : 1;
    bt.bs = b.bs;
    return launch_convert_f64_to_f32(b.U, b.U32, (long)b.count * b.n * b.r, s, bt);
}

}  // namespace tk
