// Host-side launch interface of the gfx950 kernels (one translation unit per kernel family).
// Every launcher enqueues on `s` and returns hipSuccess or the launch error; shapes are
// checked by the callers in tk_api.cpp before anything is launched.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tk_device.h"

namespace tk {

// A launch over nb problems of equal shape whose workspaces lie bs bytes apart (grid z; every
// pointer argument that lies in a workspace moves with the problem).  Each problem runs the
// same work-groups with the same arithmetic as when launched alone.
struct Bat {
    int nb = 1;
    long bs = 0;
};
constexpr int BATCH_MAX = 32;   // problems per batched grid evaluation (parameters passed by value)
struct KernelParamsBatch {
    KernelParams k[BATCH_MAX];
};

// ---------------------------------------------------------------- a1: grid evaluation ----
struct GridAxes {
    int n[3];
    double x0[3];   // first node
    double h[3];    // spacing
};
// kps: bt.nb kernel parameter sets, one per problem (bt.nb <= BATCH_MAX).
hipError_t launch_grid_eval_f32(float* A, const GridAxes& g, const KernelParams* kps, hipStream_t s,
                                Bat bt = Bat());
hipError_t launch_grid_eval_f64(double* A, const GridAxes& g, const KernelParams* kps, hipStream_t s,
                                Bat bt = Bat());

// Radial-table route for Matern orders without a closed form on grids of common spacing h with
// first nodes in (h/2) Z and an isotropic metric: every squared radius is q m for an integer m,
// the kernel is tabulated once per m (T entries, at most radial_table_cap(n)) and the grid
// gathers from the table.  radial_plan fills rg and returns true when the route applies to all
// nb kernels; launch_grid_eval_radial then needs `table`: T doubles per problem (moving by bt.bs
// like A).  Storage esz 4 (float) or 8 (double).
struct RadialGrid {
    double q;      // a (h/2)^2: r^2 = q m
    long T;        // table entries
    int c[3];      // 2 x0_k / h
    int mode;      // m from the index: 4 idx (all c_k even), 8 idx + 3 (all odd), idx
};
long radial_table_cap(const int n[3]);
bool radial_plan(const GridAxes& g, const KernelParams* kps, int nb, RadialGrid* rg);
hipError_t launch_grid_eval_radial(void* A, int esz, const GridAxes& g, const KernelParams* kps, const RadialGrid& rg,
                                   double* table, hipStream_t s, Bat bt = Bat());

// Uneven batches: float grids of any sizes in one persistent launch.  A job is one grid (its
// float tensor A, axes and kernel); its work items are its (n0 + 1) / 2 plane pairs.
// first_item_dev[j] = items of the jobs before j (first_item_dev[njobs] = nitems); *counter_dev
// must be zero when the launch starts.  Values equal launch_grid_eval_f32's for each grid.
struct GridJob {
    float* A;
    GridAxes g;
    KernelParams kp;
    int qpr;
    int sym;
};
GridJob grid_job_f32(float* A, const GridAxes& g, const KernelParams& kp);
int grid_job_items(const GridJob& j);
hipError_t launch_grid_eval_f32_queue(const GridJob* jobs_dev, int njobs, const int* first_item_dev, int nitems,
                                      unsigned* counter_dev, hipStream_t s);

// Kernel-node parameters of the grid evaluation as launch_grid_eval_* would launch it (for
// updating a captured graph); the argument values live in the struct, which must outlive the
// update call.
struct GridEvalNode {
    hipKernelNodeParams p;
    void* args[7];
    void* A;
    GridAxes g;
    KernelParamsBatch kps;
    long total;      // double storage: quads of 4 elements
    int sym;         // float storage: whether rows (i0, i1), (i1, i0) coincide
    int qpr;
    long bs;
};
void grid_eval_node_f32(float* A, const GridAxes& g, const KernelParams* kps, Bat bt, GridEvalNode* nd);
void grid_eval_node_f64(double* A, const GridAxes& g, const KernelParams* kps, Bat bt, GridEvalNode* nd);

// ----------------------------------------------------------------- a2: Gram (SYRK) ----
// G (n_mode x n_mode, double, full) = A_(mode) A_(mode)^T.  `work` must hold
// gram_work_bytes(...) bytes.  nsplit (a "code"): the number of K chunks per tile pair of the
// 64 x 64-tile kernel, or GRAM_BIG + that number for the 128 x 128-tile FP32 kernel (every n a
// multiple of 32, n_mode >= 128), 0 for the default of the shape (gram_default_splits); the
// partial sums of the chunks are added in FP64 in chunk order, so a given code gives the same
// result every time.
constexpr int GRAM_BIG = 1 << 20;
constexpr int GRAM_MAX_CANDIDATES = 8;
int gram_default_splits(const int n[3], int mode, int prec);
// Codes worth timing for the shape (out[0] the default; none needs more workspace than the
// default): returns how many were written (at most GRAM_MAX_CANDIDATES).
int gram_split_candidates(const int n[3], int mode, int prec, int out[GRAM_MAX_CANDIDATES]);
size_t gram_work_bytes(const int n[3], int mode, int prec, int nsplit = 0);
hipError_t launch_gram(const void* A, const int n[3], int mode, int prec, double* G, void* work,
                       hipStream_t s, Bat bt = Bat(), int nsplit = 0);
// The three mode Grams of one tensor (G_k at G + k sG) in one launch plus one reduction launch,
// when every mode takes the large-tile kernel with its split code; the partials of the three
// modes lie back to back in `work` (gram3_work_bytes).  Same results as three launch_gram calls.
bool gram3_eligible(const int n[3], int prec, const int codes[3]);
size_t gram3_work_bytes(const int n[3], int prec, const int codes[3]);
hipError_t launch_gram3(const void* A, const int n[3], int prec, double* G, long sG, void* work, hipStream_t s,
                        Bat bt, const int codes[3]);

// ------------------------------------------------------------ small dense products ----
// C[b](m,n) = alpha * sum_k A[b](m,k) B[b](k,n) + beta * C[b](m,n) with arbitrary element
// strides, FP64 accumulation.  TA/TB/TC in {float, double}.
struct GemmArgs {
    int M, N, K, batch;
    int reduce_batch;   // 1: C = alpha * sum_b A[b] B[b] + beta * C (one output, no C stride)
    const void* A; long sAb, sAm, sAk;
    const void* B; long sBb, sBk, sBn;
    void* C;       long sCb, sCm, sCn;
    double alpha, beta;
    int nb;        // problems (grid z; 0 counts as 1); A, B, C move by bs bytes per problem
    long bs;
};
template <typename TA, typename TB, typename TC>
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);

// ------------------------------------------------------------- a3: eigensolver ----
// `count` problems of equal size: leading r eigenpairs of symmetric n x n matrices G
// (row-major, problem stride sG), with a working block of p columns (r <= p <= min(n, 56)).
// Workspaces (contiguous per problem): Q, Y: n x p; H: p x p; Vs: p x r.
// warm (optional): n x rw start vectors per problem (ld ldw, stride sW).
// Outputs: U (n x r per problem, ld ldu, stride sU), lam (r per problem, stride sL),
// trace (optional, trace(G), stride sTrace).
constexpr int EIG_PMAX = 56;
// Thresholds of the Cholesky QR (squared sines of its pivots): first-pass pivots below floor are
// raised to it; one pass when all are >= one_pass; the second pass needs all >= accept2, else
// the block takes Householder QR.  floor <= 0: Householder only.
struct CholQr {
    double floor = 0.0, one_pass = 1e-4, accept2 = 0.25;
};
struct EigBatch {
    int count, n, p, r, rw, ldw;
    const double* G; long sG;
    const double* warm; long sW;
    double* Q; double* Y; double* H; double* Vs;
    double* U; long sU; int ldu;
    double* lam; long sL;
    double* trace; long sTrace;
    int span_only;   // 1: p == r < n; U = orthonormal basis of span(G^iters W) (W the warm block or a
                     // random one), no Rayleigh-Ritz (for callers that rotate the factors afterwards)
    int nb;          // batched problems (0 counts as 1): every pointer above moves by bs bytes
    long bs;
    float* U32;      // optional FP32 copy of U (ld r, stride n r); written by the last QR where it
                     // writes U itself, by a conversion otherwise; moves by bs like the others
    CholQr cholqr;   // span-only: orthonormalise by Cholesky QR when cholqr.floor > 0
    double jacobi_tol;   // p == n: Jacobi stops at off(H) <= jacobi_tol ||H||_F (0: 1e-15)
};
hipError_t launch_eig(const EigBatch& b, int iters, hipStream_t s);
// Convergence test of the r Ritz pairs (lam, U) of each problem of b against its G:
// flags[c] (c < count, moving by bs per batched problem) = 1 when every column has
// ||G u_j - lam_j u_j|| <= max(tau lam_j, cfloor sqrt(n) u ||G||_F), else 0.  n <= 1024,
// r <= 48; `part` holds count * EIG_CHECK_DOUBLES doubles of partial sums (moving by bs).
constexpr int EIG_CHECK_NMAX = 1024;
constexpr int EIG_CHECK_COLS = 48;
constexpr int EIG_CHECK_DOUBLES = (EIG_CHECK_NMAX / 64) * (EIG_CHECK_COLS + 1);
hipError_t launch_eig_check(const EigBatch& b, double tau, double cfloor, int* flags, double* part, hipStream_t s);
// ------------------------------------------- separable covariance (rank-1 Kronecker) ----
// C (n x n, row-major) = k(|x_i - x_j|) + nugget on the diagonal, x_i = x0 + i h.
hipError_t launch_cov1d(double* C, int n, double x0, double h, const KernelParams& kp, double nugget, hipStream_t s);
// In-place Cholesky A = L L^T (lower triangle, strict upper zeroed); `work` holds
// cholesky_work_bytes(n); *info (device, zero on entry) = index + 1 of the first pivot <= 0.
size_t cholesky_work_bytes(int n);
hipError_t launch_cholesky(double* A, int n, void* work, int* info, hipStream_t s);
// out[0] = 2 sum log L_ii;  X = L^-1 (lower-triangular, n x n)
hipError_t launch_logdet_chol(const double* L, int n, double* out, hipStream_t s);
// work: 64 x n doubles
hipError_t launch_trinv(const double* L, int n, double* X, double* work, hipStream_t s);

// Householder QR of `count` n x p row-major blocks (consecutive): out = the explicit orthonormal
// factor (in == out allowed).  p <= EIG_PMAX.
hipError_t launch_qr(const double* in, double* out, int count, int n, int p, hipStream_t s);
// Multigrid prolongation of a factor: Uf (nf x r) = the columns of Uc (nc x r), read as functions
// on the uniform nodes x0c + i hc, linearly interpolated at x0f + j hf.
hipError_t launch_interp_factor(const double* Uc, int nc, double x0c, double hc, double* Uf, int nf, double x0f,
                                double hf, int r, hipStream_t s);
// Sign rule on the columns of U (n x r, ld ldu): a column whose entry of largest magnitude (ties
// within 1e-10 relative, lowest index) is negative is negated, together with column c of V
// (nv x r, ld ldv).
hipError_t launch_signfix_pair(double* U, int ldu, int n, double* V, int ldv, int nv, int r, hipStream_t s,
                               Bat bt = Bat());
hipError_t eig_set_attributes();

// ------------------------------------------------------------------- a5/a6: TTM ----
// T[row, c] = sum_k A[row, k] U[k, c]   (A x_3 U^T): A rows x n2, U n2 x r, T rows x r
hipError_t launch_ttm_last_f32(const float* A, long rows, int n2, const float* U, int r, float* T,
                               hipStream_t s, Bat bt = Bat());
// S[a, col] = sum_i U[i, a] A[i, col]   (A x_1 U^T): A n0 x cols, U n0 x r, S r x cols
hipError_t launch_ttm_first_f32(const float* A, int n0, long cols, const float* U, int r, float* S,
                                hipStream_t s, Bat bt = Bat());

// ------------------------------------------------------------------ a7: error norm ----
// partials[2b] = sum A^2, partials[2b+1] = sum (A - H U3^T)^2 over work-group b's rows;
// H: rows x r, U3: n2 x r.  recon_diff_parts(rows) work-groups.
int recon_diff_parts(long rows);
hipError_t launch_recon_diff_f32(const float* A, long rows, int n2, const double* H, const double* U3,
                                 int r, double* partials, hipStream_t s, Bat bt = Bat());
// partials[2b] = sum X^2, partials[2b+1] = sum (X - Y)^2 (grid-stride, nparts work-groups)
template <typename T>
hipError_t launch_diff_norm(const T* X, const T* Y, long n, double* partials, int nparts,
                            hipStream_t s, Bat bt = Bat());
hipError_t launch_reduce_partials(const double* partials, int nparts, int width, double* out,
                                  hipStream_t s, Bat bt = Bat());

// --------------------------------------------------------------- conversions/misc ----
hipError_t launch_convert_f64_to_f32(const double* x, float* y, long n, hipStream_t s, Bat bt = Bat());
hipError_t launch_convert_f32_to_f64(const float* x, double* y, long n, hipStream_t s);
hipError_t launch_fill_f64(double* x, double v, long n, hipStream_t s, Bat bt = Bat());
// y[i] = x[i] for i < n (batched copies inside workspaces)
hipError_t launch_copy_f64(const double* x, double* y, long n, hipStream_t s, Bat bt = Bat());
// Gather `words` 4-byte words of each of nb records src + b * bs (b < nb) into dst[b * words + i].
hipError_t launch_gather_u32(const void* src, long bs, int words, void* dst, int nb, hipStream_t s);
// out[0] = sum x*y (FP64 accumulation, deterministic two-level reduction)
template <typename T>
hipError_t launch_dot(const T* x, const T* y, long n, double* partials, int nparts, double* out,
                      hipStream_t s);

// ----------------------------------------------------------- a8: Toeplitz products ----
// left : Out[s][g][i'][n] (+)= sum_{b<nb} sum_{i<K} u_{g,b}[off + |i' - i|] In[s][g][b][i][n]
//        (i' < M, n < N; n contiguous in In and Out).  Generator u_{g,b}: element idx at
//        gen[idx * gs_idx + (g * gstride_g + b * gstride_b) * gs_col], glen entries used.
struct ToepLeftArgs {
    int M, N, K, nb;
    const void* gen; long gs_idx, gs_col, gstride_g, gstride_b; int glen, glen_pad, off;
    const void* In; long sIs, sIg, sIb, sIi;
    void* Out; long sOs, sOg, sOi;
    int accumulate;
};
// right: Out[row][b*m + j'] = sum_{j<K} In[row][j] u_b[off + |j - j'|]   (row < R, j' < m)
//        Generator u_b: element idx at gen[idx * gs_idx + b * gs_col].
struct ToepRightArgs {
    long R; int K, m, nb;
    const void* gen; long gs_idx, gs_col; int glen, off;
    const void* In; long ldi;
    void* Out; long ldo;
};
template <typename T>
hipError_t launch_toep_left(const ToepLeftArgs& a, int nslab, int ngroup, hipStream_t s);
template <typename T>
hipError_t launch_toep_right(const ToepRightArgs& a, hipStream_t s);
hipError_t kron_set_attributes();

// ---------------------------------------------------- a8: FFT form of the matvec ----
struct FftPassArgs {
    int L, logL;               // transform length 2^logL (2 <= L <= 2048)
    int n_inner;               // fibres along the inner index
    long n_outer;              // outer index range (set by launch_fft_pass)
    int len_in, len_out;       // valid input length (zero padded to L), output length kept
    long s_in_o, s_in_i, s_in_k, s_out_o, s_out_i, s_out_k;   // element strides
    const void* in; void* out;
    int in_real, out_real, mode;
    float scale;
    const float* Hs; const float* Uh3; int r2p;               // mode 3: Hs[f1][f0][c], Uh3[f2][c], c < r2p
    const float2* tw;                                          // exp(-2 pi i q / L), q < L
    // mode 2 only, optional: dot_part[b] = the FP64 sum of z * y over the outputs work-group b
    // stored (z laid out like the output); at most dot_cap work-groups run
    const float* dot_z; double* dot_part; int dot_cap;
    int no_store;              // mode 2 with dot_part: y is not stored (out may be NULL)
};
hipError_t launch_twiddles(float2* tw, int L, hipStream_t s);
hipError_t launch_f64_to_f32_padded(const double* X, long rows, int cols, int cols_pad, float* Y, hipStream_t s);
// Hs[f1][f0][c] = sum_b Uh1[f1][b] M1[f0][b][c] (c < r2), 0 for r2 <= c < r2p (Uh1: L1 x r1,
// M1: L0 x r1 x r2, FP64; Hs: L1 x L0 x r2p, FP32).  r1 <= 48, r2 <= r2p <= 256.
hipError_t launch_spectral_core(const double* Uh1, const double* M1, int L0, int L1, int r1, int r2, int r2p,
                                float* Hs, hipStream_t s);
// blocks (optional): the number of work-groups launched (partials written with dot_part)
hipError_t launch_fft_pass(const FftPassArgs& a, long n_outer, hipStream_t s, unsigned* blocks = nullptr);
// Fourier-side factors of the three axes: ax[k].Uh[f][a] = u_a[off] + 2 sum_{t=1}^{m-1}
// u_a[off + t] cos(2 pi f t / L), f < nf, a < r (U: n x r, Uh: nf x r, FP64; L a power of two
// <= 2048, m <= L).
struct FourierAxis {
    const double* U; int r, off, m, L, nf; double* Uh;
};
struct FourierAxes {
    FourierAxis ax[3];
};
hipError_t launch_fourier_factors(const FourierAxes& fa, hipStream_t s);
hipError_t fft_set_attributes();

// ------------------------------------------------------------ small scalar kernels ----
hipError_t launch_rank_rule(const double* lam, long sLam, int len, int count, const double* total, long sTotal,
                            const double* scal, int has_d2, double eps2, int* ranks, int* ok, hipStream_t s,
                            Bat bt = Bat());
template <typename TI, typename TO>
hipError_t launch_copy_block(const TI* X, int D1, int D2, TO* Y, int d0, int d1, int d2, hipStream_t s);
// Results of a batch of problems in one launch: problem b's factors U_k (n_k x r_k[b], the
// leading columns of the n_k x ld_k block at Usrc[k] + b bs bytes) and core (the leading
// r_0 x r_1 x r_2 block of the Rc_0 x Rc_1 x Rc_2 array at core_src + b bs bytes) are copied
// to its result block, in FP64 and rounded to FP32.
struct ResultDst {
    double* U[3]; float* U32[3]; double* core; float* core32; int r[3];
};
struct ExtractArgs {
    int nb; int n[3]; int ld[3]; int Rc[3];
    const double* Usrc[3]; const double* core_src; long bs;
    ResultDst dst[BATCH_MAX];
};
hipError_t launch_extract_results(const ExtractArgs& a, hipStream_t s);
hipError_t launch_cov_trace(const double* G, int r0, int r1, int r2, const double* u0, const double* u1,
                            const double* u2, double scale, double* out, hipStream_t s);
hipError_t launch_final_err(double* scal, hipStream_t s, Bat bt = Bat(), bool zero_t2 = false);
hipError_t launch_mask_rank(double* const U[3], const int n[3], const int R[3], double* core, const int* ranks,
                            hipStream_t s, Bat bt = Bat());

// ------------------------------------------------------------ seeded N(0,1) inputs ----
// Philox4x32-10 words of counter blocks c0 .. c0 + nblocks - 1 under key (k0, k1): four words
// per block (out holds 4 nblocks words, 16-byte aligned).
hipError_t launch_philox_words(uint32_t k0, uint32_t k1, unsigned long long c0, long nblocks, uint32_t* out,
                               hipStream_t s);
// z[e] for e < count: the Box-Muller normals of blocks 0 .. ceil(count / 2) - 1 (k_rng.hip).
hipError_t launch_philox_normal(uint32_t k0, uint32_t k1, long count, float* z, hipStream_t s);

// ------------------------------------- sinc-quadrature canonical tensor (k_sinc.hip) ----
// t_k, w_k (k = 0..2M) of the R = 2M + 1 term sinc rule for the Matern of order half + 1/2
// with c = sqrt(2 nu)/ell, step h.
hipError_t launch_sinc_nodes(int M, double h, double c, int half, double sigma2, double* t, double* w, hipStream_t s);
// Side matrices Q_l (n_l x R, row-major): Q_l[i][k] = w_k^(1/3) exp(-t_k x_{l,i}^2).
hipError_t launch_sinc_factors(const GridAxes& g, int R, const double* t, const double* w, double* const Q[3],
                               hipStream_t s);
// C = A o B (n elements)
hipError_t launch_hadamard(const double* A, const double* B, double* C, long n, hipStream_t s);
// KR (R x r1 r2) with KR[k][b r2 + c] = P1[b][k] P2[c][k]
hipError_t launch_khatri_rao(const double* P1, const double* P2, int R, int r1, int r2, double* KR, hipStream_t s);
// out[0] = sum_e A[e] B[e] C[e] (fixed order)
hipError_t launch_triple_sum(const double* A, const double* B, const double* C, long n, double* out, hipStream_t s);

}  // namespace tk
