/*
 * tk.h -- C ABI of the MI355X (gfx950) Tucker engine for Matern / Slater covariance tensors.
 *
 * Method: Litvinenko, Keyes, Khoromskaia, Khoromskij, Matthies, "Tucker tensor analysis of
 * Matern functions in spatial statistics" (arXiv 1711.06874).
 *
 *   - Task 1 of Sec. 2.1: approximate a covariance function sampled on an n1 x n2 x n3 tensor
 *     grid by a low-rank Kronecker/Tucker format within a tolerance eps;
 *   - the Tucker format of Sec. 3.1 eq. (3.4): A ~ G x_1 U1 x_2 U2 x_3 U3 with orthonormal
 *     factor columns, computed by HOSVD and then Tucker-ALS (HOOI) as in Sec. 3.2;
 *   - the covariance operator of Sec. 3.6 eq. (3.16)-(3.18), a sum of Kronecker products of
 *     symmetric Toeplitz matrices defined by their first column, applied to a vector as in
 *     Sec. 4 eq. (4.1), with its trace from Sec. 4 eq. (4.3) and the quadratic form z^T C z.
 *
 * Conventions for every entry point:
 *   - no call aborts or throws; every call returns a tk_status (TK_OK = 0, errors < 0), and
 *     tk_last_error() returns a message for the last failing call on the calling thread;
 *   - tensors are dense C-order (last index fastest) arrays; matrices are row-major;
 *   - "device" pointers are HIP device memory on the context's device (for example the
 *     data_ptr() of a torch.cuda tensor); "host" pointers are ordinary host memory;
 *   - hip_stream is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     enqueued on that stream in order; calls documented as synchronising wait for it;
 *   - caller-owned buffers stay caller-owned; objects returned through a `**out` argument
 *     are owned by the caller and released with the matching _free / _destroy call.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------------------- */
/* Status codes                                                                              */
/* ---------------------------------------------------------------------------------------- */
typedef enum {
    TK_OK = 0,
    TK_EINVAL = -1,        /* bad argument: NULL pointer, n < 2, ell <= 0, sigma2 <= 0,
                              non-finite value, neither eps nor ranks given, ...            */
    TK_EUNSUPPORTED = -2,  /* valid but not implemented: Matern nu above 30, more than
                              1024 points per axis, rank above the library cap               */
    TK_ELAYOUT = -3,       /* covariance operation on a grid without an origin node
                              (an even-sized centred grid)                                   */
    TK_ENOMEM = -4,        /* the estimated device memory exceeds the context's remaining
                              HBM budget (nothing was allocated), or an allocation failed    */
    TK_EHIP = -5,          /* a HIP runtime error (including asynchronous kernel faults seen
                              at the next synchronising call)                                */
    TK_ENOCONV = -6,       /* the requested eps could not be met within r_max               */
} tk_status;

/* ---------------------------------------------------------------------------------------- */
/* Problem description                                                                       */
/* ---------------------------------------------------------------------------------------- */
typedef enum {
    TK_MATERN = 0,  /* sigma2 * C_{nu,ell}(r), Sec. 2.2 eq. (2.3); 0 < nu <= 30.  nu = 1/2, 3/2,
                       5/2 take the closed forms, other orders K_nu (Temme's series for
                       arguments <= 2, Steed's continued fraction above, upward recurrence)   */
    TK_SLATER = 1,  /* sigma2 * exp(-alpha * (r/ell)^p), the p-Slater function of Sec. 3.7
                       eq. (3.27) with an amplitude, a rate and a length scale               */
    TK_GAUSS = 2,   /* sigma2 * exp(-(r/ell)^2): the separable (rank-1) case of Sec. 4.4      */
    TK_SPECTRAL = 3,/* sigma2 * f_{alpha,nu}(rho), the Matern spectral density of Diagram 1
                       in Sec. 2.2 / eq. (3.28) in d = 3: Gamma(nu+3/2) alpha^(2nu) /
                       (pi^(3/2) Gamma(nu)) (alpha^2 + rho^2)^-(nu+3/2), rho the grid radius;
                       uses nu and alpha (ell is ignored)                                     */
} tk_family;

typedef enum {
    TK_CENTERED = 0, /* x_i = -b + i h, i = 0..n-1, h = 2b/(n-1): the vertex grid of Sec. 3.7
                        eq. (3.25) on [-b, b]                                                */
    TK_OFFSET = 1,   /* x_i = i h with the same h: the generator at every difference of two
                        centred-grid nodes, i.e. the first columns of the Toeplitz factors of
                        the covariance of the centred grid (Sec. 3.6)                         */
} tk_layout;

typedef enum {
    TK_FP64 = 0,     /* tensor and every contraction in IEEE double                          */
    TK_FP32 = 1,     /* tensor in float; Gram and big contractions on FP32 MFMA with FP32
                        accumulation; eigensolves, small Grams and error norms in FP64        */
    TK_BF16X3 = 2,   /* as TK_FP32, but the Gram contractions split each float into a bf16
                        high and low part and sum three bf16 MFMA products (hi*hi + hi*lo +
                        lo*hi) with FP32 accumulation                                          */
} tk_precision;

typedef struct {
    int family;      /* tk_family */
    double nu;       /* Matern smoothness (TK_MATERN only) */
    double ell;      /* length scale, > 0 */
    double sigma2;   /* variance, > 0 */
    double alpha;    /* Slater rate, > 0 (TK_SLATER); spectral density parameter (TK_SPECTRAL) */
    double p;        /* Slater exponent, in (0, 2] (TK_SLATER only) */
    double metric[3];/* anisotropic distance r^2 = sum_k metric[k] x_k^2, a positive diagonal
                        metric (Sec. 2.2); all zero = the Euclidean distance.  The covariance
                        stays stationary, so the Toeplitz operators of Sec. 3.6 still apply   */
} tk_kernel;

typedef struct {
    int n[3];        /* points per axis, 2 <= n <= 1024 */
    double b[3];     /* half-width of the box per axis, > 0 */
    int layout;      /* tk_layout */
} tk_grid;

typedef struct {
    double eps;      /* > 0: choose ranks so the relative Frobenius error is <= eps;
                        0: use ranks[] */
    int ranks[3];    /* fixed Tucker ranks (used when eps == 0); clamped to n_k.  After
                        clamping at most 48 on TK_FP32 / TK_BF16X3 and at most 56 on TK_FP64
                        (TK_EUNSUPPORTED above)                                            */
    int r_max;       /* eps mode: largest rank considered per mode (0 = library default 24);
                        at most 48 */
    int hooi_sweeps; /* Tucker-ALS sweeps after HOSVD (0 = HOSVD only); TK_HOOI_CONVERGE =
                        sweep until | ||G|| - ||G_prev|| | <= 1e-13 ||A|| (the first G_prev
                        is the HOSVD core; at most 50 sweeps; one problem per pass, the core
                        norm is read back after every sweep); other values < 0 = library
                        default (2) */
    int prec;        /* tk_precision */
} tk_opts;

#define TK_HOOI_CONVERGE (-2)   /* tk_opts.hooi_sweeps: Tucker-ALS to convergence (Sec. 3.2) */

typedef struct tk_ctx tk_ctx;
typedef struct tk_tucker tk_tucker;

/* ---------------------------------------------------------------------------------------- */
/* Context                                                                                   */
/* ---------------------------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device memory that the
 * context's calls may hold at once (0 = 90% of the free device memory).  Synchronising.
 * Errors: TK_EINVAL (out == NULL, bad device), TK_EHIP. */
tk_status tk_ctx_create(int device, size_t hbm_budget_bytes, tk_ctx **out);

/* Wait for all work of the context and release its streams and staging buffers.  Results made
 * with it that are still alive may afterwards only be passed to tk_tucker_free (every other
 * call on them returns TK_EINVAL); the context's bookkeeping goes with the last of them.
 * NULL is ignored. */
void tk_ctx_destroy(tk_ctx *ctx);

/* Bytes of the budget currently reserved by the context's calls and resident results.  Idle
 * cached device blocks (workspaces kept per stream, blocks of freed results) are not included,
 * but they count against the budget as well: a reservation that would take reserved + idle
 * bytes past the budget first frees every idle block, so the device memory the context holds
 * stays within the budget plus at most 16 MiB of rounding per busy workspace block. */
tk_status tk_ctx_budget(const tk_ctx *ctx, size_t *budget_bytes, size_t *in_use_bytes);

/* Peak device bytes a tk_compress of this grid with these options needs (workspace plus the
 * result).  Pure host computation.  Errors: TK_EINVAL. */
tk_status tk_estimate_bytes(const tk_grid *grid, const tk_opts *opts, size_t *peak_bytes);

/* ---------------------------------------------------------------------------------------- */
/* Compression (Task 1 of Sec. 2.1; HOSVD and HOOI of Sec. 3.2)                              */
/* ---------------------------------------------------------------------------------------- */

/* Sample the covariance function on the grid (Sec. 3.7 eq. (3.25)) and compress it.
 *  - eps > 0: the FP64 path takes per-mode ranks from the HOSVD Gram eigenvalues
 *    (smallest r with sum_{i>r} lambda_i <= eps^2 ||A||^2 / 3), then runs hooi_sweeps sweeps;
 *    the FP32/BF16x3 paths run HOSVD and HOOI at r_max and then truncate the core by its own
 *    HOSVD to the smallest ranks whose error bound stays <= eps.  TK_ENOCONV if r_max does
 *    not reach eps (the result is still returned through *out, at rank r_max).
 *  - eps == 0: fixed ranks[] (clamped to n_k).
 * On the FP64 path every eigensolve iterates until its Ritz pairs pass the residual test of
 * tk_eig_topr; one that does not within its cap makes the call return TK_ENOCONV (the result
 * is still returned through *out).
 * The result keeps its factors and core resident on the device.  Synchronising: when the call
 * returns the result is complete and may be used from any stream.
 * Errors: TK_EINVAL, TK_EUNSUPPORTED, TK_ENOMEM, TK_EHIP, TK_ENOCONV. */
tk_status tk_compress(tk_ctx *ctx, const tk_kernel *kernel, const tk_grid *grid,
                      const tk_opts *opts, void *hip_stream, tk_tucker **out);

/* Compress a caller-supplied tensor A_dev (n[0] x n[1] x n[2], C-order, float for TK_FP32 and
 * TK_BF16X3, double for TK_FP64; not modified) instead of a sampled kernel.  The grid gives
 * the sizes and the layout that later covariance calls use.  Synchronising. */
tk_status tk_compress_tensor(tk_ctx *ctx, const void *A_dev, const tk_grid *grid,
                             const tk_opts *opts, void *hip_stream, tk_tucker **out);

/* Multigrid Tucker (Sec. 3.2, last paragraph; Fig. 7 of Sec. 3.7): the truncated HOSVD runs
 * only on the coarsest of levels + 1 grids over the same box (each coarser grid has (n + 1) / 2
 * points per axis: 2^k + 1 -> 2^(k-1) + 1 nests the vertex grids, 2^k -> 2^(k-1) halves them).
 * On each finer grid the factors of the previous level, linearly interpolated to the new nodes
 * and orthonormalised (Householder QR), start opts->hooi_sweeps Tucker-ALS sweeps (at least
 * one; TK_HOOI_CONVERGE on the FP64 path) on that grid's tensor: no Gram of a fine-grid tensor
 * is formed, so the cost is linear in the number of grid points.  The ranks are those of the
 * coarsest level (fixed ranks, or the eps rule applied there); the error returned is measured
 * on the finest grid, and TK_ENOCONV is returned with the result when it exceeds eps.
 * levels = 0 is tk_compress.  Synchronising.  Errors: as tk_compress; TK_EINVAL when the
 * coarsest grid would have fewer than 2 points per axis or levels > 8. */
tk_status tk_compress_multigrid(tk_ctx *ctx, const tk_kernel *kernel, const tk_grid *grid, int levels,
                                const tk_opts *opts, void *hip_stream, tk_tucker **out);

/* Sinc-quadrature canonical tensor and canonical-to-Tucker (Sec. 3.4; Laplace weights of
 * Sec. 3.5).  For a Matern covariance of order nu in {1/2, 3/2, 5/2} (isotropic distance) the
 * Laplace representation C(r) = sigma2 int_0^inf omega(t) exp(-r^2 t) dt is discretised by the
 * sinc rule on t = (c^2/4) e^u, c = sqrt(2 nu)/ell, with step h = C0 log(M)/M at u = k h,
 * k = -M..M: a canonical tensor of rank R = 2M + 1 whose side matrices are
 * Q_l[i][k] = w_k^(1/3) exp(-t_k x_{l,i}^2) on the grid's nodes.  Its Tucker form: factors from
 * the leading ranks[l] eigenvectors of Q_l Q_l^T (reduced HOSVD), then `sweeps` ALS sweeps on the
 * canonical data (single-hole Gram Q_a (P_j^T P_j o P_m^T P_m) Q_a^T, P_l = V_l^T Q_l), core
 * G = sum_k (V_1^T q_1k) (x) (V_2^T q_2k) (x) (V_3^T q_3k).  Everything runs on products of the
 * n_l x R side matrices (FP64); the n1 n2 n3 tensor is never formed.  The result's rel_err is
 * ||CP - T|| / ||CP|| against the canonical tensor (from ||CP||^2 - ||G||^2, so values below
 * about 1e-7 are not resolved) and norm_a is ||CP||.  ranks are clamped to n_l and R; 1 <= M <= 256,
 * C0 > 0, 0 <= sweeps <= 50.  Synchronising.  Errors: TK_EINVAL, TK_EUNSUPPORTED (another family
 * or order, an anisotropic metric, a rank above 48), TK_ENOMEM, TK_EHIP, TK_ENOCONV (an
 * eigensolve missed its residual test; the result is returned). */
tk_status tk_compress_sinc(tk_ctx *ctx, const tk_kernel *kernel, const tk_grid *grid, int M, double C0,
                           const int ranks[3], int sweeps, void *hip_stream, tk_tucker **out);

/* Compress `count` independent problems (kernels[i] on grids[i], sizes may differ, all with
 * *opts) in one call.  Problems on the same grid share their launches: up to 32 of them (fewer
 * if the HBM budget asks; a group is also split into near-equal parts of at least three
 * problems, up to its share of the tk_ctx_set_workers streams in proportion to its problems,
 * which run concurrently) run every step of the pipeline as one launch whose
 * third grid dimension walks the problems, so one eigensolve or Gram launch serves them all.  Such groups
 * (and problems that run alone: other grids, the FP64 path, which reads the eigensolver's
 * convergence flags and in eps mode the ranks back between steps, and converged HOOI) run
 * concurrently, largest first, on the context's worker streams
 * (tk_ctx_set_workers, default 4) with one host worker each, so the latency-bound steps of one
 * group overlap the bandwidth-bound passes of others.  They start after the work queued on
 * hip_stream.  Admission follows the HBM budget: a group that does not fit while others run
 * waits for one of them to finish.  outs[i] receives the i-th result, bitwise identical to
 * what tk_compress returns for that problem alone (TK_ENOCONV results included).
 * Synchronising: when the call returns every result is complete and may be used from any
 * stream.  On error no result is returned (outs[] set to NULL). */
tk_status tk_compress_batch(tk_ctx *ctx, int count, const tk_kernel *kernels,
                            const tk_grid *grids, const tk_opts *opts, void *hip_stream,
                            tk_tucker **outs);

/* Compress 1..32 problems that share one grid and one set of options in a single pass on
 * hip_stream: every step of the pipeline is one launch over all of them (as for a group inside
 * tk_compress_batch).  outs[i] / statuses[i]: the result of kernels[i], bitwise what tk_compress
 * returns for it alone, and TK_OK or TK_ENOCONV (eps not reached; the result is returned
 * anyway).  The FP64 path and converged HOOI run the problems one after another.  Synchronising: the results
 * are complete when the call returns.  Errors (no results): TK_EINVAL, TK_EUNSUPPORTED,
 * TK_ENOMEM (the group's workspaces and results exceed the budget), TK_EHIP. */
tk_status tk_compress_group(tk_ctx *ctx, int count, const tk_kernel *kernels, const tk_grid *grid,
                            const tk_opts *opts, void *hip_stream, tk_tucker **outs, int *statuses);

/* Autotuning of the Gram contraction: for grids of grid->n and precision prec, times each mode's
 * Gram with its default number of K chunks per 64 x 64 tile pair and with half and a quarter of
 * it (on a synthetic tensor of that shape, on hip_stream) and keeps the fastest in the context.
 * Later compressions of that shape and precision, alone or batched, use it (so batched and
 * single results stay bitwise equal; untuned shapes keep the default).  nsplit_out / ms_out
 * (optional): the chosen counts and their times per mode.  Synchronising.
 * Errors: TK_EINVAL, TK_ENOMEM, TK_EHIP. */
tk_status tk_autotune(tk_ctx *ctx, const tk_grid *grid, int prec, void *hip_stream, int nsplit_out[3],
                      double ms_out[3]);
/* Write / read the context's tuned entries as JSON ({"format": "tk-autotune-1", "entries":
 * [{"n": [n0, n1, n2], "mode": k, "prec": p, "nsplit": s}, ...]}); loading adds to (and
 * overrides) the entries present.  Errors: TK_EINVAL (unreadable or malformed file). */
tk_status tk_autotune_save(tk_ctx *ctx, const char *path);
tk_status tk_autotune_load(tk_ctx *ctx, const char *path);

/* Workspaces: each call takes its device workspace from a block the context keeps per HIP
 * stream, grown when a call needs more and reused by the next call on that stream, so calls in
 * steady state allocate nothing.  The budget charges each call's workspace while the call runs
 * (a kept block more than 16 MiB larger than the call needs is charged at its full size, or
 * replaced when that does not fit); idle blocks (at most two per stream: the largest workspace a
 * call on it needed, and a quadratic form's own y) are freed when a reservation needs their room
 * (see tk_ctx_budget).  tk_ctx_release_stream frees the blocks of a stream
 * (call it before destroying a stream the context has worked on); tk_ctx_destroy frees all.
 * Errors: TK_EINVAL (ctx NULL, a call on the stream still running), TK_EHIP. */
tk_status tk_ctx_release_stream(tk_ctx *ctx, void *hip_stream);

/* Graph replay of the compression pipeline (off by default).  When on, the launches of a call
 * that samples its own tensor (tk_compress, tk_compress_batch, tk_compress_group; not the FP64
 * eps path, which reads ranks back between steps, and not while tk_profile_enable is on) are
 * captured into a HIP graph the first time a shape, option set and problem count meets a given
 * workspace, and replayed on later calls with the sampling launch updated to the call's kernels
 * and grid: one graph launch instead of some hundred kernel launches.  Results are bitwise those
 * of the direct launches.  The context keeps at most 64 graphs (all dropped when more are
 * needed) until tk_ctx_destroy.  Host only.  Errors: TK_EINVAL (ctx NULL). */
tk_status tk_ctx_set_graphs(tk_ctx *ctx, int on);

/* Orthonormalisation of the float eps path (Sec. 3.2: the HOSVD start and the HOOI updates only
 * carry the leading subspace, which the core's HOSVD rotates at the end).  Its n x p block Y
 * (n <= 256 and p <= 32, or n <= 512 and p <= 24; larger blocks take Householder QR) is
 * orthonormalised by Cholesky QR, W = Y^T Y = L D L^T,
 * Q = Y L^-T D^-1/2, steered per block inside the kernel by the pivots' squared sines
 * s_j = d_j / W_jj.  First pass: pivots with s_j < floor are raised to floor W_jj (such columns
 * lie in the span of the earlier ones to rounding); all s_j >= one_pass ends there, else a
 * second pass orthonormalises the result.  Columns whose second-pass s_j < accept2 (rounding
 * noise inside the span of the others) are replaced by fixed pseudo-random columns and a third
 * pass runs; if its s_j are not all >= accept2 either, the block is orthonormalised by
 * Householder QR instead.  The first block of a cold start always takes Householder.  Defaults floor = 1e-12, one_pass = 1e-4, accept2 = 0.25.  floor <= 0:
 * Householder for every block; one_pass > 1: always two passes; accept2 > 1 (with one_pass
 * > 1): every Cholesky attempt falls back.  The factors then differ from the Householder route only by rounding
 * (the final factors are sign-normalised).  Drops the context's captured graphs.  Host only.
 * Errors: TK_EINVAL (ctx NULL, a threshold NaN). */
tk_status tk_ctx_set_cholqr(tk_ctx *ctx, double floor, double one_pass, double accept2);

/* Number of worker streams / host workers tk_compress_batch uses (1..16; default 4, the
 * number of hardware queues a process gets by default).  Host only. */
tk_status tk_ctx_set_workers(tk_ctx *ctx, int workers);

/* Sizes, ranks and the measured relative Frobenius error ||A - A_r|| / ||A|| (Sec. 3.7
 * eq. (3.26)).  Any output pointer may be NULL.  Host only. */
tk_status tk_tucker_info(const tk_tucker *t, int n[3], int ranks[3], double *rel_err_fro,
                         double *norm_a, int *layout);

/* Copy the result to host memory in FP64: U_host[k] receives n_k x r_k (row-major), core_host
 * r1 x r2 x r3 (C-order).  Any pointer may be NULL.  Synchronising. */
tk_status tk_tucker_get(const tk_tucker *t, double *U_host[3], double *core_host);

/* Device pointers of the resident FP64 factors (n_k x r_k row-major) and core (C-order).
 * Owned by the tk_tucker.  Host only. */
tk_status tk_tucker_device(const tk_tucker *t, const double *U_dev[3], const double **core_dev);

/* Write the reconstruction G x_1 U1 x_2 U2 x_3 U3 (n1 x n2 x n3, C-order) to A_dev as double
 * (io = TK_FP64) or float (io = TK_FP32).  Stream-ordered. */
tk_status tk_reconstruct(tk_ctx *ctx, const tk_tucker *t, void *A_dev, int io, void *hip_stream);

/* Save / load a result as a versioned little-endian binary file (header, sizes, ranks, FP64
 * factors and core).  Both synchronise.  Errors: TK_EINVAL (bad file), TK_ENOMEM, TK_EHIP. */
tk_status tk_tucker_save(const tk_tucker *t, const char *path);
tk_status tk_tucker_load(tk_ctx *ctx, const char *path, tk_tucker **out);

/* Release a result (after the work queued on it) and its device memory.  The context keeps the
 * device block (at most 256 blocks and 256 MB) for its next results of a similar size, so
 * steady-state compression allocates nothing; the kept blocks are freed with the context, or
 * earlier when a reservation needs their room in the budget.
 * NULL is ignored. */
void tk_tucker_free(tk_tucker *t);

/* ---------------------------------------------------------------------------------------- */
/* Covariance operator in Kronecker-Toeplitz form (Sec. 3.6; Sec. 4)                          */
/* ---------------------------------------------------------------------------------------- */
/* The result of compressing the generator on an OFFSET grid (or an odd CENTERED grid, whose
 * middle node is the origin) defines the covariance of m1 x m2 x m3 points:
 *     C = sum_abc G_abc T(U1[off1:, a]) (x) T(U2[off2:, b]) (x) T(U3[off3:, c]),
 *     T(u)_{ij} = u[|i - j|]  (symmetric Toeplitz, defined by its first column),
 * with off_k = 0, m_k = n_k for OFFSET grids and off_k = (n_k - 1)/2, m_k = (n_k + 1)/2 for
 * odd CENTERED grids (the non-negative sector).  Kronecker order follows C-order vectors:
 * (M1 (x) M2 (x) M3) vec(Z) = vec(Z x_1 M1 x_2 M2 x_3 M3).  Even CENTERED -> TK_ELAYOUT. */

/* Dimensions m[3] of the covariance operator of t.  Host only.  TK_ELAYOUT as above. */
tk_status tk_cov_dims(const tk_tucker *t, int m[3]);

/* y = C z (Sec. 4 eq. (4.1) for a general, non-separable z).  z_dev, y_dev: device arrays of
 * m1*m2*m3 elements, float (io = TK_FP32) or double (io = TK_FP64), C-order; y must not
 * overlap z.  The Toeplitz mode products run on FP32 MFMA (FP64 for io = TK_FP64).
 * Stream-ordered, asynchronous. */
tk_status tk_kron_matvec(tk_ctx *ctx, const tk_tucker *t, const void *z_dev, void *y_dev,
                         int io, void *hip_stream);

/* Allocation-free y = C z, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The FP32 FFT form of
 * tk_kron_matvec (same kernels, same launch shapes, so the same y bit for bit) with its whole
 * workspace in a fixed 16 MiB device array that the library holds on every device it runs on
 * until the process ends: operators of up to 64 points per axis (an OFFSET grid up to n = 64,
 * an odd CENTERED grid up to n = 127), at every rank the FFT form takes.  The call allocates
 * nothing, charges nothing to the context's budget and never synchronises.
 * z_dev, y_dev: caller-owned device float arrays of m1*m2*m3 elements (tk_cov_dims), C-order;
 * y must not overlap z.  The scratch array is shared by every call on a device and keeps the
 * last call's contents (nothing in it needs to start at zero): calls that overlap on one
 * device, on any streams or contexts, race and must be ordered by the caller.
 * Errors: TK_EINVAL (NULL argument, y aliases z), TK_ELAYOUT (even CENTERED grid),
 * TK_EUNSUPPORTED (third rank above 48), TK_ENOMEM (operator larger than the scratch holds:
 * nothing runs), TK_EHIP. */
tk_status tk_kron_matvec_noalloc(tk_ctx *ctx, const tk_tucker *t, const float *z_dev, float *y_dev,
                                 void *hip_stream);

/* Matvec algorithm of a context: TK_MV_AUTO (default: the FFT form for io = TK_FP32, dense
 * Toeplitz mode products for TK_FP64), TK_MV_FFT (FP32 only), TK_MV_DENSE.  A result whose
 * third rank exceeds 48 (an FP64 compression or a loaded file) always takes the dense form.
 * FFT form: every Toeplitz factor embeds in a circulant of length L >= 2m - 1 (Sec. 3.6:
 * O(n log n) Toeplitz products), so C = P F^-H diag(chat) F P^T with F the 3-D DFT and chat
 * the Tucker tensor with DFT'd, circulant-embedded factors; five FP32 FFT passes.
 * Dense form: r1 + 2 r1 r2 mode products with the Toeplitz matrices on MFMA.
 * Errors: TK_EINVAL. */
typedef enum { TK_MV_AUTO = 0, TK_MV_FFT = 1, TK_MV_DENSE = 2 } tk_matvec_method;
tk_status tk_set_matvec_method(tk_ctx *ctx, int method);

/* Device workspace bytes that tk_kron_matvec / tk_quadratic_form (with y supplied) need for t
 * with io precision under the context's current matvec method.  Host only.
 * Errors: TK_EINVAL, TK_ELAYOUT. */
tk_status tk_estimate_matvec_bytes(tk_ctx *ctx, const tk_tucker *t, int io, size_t *bytes);

/* trace(C) = sum_abc G_abc prod_k trace T(U_k[off_k:, .]) = m1 m2 m3 * A_r(origin)
 * (Sec. 4 eq. (4.3) and the value-at-origin form that follows it).  Computed on the device
 * in FP64; synchronising (one scalar read). */
tk_status tk_trace(tk_ctx *ctx, const tk_tucker *t, void *hip_stream, double *out);

/* z^T C z (FP64 accumulation of the dot product with C z).  If y_dev is not NULL it also
 * receives C z (same type and size as z); on the FFT path the dot product is summed as C z is
 * formed, so without y_dev C z is never stored.  Synchronising (one scalar read). */
tk_status tk_quadratic_form(tk_ctx *ctx, const tk_tucker *t, const void *z_dev, int io,
                            void *hip_stream, double *out, void *y_dev);
/* tk_quadratic_form for `count` results at once: out[i] = z_i^T C_i z_i (and y_devs[i] = C_i z_i
 * when y_devs and y_devs[i] are not NULL), after the work queued on hip_stream.  On the FFT path
 * the small per-item preambles run on a worker stream of the context while the five data passes
 * of the items run back to back on hip_stream (one pair of spectrum buffers serves them all, and
 * the values are read back together); on the dense path the items run concurrently on the
 * worker streams (tk_ctx_set_workers).  Each value is bitwise the one the single call returns.
 * Synchronising.  Errors: as tk_quadratic_form, for the first failing item. */
tk_status tk_quadratic_form_batch(tk_ctx *ctx, int count, const tk_tucker *const *ts,
                                  const void *const *z_devs, int io, void *hip_stream, double *out,
                                  void *const *y_devs);

/* ---------------------------------------------------------------------------------------- */
/* Separable covariance: rank-1 Kronecker algebra (Sec. 4, "Separable covariance matrices")   */
/* ---------------------------------------------------------------------------------------- */
/* A covariance that factors over the axes, C = C_1 (x) C_2 (x) C_3 with
 * C_k[i][j] = kernels[k](|x_i - x_j|) + nugget[k] [i == j] on axis k of the grid (for the
 * Gaussian exp(-|x - y|^2 / ell^2) this is exactly its covariance on the 3-D grid).  The
 * product of the three kernels' sigma2 scales C (give it on one axis and 1 on the others).
 * The operator acts on n1 x n2 x n3 vectors in C order, (M1 (x) M2 (x) M3) vec(Z) =
 * vec(Z x_1 M1 x_2 M2 x_3 M3).  The lemmas of Sec. 4 reduce every operation to the factors:
 *   Cholesky: C = L L^T with L = L_1 (x) L_2 (x) L_3 (each L_k by a blocked FP64 Cholesky);
 *   inverse: C^-1 = C_1^-1 (x) C_2^-1 (x) C_3^-1;
 *   log det C = sum_j (N / n_j) log det C_j, log det C_j = 2 sum_i log L_j[i][i];
 *   log-likelihood of z under N(0, C): -1/2 (N log(2 pi) + log det C + z^T C^-1 z).
 * (The printed log-likelihood formula of that section is garbled; this is the Gaussian one.) */
typedef struct tk_kron1 tk_kron1;
typedef enum { TK_KRON1_SOLVE = 0, TK_KRON1_CHOL = 1 } tk_kron1_op;

/* Build the three factors on the device and their Cholesky factors and log-determinants.
 * kernels: 3 covariance functions (any family; metric ignored), grid: points and box per axis
 * (n_k <= 16384; layout as for tk_compress), nugget: 3 values >= 0 (NULL = none).  The
 * factors stay resident (8 n_k^2 bytes each, charged to the budget) until tk_kron1_free.
 * Synchronising.  Errors: TK_EINVAL (NULL, bad kernel, a factor that is not positive definite:
 * add a nugget), TK_EUNSUPPORTED, TK_ENOMEM, TK_EHIP. */
tk_status tk_kron1_create(tk_ctx *ctx, const tk_kernel kernels[3], const tk_grid *grid, const double nugget[3],
                          void *hip_stream, tk_kron1 **out);
/* log det C (and, if logdet_axis is not NULL, log det C_k per axis).  Host only. */
tk_status tk_kron1_logdet(const tk_kron1 *k, double *out, double logdet_axis[3]);
/* Copy L_axis (n x n row-major, lower triangular) to host memory.  Synchronising. */
tk_status tk_kron1_factor(const tk_kron1 *k, int axis, double *L_host);
/* y = C^-1 z (op TK_KRON1_SOLVE) or y = L z (op TK_KRON1_CHOL: with z ~ N(0, I), y ~ N(0, C)).
 * z_dev, y_dev: N = n1 n2 n3 doubles on the device, y may not alias z.  The solve forms
 * C_k^-1 = L_k^-T L_k^-1 once (n_k <= 1024, kept with the object; synchronising the first time)
 * and applies it along each mode on FP64 MFMA.  Stream-ordered.
 * Errors: TK_EINVAL, TK_EUNSUPPORTED (solve with an axis above 1024), TK_ENOMEM, TK_EHIP. */
tk_status tk_kron1_apply(tk_ctx *ctx, tk_kron1 *k, int op, const double *z_dev, double *y_dev, void *hip_stream);
/* Gaussian log-likelihood of z (device, N doubles) under N(0, C); quad_out (optional) receives
 * z^T C^-1 z.  Synchronising.  Errors: as tk_kron1_apply. */
tk_status tk_kron1_loglik(tk_ctx *ctx, tk_kron1 *k, const double *z_dev, void *hip_stream, double *out,
                          double *quad_out);
/* Release the factors (after the work queued on them).  NULL is ignored. */
void tk_kron1_free(tk_kron1 *k);

/* ---------------------------------------------------------------------------------------- */
/* Seeded inputs                                                                             */
/* ---------------------------------------------------------------------------------------- */

/* Seeded N(0,1) input vectors made on the device (the z of the covariance matvec and quadratic
 * form).  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11: ten rounds with multipliers
 * 0xD2511F53, 0xCD9E8D57 and key increments 0x9E3779B9, 0xBB67AE85) keyed by (seed, stream_id);
 * counter block c = (c mod 2^32, c / 2^32, 0, 0) yields words x0..x3, the FP64 uniforms
 * u_a = ((x1 2^32 + x0) >> 11) 2^-53 and u_b = ((x3 2^32 + x2) >> 11) 2^-53, and by the
 * Box-Muller transform z[2c] = rho cos(phi), z[2c+1] = rho sin(phi) with
 * rho = sqrt(-2 log(1 - u_a)), phi = 2 pi u_b, each rounded once to float.
 * z_dev: caller-owned device floats, count <= 2^32.  Stream-ordered.  Errors: TK_EINVAL, TK_EHIP. */
tk_status tk_normal_fill(tk_ctx *ctx, uint32_t seed, uint32_t stream_id, float *z_dev, size_t count,
                         void *hip_stream);

/* The raw Philox4x32-10 words of counter blocks counter0 .. counter0 + nblocks - 1 (counter
 * (c mod 2^32, c / 2^32, 0, 0)) under key[2]: 4 nblocks words to out_dev (16-byte aligned).
 * nblocks <= 2^31.  Stream-ordered.  Errors: TK_EINVAL, TK_EHIP. */
tk_status tk_philox4x32(tk_ctx *ctx, const uint32_t key[2], uint64_t counter0, size_t nblocks,
                        uint32_t *out_dev, void *hip_stream);

/* ---------------------------------------------------------------------------------------- */
/* Individual steps (the same kernels tk_compress runs), exposed for testing and profiling   */
/* ---------------------------------------------------------------------------------------- */

/* a1: A_dev (n1 x n2 x n3, double for TK_FP64 else float) = sigma2 * k(||x||) on the grid.
 * Stream-ordered.  Errors: TK_EINVAL, TK_EUNSUPPORTED. */
tk_status tk_grid_eval(tk_ctx *ctx, const tk_kernel *kernel, const tk_grid *grid, int prec,
                       void *A_dev, void *hip_stream);

/* a2: G_dev (n_mode x n_mode, double, full symmetric) = A_(mode) A_(mode)^T for the
 * n[0] x n[1] x n[2] tensor A_dev (double for TK_FP64, float for TK_FP32 / TK_BF16X3).
 * Stream-ordered. */
tk_status tk_gram(tk_ctx *ctx, const void *A_dev, const int n[3], int mode, int prec,
                  double *G_dev, void *hip_stream);

/* a3: leading r eigenpairs of `count` symmetric positive semidefinite n x n matrices
 * (G_dev: count consecutive n*n doubles).  lambda_dev: count x r (descending);
 * U_dev: count x n x r row-major, unit columns, each signed so that its entry of largest
 * magnitude is positive (ties within 1e-10 relative go to the lowest index).  r <= 48.
 * n > 56: block subspace iteration with r + 8 columns and Rayleigh-Ritz, repeated until every
 * Ritz pair has ||G u - lambda u|| <= max(1e-12 lambda, 4 sqrt(n) u ||G||_F) (u = 2^-53), at
 * most 35 iterations; n <= 56: Jacobi on G itself.  Synchronising.  Errors: TK_EINVAL,
 * TK_EUNSUPPORTED, TK_ENOMEM, TK_EHIP, TK_ENOCONV (the residual test was not met; the outputs
 * hold the last iterate). */
tk_status tk_eig_topr(tk_ctx *ctx, int count, int n, int r, const double *G_dev,
                      double *lambda_dev, double *U_dev, void *hip_stream);

/* ---------------------------------------------------------------------------------------- */
/* Serving: a request loop over resident results                                            */
/* ---------------------------------------------------------------------------------------- */
/* Requests are queued in arrival order and run on `workers` worker threads, each with its own
 * HIP stream.  A free worker takes the first queued request that can run now: a compress when
 * its tk_estimate_bytes fits the context's HBM budget next to the resident results and the
 * requests already admitted, a follow-up (matvec, trace, quadratic form) when the compress it
 * names has finished and its tk_estimate_matvec_bytes fits.  Requests that cannot run yet stay
 * queued while later ones go ahead, so work that arrives while others are on the GPU is
 * admitted as workers and memory free up.  Compress results stay resident, owned by the
 * server, until tk_server_release or tk_server_destroy.  Every result is the one the plain
 * entry point returns for the same request alone. */
typedef enum { TK_REQ_COMPRESS = 0, TK_REQ_MATVEC = 1, TK_REQ_TRACE = 2, TK_REQ_QUADFORM = 3 } tk_req_kind;
typedef struct {
    int kind;            /* tk_req_kind */
    tk_kernel kernel;    /* compress */
    tk_grid grid;        /* compress */
    tk_opts opts;        /* compress */
    long long target;    /* follow-ups: ticket of an earlier compress request */
    const void *z_dev;   /* matvec, quadratic form: input vector (caller-owned, io precision) */
    void *y_dev;         /* matvec: output (required); quadratic form: optional output */
    int io;              /* TK_FP32 or TK_FP64 */
    void *stream;        /* matvec, quadratic form: work queued on this HIP stream before
                            tk_server_submit (for example the copy that fills z_dev) completes before
                            the request starts; NULL: the legacy default stream; TK_STREAM_READY:
                            the vectors are complete already (no ordering with any stream, so the
                            request never waits behind unrelated work of that stream).  Compress and
                            trace requests have no device inputs and are never ordered. */
} tk_request;
#define TK_STREAM_READY ((void *)(intptr_t)-1)
typedef struct {
    int status;                        /* tk_status of the request */
    int kind;
    int ranks[3];                      /* compress */
    double rel_err;                    /* compress */
    double value;                      /* trace or quadratic form */
    double t_submit, t_start, t_end;   /* seconds since tk_server_create */
    char error[192];                   /* status != TK_OK: the failing call's message (the
                                          worker's tk_last_error, truncated); else empty */
} tk_result;
typedef struct tk_server tk_server;

/* workers in 1..16.  Errors: TK_EINVAL, TK_ENOMEM, TK_EHIP. */
tk_status tk_server_create(tk_ctx *ctx, int workers, tk_server **out);
/* Continuous batching: a worker that takes a compress request also takes the queued compress
 * requests with the same grid and options (up to max_group in all, while their estimates fit
 * the budget) and runs them as one tk_compress_group pass; each result is bitwise the one the
 * request gets alone.  max_group in 1..32 (1: one request per pass); default 32.
 * Errors: TK_EINVAL. */
tk_status tk_server_set_batching(tk_server *sv, int max_group);
/* Queue a request (copied; the vectors must stay valid until the request finishes) and return
 * its ticket.  Non-blocking.  Errors: TK_EINVAL (bad kind, missing vectors, server stopping). */
tk_status tk_server_submit(tk_server *sv, const tk_request *req, long long *ticket);
/* Block until the request finished and return its result (once per ticket).  A follow-up on an
 * unknown, failed or released compress finishes with status TK_EINVAL.  Errors: TK_EINVAL
 * (unknown or already collected ticket). */
tk_status tk_server_wait(tk_server *sv, long long ticket, tk_result *out);
/* The resident result of a finished compress request (owned by the server). */
tk_status tk_server_tucker(tk_server *sv, long long compress_ticket, const tk_tucker **out);
/* Drop a resident result (freed once the follow-ups running on it finish); later follow-ups on
 * it fail with TK_EINVAL. */
tk_status tk_server_release(tk_server *sv, long long compress_ticket);
/* Finish every queued request, then free the resident results, streams and workers. */
void tk_server_destroy(tk_server *sv);

/* ---------------------------------------------------------------------------------------- */
/* Kernel timing                                                                              */
/* ---------------------------------------------------------------------------------------- */
/* When enabled, every launch of the classes below is bracketed by HIP events recorded on the
 * stream it runs on (process-wide, all contexts).  tk_profile_read synchronises on the
 * recorded events and returns the number of launches and their summed duration in ms. */
typedef enum {
    TK_PROF_GRID = 0, TK_PROF_GRAM = 1, TK_PROF_EIG = 2, TK_PROF_TTM = 3, TK_PROF_NORM = 4,
    TK_PROF_TOEP_RIGHT = 5, TK_PROF_TOEP_LEFT = 6, TK_PROF_SMALL = 7, TK_PROF_FFT = 8,
    TK_PROF_FFT_AXIS0 = 9, TK_PROF_COUNT = 10
} tk_prof_class;
tk_status tk_profile_enable(int on);
/* Only the classes whose bit (1 << class) is set in mask are bracketed (default: all).  Each
 * pair of events costs the stream a few microseconds between its launches. */
tk_status tk_profile_select(unsigned mask);
tk_status tk_profile_reset(void);
tk_status tk_profile_read(int cls, long long *launches, double *total_ms);

/* Message for the last failing call on this thread ("" if none). */
const char *tk_last_error(void);

/* Static name of a status code. */
const char *tk_strerror(tk_status s);

/* Library version string. */
const char *tk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TK_H */
