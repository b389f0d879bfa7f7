// Host driver and C ABI of the Tucker engine (declared in include/tk.h).
//
// A compression enqueues, on the caller's stream:
//   grid evaluation -> three mode Grams -> leading eigenvectors (HOSVD, Sec. 3.2)
//   -> HOOI sweeps (Sec. 3.2: single-hole tensors with the latest factors, Gauss-Seidel over
//      modes 1, 2, 3) -> core from the last single-hole tensor -> reconstruction error
//      (Sec. 3.7 eq. (3.26)) -> eps truncation,
// and synchronises once at the end to read the ranks and the error.  All arithmetic runs in
// the HIP kernels of this library; the host only plans shapes, allocates and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <map>
#include <mutex>
#include <utility>
#include <thread>
#include <new>
#include <string>
#include <vector>

#include "../../include/tk.h"
#include "tk_kernels.h"

using namespace tk;

// Device scratch of the allocation-free matvec (tk_kron_matvec_noalloc): the whole FFT workspace
// of one call (twiddles, Fourier-side factors, spectral core, both half spectra) for operators
// of up to 64 points per axis at every rank (12.9 MB at m = 64, r = 48).  Each device holds its
// own copy until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns on that device (scratch_address below), never through this name.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

tk_status fail(tk_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define TK_HIP(x)                                                                                  \
    do {                                                                                           \
        hipError_t _e = (x);                                                                       \
        if (_e != hipSuccess) return fail(TK_EHIP, "%s failed: %s", #x, hipGetErrorString(_e));    \
    } while (0)

constexpr int LIB_RMAX = 48;          // largest rank the kernels support
constexpr int DEFAULT_RMAX = 24;      // eps mode working rank when r_max == 0
constexpr int DEFAULT_SWEEPS = 2;
constexpr int CONVERGE_MAX_SWEEPS = 50;   // cap of the converged-HOOI mode
constexpr double CONVERGE_TOL = 1e-13;    // ... its test on the core norm, relative to ||A||
constexpr int COLD_ITERS = 3;         // subspace iterations from a random start (FP64 path)
constexpr int COLD_ITERS_F32 = 2;     // ... float paths (HOOI refines the subspaces anyway)
constexpr int WARM_ITERS = 2;         // ... from the previous factor (FP64 path: exact HOOI steps)
constexpr int WARM_ITERS_F32 = 1;     // ... float paths: one block power step per HOOI update
constexpr int SPAN_ITERS_F32 = 2;     // float eps path, HOSVD start: R-column block, subspace only
// Jacobi of the core Grams in the float eps truncation: off(H) <= 1e-10 ||H||_F leaves the
// eigenvalues off by about off(H)^2 / gap, far below the eps^2 a2 / 3 budget of the rank rule,
// and V orthogonal to rounding (a product of rotations); the truncated result's error is then
// measured against A
constexpr double CORE_JACOBI_TOL = 1e-10;
constexpr int NMAX = 1024;
constexpr double MATERN_NU_MAX = 30.0;  // general orders: K_nu s^nu stays inside the double range
constexpr int KRON1_NMAX = 16384;       // points per axis of a separable covariance factor

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device address of `scratch` on `device` (which must be current), looked up once per device.
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

hipError_t scratch_address(int device, void** out)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Two-pass arena: pass 1 (base == nullptr) sums sizes, pass 2 hands out aligned pointers.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count)
    {
        size_t o = align_up(off, 256);
        off = o + align_up(count * sizeof(T), 256);
        return base ? reinterpret_cast<T*>(base + o) : nullptr;
    }
};

// ---- kernel timing: events around launches of selected classes ----------------------------
struct ProfRec {
    int cls;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::atomic<unsigned> g_prof_mask{~0u};    // classes whose launches are bracketed (tk_profile_select)
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(int c, hipStream_t st) : cls(c), s(st)
    {
        if (!g_prof_on.load() || !((g_prof_mask.load() >> c) & 1u)) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        a = pool_event();
        if (a) (void)hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        hipEvent_t b = pool_event();
        if (!b) return;
        (void)hipEventRecord(b, s);
        g_prof.push_back({cls, a, b});
    }
};

}  // namespace

struct tk_ctx {
    int device = 0;
    int matvec_method = TK_MV_AUTO;
    void* scratch = nullptr;   // this device's copy of the no-allocation scratch
    size_t budget = 0;
    std::atomic<size_t> in_use{0};
    // results made with the context; a destroyed context is deleted with its last result
    std::mutex life_mu;
    int live_results = 0;
    bool closing = false;
    // scalar readbacks go through pinned host slots (and matching device slots) handed out per
    // call, so concurrent calls on different streams do not share a staging buffer
    static constexpr int kSlots = 64;
    static constexpr size_t kSlotBytes = 256;
    char* pinned = nullptr;
    char* dev_slots = nullptr;
    std::mutex slot_mu;
    uint64_t slot_used = 0;
    // streams of the batch workers, created on first use, destroyed with the context
    std::mutex pool_mu;
    std::vector<hipStream_t> streams;
    int workers = 4;
    // per-stream workspaces (slot 0: a call's workspace, slot 1: a quadratic form's own y),
    // grown when a call needs more and kept for the next call on the stream
    struct WsBlock {
        void* ptr = nullptr;
        size_t bytes = 0;
        bool busy = false;
    };
    std::mutex ws_mu;
    std::map<std::pair<hipStream_t, int>, WsBlock> ws;
    // bytes of device blocks the context keeps while no call uses them: idle workspace blocks
    // and the result-block cache.  A reservation that would take in_use + idle past the budget
    // frees them first (trim_idle), so the context never holds more than the budget plus the
    // rounding of the busy workspace blocks.
    std::atomic<size_t> idle{0};
    // autotuned Gram split counts, key {n0, n1, n2, mode, prec}
    std::mutex tune_mu;
    std::map<std::array<int, 5>, int> tune;
    // captured compression pipelines (tk_ctx_set_graphs), key: shape, options, batch, workspace
    struct GraphEntry {
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        hipGraphNode_t grid_node = nullptr;
    };
    bool graphs_on = false;
    // float eps path: thresholds of the Cholesky QR (tk_ctx_set_cholqr)
    CholQr cholqr{1e-12, 1e-4, 0.25};
    // device blocks of freed results, kept for the next results (size -> block); at most
    // kResultCache blocks and kResultCacheBytes bytes, freed with the context
    static constexpr size_t kResultCache = 256;
    static constexpr size_t kResultCacheBytes = (size_t)256 << 20;
    std::mutex rc_mu;
    std::multimap<size_t, void*> rcache;
    size_t rcache_bytes = 0;
    std::mutex graph_mu;
    std::map<std::array<long, 19>, GraphEntry> graphs;
};

struct tk_tucker {
    tk_ctx* ctx = nullptr;
    int n[3] = {0, 0, 0}, r[3] = {0, 0, 0};
    double b[3] = {1, 1, 1};
    int layout = TK_CENTERED;
    int prec = TK_FP32;
    double rel_err = 0.0, norm_a = 0.0;
    void* block = nullptr;        // one device allocation for everything below
    size_t block_bytes = 0;       // its size (a reused block may be larger than `bytes`)
    double* U[3] = {nullptr, nullptr, nullptr};
    double* core = nullptr;
    float* U32[3] = {nullptr, nullptr, nullptr};
    float* core32 = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
};

namespace {

void trim_idle(tk_ctx* c);

// Charge `bytes` to the budget.  Idle cached blocks count against it too: when they are in the
// way they are freed (trim_idle) and the check is repeated once.
bool reserve(tk_ctx* c, size_t bytes, bool may_trim = true)
{
    for (int attempt = 0; attempt < 2; ++attempt) {
        size_t cur = c->in_use.load();
        while (cur + bytes + c->idle.load() <= c->budget)
            if (c->in_use.compare_exchange_weak(cur, cur + bytes)) return true;
        if (cur + bytes > c->budget || !may_trim || c->idle.load() == 0) return false;
        trim_idle(c);
    }
    return false;
}
void release(tk_ctx* c, size_t bytes) { c->in_use.fetch_sub(bytes); }

struct Reservation {
    tk_ctx* c;
    size_t bytes;
    bool held;
    Reservation(tk_ctx* c_, size_t b) : c(c_), bytes(b), held(false) {}
    bool take() { held = reserve(c, bytes); return held; }
    // take `b` bytes (a reservation made empty and filled once its size is known)
    bool take_bytes(size_t b)
    {
        if (held) return false;
        bytes = b;
        return take();
    }
    // part of the reservation passes to an object that releases it itself (a result)
    bool hand_over(size_t b)
    {
        if (!held || b > bytes) return false;
        bytes -= b;
        return true;
    }
    ~Reservation() { if (held) release(c, bytes); }
};

// Device workspace of one call on stream s: the stream's cached block, grown when too small
// and kept afterwards (calls on one stream run in stream order, so the next call may reuse it
// at once), or a one-off block when another host thread holds it.  The pool allocator is
// slow when many workspaces of varying sizes come and go, so steady-state calls allocate
// nothing.  An idle cached block is not charged to the budget; the call's Reservation is.
struct Ws {
    tk_ctx* c = nullptr;
    hipStream_t s = nullptr;
    int slot = 0;
    void* p = nullptr;
    bool cached = false;
    size_t extra = 0;    // bytes of the cached block beyond the call's request, charged while busy
    Ws() = default;
    Ws(const Ws&) = delete;
    Ws& operator=(const Ws&) = delete;
    ~Ws()
    {
        if (!p) return;
        if (cached) {
            std::lock_guard<std::mutex> g(c->ws_mu);
            tk_ctx::WsBlock& b = c->ws[{s, slot}];
            b.busy = false;
            c->idle.fetch_add(b.bytes);
            release(c, extra);
        } else {
            (void)hipFreeAsync(p, s);
        }
    }
};

hipError_t ws_get(tk_ctx* c, hipStream_t s, int slot, size_t bytes, Ws& w)
{
    w.c = c;
    w.s = s;
    w.slot = slot;
    std::lock_guard<std::mutex> g(c->ws_mu);
    tk_ctx::WsBlock& b = c->ws[{s, slot}];
    if (b.busy) {
        hipError_t e = hipMallocAsync(&w.p, bytes, s);
        if (e != hipSuccess) w.p = nullptr;
        return e;
    }
    c->idle.fetch_sub(b.bytes);   // the block leaves the idle set (or is replaced below)
    // a kept block much larger than this call needs would hold budget it does not charge:
    // its excess is charged while the call runs, or, when that does not fit, it is replaced
    const size_t round = (size_t)1 << 24;
    if (b.bytes >= bytes && b.bytes - bytes > round && !reserve(c, b.bytes - bytes, false)) {
        (void)hipFreeAsync(b.ptr, s);
        b.ptr = nullptr;
        b.bytes = 0;
    } else if (b.bytes >= bytes && b.bytes - bytes > round) {
        w.extra = b.bytes - bytes;
    }
    if (b.bytes < bytes) {
        if (b.ptr) (void)hipFreeAsync(b.ptr, s);   // after the earlier calls on s, in stream order
        b.ptr = nullptr;
        b.bytes = 0;
        const size_t want = align_up(bytes, round);
        hipError_t e = hipMallocAsync(&b.ptr, want, s);
        if (e == hipSuccess) {
            b.bytes = want;
        } else {
            (void)hipGetLastError();
            e = hipMallocAsync(&b.ptr, bytes, s);
            if (e != hipSuccess) {
                b.ptr = nullptr;
                return e;
            }
            b.bytes = bytes;
        }
    }
    b.busy = true;
    w.p = b.ptr;
    w.cached = true;
    return hipSuccess;
}

// Free every idle workspace block and the result-block cache, and hand the freed memory of
// the stream-ordered pool back to the device.
void trim_idle(tk_ctx* c)
{
    {
        std::lock_guard<std::mutex> g(c->ws_mu);
        for (auto it = c->ws.begin(); it != c->ws.end();) {
            if (it->second.busy) { ++it; continue; }
            if (it->second.ptr) (void)hipFreeAsync(it->second.ptr, it->first.first);
            c->idle.fetch_sub(it->second.bytes);
            it = c->ws.erase(it);
        }
    }
    {
        std::lock_guard<std::mutex> g(c->rc_mu);
        for (auto& kv : c->rcache) (void)hipFree(kv.second);
        c->idle.fetch_sub(c->rcache_bytes);
        c->rcache.clear();
        c->rcache_bytes = 0;
    }
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) {
        (void)hipDeviceSynchronize();
        (void)hipMemPoolTrimTo(pool, 0);
    }
}

bool finite(double x) { return std::isfinite(x); }

tk_status check_kernel(const tk_kernel* k, KernelParams* kp)
{
    if (!k) return fail(TK_EINVAL, "kernel is NULL");
    if (!finite(k->sigma2) || k->sigma2 <= 0) return fail(TK_EINVAL, "sigma2 must be finite and > 0");
    if (k->family != TK_SPECTRAL && (!finite(k->ell) || k->ell <= 0))
        return fail(TK_EINVAL, "ell must be finite and > 0");
    kp->family = k->family;
    kp->sigma2 = k->sigma2;
    kp->alpha = k->alpha;
    kp->p = k->p;
    kp->half = 0;
    kp->nu = k->nu;
    kp->lpref = 0.0;
    // anisotropic metric: all zero = the identity; otherwise every entry finite and > 0
    const bool iso = k->metric[0] == 0.0 && k->metric[1] == 0.0 && k->metric[2] == 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!iso && !(finite(k->metric[a]) && k->metric[a] > 0))
            return fail(TK_EINVAL, "metric[%d]=%g: the diagonal metric needs entries > 0 (or all 0)", a, k->metric[a]);
        kp->axs[a] = iso ? 1.0 : std::sqrt(k->metric[a]);
    }
    if (k->family == TK_MATERN) {
        if (!finite(k->nu) || k->nu <= 0) return fail(TK_EINVAL, "Matern nu must be finite and > 0");
        if (k->nu > MATERN_NU_MAX) return fail(TK_EUNSUPPORTED, "Matern nu=%g exceeds %g", k->nu, MATERN_NU_MAX);
        int half = -1;
        for (int h = 0; h < 3; ++h)
            if (std::fabs(k->nu - (h + 0.5)) < 1e-12) half = h;
        kp->half = half;
        kp->inv_len = std::sqrt(2.0 * (half >= 0 ? half + 0.5 : k->nu)) / k->ell;
        if (half < 0) kp->lpref = (1.0 - k->nu) * std::log(2.0) - std::lgamma(k->nu);
    } else if (k->family == TK_SLATER) {
        if (!finite(k->alpha) || k->alpha <= 0) return fail(TK_EINVAL, "Slater alpha must be > 0");
        if (!finite(k->p) || k->p <= 0 || k->p > 2) return fail(TK_EINVAL, "Slater p must be in (0, 2]");
        kp->inv_len = 1.0 / k->ell;
    } else if (k->family == TK_GAUSS) {
        kp->inv_len = 1.0 / k->ell;
    } else if (k->family == TK_SPECTRAL) {
        if (!finite(k->nu) || k->nu <= 0 || k->nu > MATERN_NU_MAX)
            return fail(TK_EINVAL, "spectral density nu must be in (0, %g]", MATERN_NU_MAX);
        if (!finite(k->alpha) || k->alpha <= 0) return fail(TK_EINVAL, "spectral density alpha must be > 0");
        kp->alpha = k->alpha * k->alpha;
        kp->inv_len = 1.0;
        kp->lpref = std::lgamma(k->nu + 1.5) - std::lgamma(k->nu) + 2.0 * k->nu * std::log(k->alpha) -
                    1.5 * std::log(M_PI);
    } else {
        return fail(TK_EINVAL, "unknown kernel family %d", k->family);
    }
    return TK_OK;
}

tk_status check_grid(const tk_grid* g)
{
    if (!g) return fail(TK_EINVAL, "grid is NULL");
    for (int k = 0; k < 3; ++k) {
        if (g->n[k] < 2) return fail(TK_EINVAL, "grid n[%d]=%d must be >= 2", k, g->n[k]);
        if (g->n[k] > NMAX) return fail(TK_EUNSUPPORTED, "grid n[%d]=%d exceeds %d", k, g->n[k], NMAX);
        if (!finite(g->b[k]) || g->b[k] <= 0) return fail(TK_EINVAL, "grid b[%d] must be finite and > 0", k);
    }
    if (g->layout != TK_CENTERED && g->layout != TK_OFFSET) return fail(TK_EINVAL, "unknown layout %d", g->layout);
    return TK_OK;
}

GridAxes axes_of(const tk_grid* g)
{
    GridAxes a;
    for (int k = 0; k < 3; ++k) {
        a.n[k] = g->n[k];
        a.h[k] = 2.0 * g->b[k] / (double)(g->n[k] - 1);
        a.x0[k] = (g->layout == TK_CENTERED) ? -g->b[k] : 0.0;
    }
    return a;
}

struct Plan {
    int n[3];
    int R[3];          // working ranks (HOSVD/HOOI)
    int p[3];          // eigensolver block per mode
    int prec;
    bool eps_mode;
    double eps;
    int sweeps;
    bool converge;     // HOOI until | ||G|| - ||G_prev|| | <= 1e-13 ||A|| (at most `sweeps`)
    const double* init_U[3];   // start factors (n_k x R_k, orthonormal) instead of the HOSVD
    bool cubic;
    int gsplit[3];     // K chunks per tile pair of the Gram of A per mode (0: default)
};

tk_status make_plan(const tk_grid* g, const tk_opts* o, Plan* P)
{
    if (!o) return fail(TK_EINVAL, "opts is NULL");
    if (o->prec < TK_FP64 || o->prec > TK_BF16X3) return fail(TK_EINVAL, "unknown precision %d", o->prec);
    if (!finite(o->eps) || o->eps < 0) return fail(TK_EINVAL, "eps must be finite and >= 0");
    P->prec = o->prec;
    P->eps_mode = o->eps > 0;
    P->eps = o->eps;
    P->converge = o->hooi_sweeps == TK_HOOI_CONVERGE;
    P->sweeps = P->converge ? CONVERGE_MAX_SWEEPS : o->hooi_sweeps < 0 ? DEFAULT_SWEEPS : o->hooi_sweeps;
    if (P->sweeps > 100) return fail(TK_EINVAL, "hooi_sweeps=%d too large", o->hooi_sweeps);
    int rmax = o->r_max > 0 ? o->r_max : DEFAULT_RMAX;
    if (rmax > LIB_RMAX) return fail(TK_EUNSUPPORTED, "r_max=%d exceeds %d", rmax, LIB_RMAX);
    for (int k = 0; k < 3; ++k) {
        P->n[k] = g->n[k];
        int want;
        if (P->eps_mode) want = rmax;
        else {
            if (o->ranks[k] < 1) return fail(TK_EINVAL, "ranks[%d]=%d: give eps > 0 or ranks >= 1", k, o->ranks[k]);
            want = o->ranks[k];
            if (want > LIB_RMAX && want < g->n[k])
                return fail(TK_EUNSUPPORTED, "rank %d exceeds %d", want, LIB_RMAX);
        }
        P->R[k] = want < g->n[k] ? want : g->n[k];
        if (P->R[k] > EIG_PMAX) return fail(TK_EUNSUPPORTED, "rank %d exceeds %d", P->R[k], EIG_PMAX);
        // the float paths' A-streaming TTMs and error norm hold at most LIB_RMAX rank columns
        // in registers (three 16-column MFMA blocks); only the FP64 path goes up to EIG_PMAX
        if (P->prec != TK_FP64 && P->R[k] > LIB_RMAX)
            return fail(TK_EUNSUPPORTED, "rank %d (n[%d]=%d) exceeds %d on the FP32/BF16x3 paths", P->R[k], k,
                        g->n[k], LIB_RMAX);
        P->p[k] = (g->n[k] <= EIG_PMAX) ? g->n[k] : ((P->R[k] + 8 < EIG_PMAX) ? P->R[k] + 8 : EIG_PMAX);
    }
    P->cubic = (g->n[0] == g->n[1] && g->n[1] == g->n[2]);
    for (int k = 0; k < 3; ++k) P->gsplit[k] = 0;
    for (int k = 0; k < 3; ++k) P->init_U[k] = nullptr;
    return TK_OK;
}

// The tuned Gram split counts of the context for P's shape and precision (if any).
void apply_tuning(tk_ctx* ctx, Plan* P)
{
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    if (ctx->tune.empty()) return;
    for (int k = 0; k < 3; ++k) {
        auto it = ctx->tune.find({P->n[0], P->n[1], P->n[2], k, P->prec});
        if (it != ctx->tune.end()) P->gsplit[k] = it->second;
    }
}

// Device workspace of one compression.
struct Work {
    void* A;                 // N reals (nullptr if the caller supplies A)
    void* gram_work;
    double* G;               // 3 * nmax^2
    double *Q, *Y, *H, *Vs;  // eigensolver, 3 problems
    double* U[3];            // n_k x R_k
    float* U32[3];
    double* lam;             // 3 * 64
    double* trace;           // 3
    void* T;                 // n0 n1 R2 reals
    void* S;                 // R0 n1 n2 reals
    double* B;               // single-hole unfoldings
    double* core;            // R0 R1 R2
    double* M1;              // n0 R1 R2
    double* Hrec;            // n0 n1 R2 doubles
    double* Ahat;            // FP64 path: N doubles
    double* partials;        // 2 * nparts
    double* scal;            // a2, d2, t2, E, ...
    int* ranks;              // 3 ranks + 3 ok flags
    // eps truncation (float paths)
    double *Gc, *Vc, *lamc, *tQ, *tY, *tH, *tVs, *coreA, *coreB, *Urot[3];
    int* eflags;             // eigensolver convergence flags (FP64 path)
    double* eres;            // ... and the partial residual sums of their test
    int nparts;
    Bat bt;                  // problems sharing this layout, bt.bs bytes apart (pointers: problem 0)
    tk_ctx* ctx = nullptr;   // for the FP64 path's convergence readbacks
    bool noconv = false;     // an FP64 eigensolve stopped at its iteration cap
    bool u32_fresh = false;  // the HOSVD eigensolve wrote U32 itself (no conversion needed)
    double* rtab = nullptr;  // radial table of the grid evaluation (kernels without a fast closed form)
};

void layout_work(Arena& ar, const Plan& P, bool own_A, Work& w)
{
    const int* n = P.n;
    const int* R = P.R;
    const size_t N = (size_t)n[0] * n[1] * n[2];
    const size_t esz = (P.prec == TK_FP64) ? 8 : 4;
    int nmax = std::max(n[0], std::max(n[1], n[2]));
    int pmax = std::max(P.p[0], std::max(P.p[1], P.p[2]));
    int Rmax = std::max(R[0], std::max(R[1], R[2]));
    w.A = own_A ? (void*)ar.take<char>(N * esz) : nullptr;
    w.rtab = own_A ? ar.take<double>((size_t)radial_table_cap(n)) : nullptr;
    size_t gw = 0;
    for (int k = 0; k < 3; ++k) gw = std::max(gw, gram_work_bytes(n, k, P.prec, P.gsplit[k]));
    if (gram3_eligible(n, P.prec, P.gsplit)) gw = std::max(gw, gram3_work_bytes(n, P.prec, P.gsplit));
    {
        // the FP64 projected Grams of the HOOI sweep and the core Grams use the same workspace
        const int R0 = P.R[0], R1 = P.R[1], R2 = P.R[2];
        const int d1[3] = {n[0], R1, R2}, d2[3] = {n[1], R0, R2}, d3[3] = {R0, n[2], R1}, dc[3] = {R0, R1, R2};
        gw = std::max(gw, gram_work_bytes(d1, 0, TK_FP64));
        gw = std::max(gw, gram_work_bytes(d2, 0, TK_FP64));
        gw = std::max(gw, gram_work_bytes(d3, 1, TK_FP64));
        for (int k = 0; k < 3; ++k) gw = std::max(gw, gram_work_bytes(dc, k, TK_FP64));
    }
    w.gram_work = ar.take<char>(gw);
    w.G = ar.take<double>(3 * (size_t)nmax * nmax);
    w.Q = ar.take<double>(3 * (size_t)nmax * pmax);
    w.Y = ar.take<double>(3 * (size_t)nmax * pmax);
    w.H = ar.take<double>(3 * (size_t)pmax * pmax);
    w.Vs = ar.take<double>(3 * (size_t)pmax * pmax);
    // equal n R on every axis with 256-byte multiples: the three factors (and their FP32 copies)
    // back to back, so one batched eigensolve writes them in place (eig_modes)
    const size_t nr = (size_t)n[0] * R[0];
    const bool packed = n[1] * R[1] == (int)nr && n[2] * R[2] == (int)nr && (nr * sizeof(float)) % 256 == 0;
    if (packed) {
        double* Ub = ar.take<double>(3 * nr);
        float* Ub32 = ar.take<float>(3 * nr);
        for (int k = 0; k < 3; ++k) {
            w.U[k] = Ub + k * nr;
            w.U32[k] = Ub32 + k * nr;
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            w.U[k] = ar.take<double>((size_t)n[k] * R[k]);
            w.U32[k] = ar.take<float>((size_t)n[k] * R[k]);
        }
    }
    w.lam = ar.take<double>(3 * 64);
    w.trace = ar.take<double>(3);
    w.T = ar.take<char>((size_t)n[0] * n[1] * R[2] * esz);
    w.S = ar.take<char>((size_t)R[0] * n[1] * n[2] * esz);
    size_t nb = std::max((size_t)n[0] * R[1] * R[2], std::max((size_t)n[1] * R[0] * R[2], (size_t)R[0] * n[2] * R[1]));
    w.B = ar.take<double>(nb);
    w.core = ar.take<double>((size_t)R[0] * R[1] * R[2]);
    w.M1 = ar.take<double>((size_t)n[0] * R[1] * R[2]);
    w.Hrec = ar.take<double>((size_t)n[0] * n[1] * R[2]);
    w.Ahat = (P.prec == TK_FP64) ? ar.take<double>(N) : nullptr;
    w.nparts = std::max(recon_diff_parts((long)n[0] * n[1]), 1024);
    w.partials = ar.take<double>(2 * (size_t)w.nparts);
    w.scal = ar.take<double>(16);
    w.ranks = ar.take<int>(16);
    w.Gc = ar.take<double>(3 * (size_t)Rmax * Rmax);
    w.Vc = ar.take<double>(3 * (size_t)Rmax * Rmax);
    w.lamc = ar.take<double>(3 * 64);
    w.tQ = ar.take<double>(3 * (size_t)Rmax * Rmax);
    w.tY = ar.take<double>(3 * (size_t)Rmax * Rmax);
    w.tH = ar.take<double>(3 * (size_t)Rmax * Rmax);
    w.tVs = ar.take<double>(3 * (size_t)Rmax * Rmax);
    w.coreA = ar.take<double>((size_t)R[0] * R[1] * R[2]);
    w.coreB = ar.take<double>((size_t)R[0] * R[1] * R[2]);
    for (int k = 0; k < 3; ++k) w.Urot[k] = ar.take<double>((size_t)n[k] * R[k]);
    w.eflags = ar.take<int>(64);
    w.eres = ar.take<double>(3 * (size_t)EIG_CHECK_DOUBLES);   // eigen batches of at most 3 here
}

size_t result_bytes(const int n[3], const int r[3])
{
    Arena ar;
    for (int k = 0; k < 3; ++k) { ar.take<double>((size_t)n[k] * r[k]); ar.take<float>((size_t)n[k] * r[k]); }
    ar.take<double>((size_t)r[0] * r[1] * r[2]);
    ar.take<float>((size_t)r[0] * r[1] * r[2]);
    return ar.off;
}

// Device bytes of one compression (workspace, gather area of the final readback, result); the
// same layout as compress_impl with one problem.
size_t estimate(const Plan& P, bool own_A)
{
    Arena ar;
    Work w;
    layout_work(ar, P, own_A, w);
    return align_up(ar.off, 256) + 256 + result_bytes(P.n, P.R);
}

// ------------------------------------------------------------------------------------------
// GEMM helpers (row-major operands; see GemmArgs)
// ------------------------------------------------------------------------------------------
GemmArgs gemm(int M, int N, int K, int batch, const void* A, long sAb, long sAm, long sAk, const void* B, long sBb,
              long sBk, long sBn, void* C, long sCb, long sCm, long sCn)
{
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch; g.reduce_batch = 0;
    g.A = A; g.sAb = sAb; g.sAm = sAm; g.sAk = sAk;
    g.B = B; g.sBb = sBb; g.sBk = sBk; g.sBn = sBn;
    g.C = C; g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.alpha = 1.0; g.beta = 0.0;
    return g;
}

// A small product of the compression pipeline, over every problem of the workspace batch.
template <typename TA, typename TB, typename TC>
hipError_t wgemm(GemmArgs g, const Work& w, hipStream_t s)
{
    g.nb = w.bt.nb;
    g.bs = w.bt.bs;
    return launch_gemm<TA, TB, TC>(g, s);
}

#define TK_LAUNCH(x)                                                                               \
    do {                                                                                           \
        hipError_t _e = (x);                                                                       \
        if (_e != hipSuccess) return fail(TK_EHIP, "launch %s: %s", #x, hipGetErrorString(_e));    \
    } while (0)

// A pinned host slot and its device twin, held for the duration of one call.
struct Slot {
    tk_ctx* c;
    int i = -1;
    explicit Slot(tk_ctx* ctx) : c(ctx)
    {
        std::lock_guard<std::mutex> g(c->slot_mu);
        for (int k = 0; k < tk_ctx::kSlots; ++k)
            if (!(c->slot_used >> k & 1)) {
                c->slot_used |= 1ull << k;
                i = k;
                break;
            }
    }
    ~Slot()
    {
        if (i < 0) return;
        std::lock_guard<std::mutex> g(c->slot_mu);
        c->slot_used &= ~(1ull << i);
    }
    char* host() const { return c->pinned + (size_t)i * tk_ctx::kSlotBytes; }
    char* dev() const { return c->dev_slots + (size_t)i * tk_ctx::kSlotBytes; }
};

// Copy up to two small device ranges (together <= kSlotBytes) to host memory, stream-ordered,
// and wait once.
tk_status readback(tk_ctx* ctx, hipStream_t s, const void* src0, size_t bytes0, void* dst0,
                   const void* src1 = nullptr, size_t bytes1 = 0, void* dst1 = nullptr)
{
    Slot slot(ctx);
    const size_t off1 = (bytes0 + 15) & ~(size_t)15;
    if (slot.i < 0 || off1 + bytes1 > tk_ctx::kSlotBytes) {
        TK_HIP(hipMemcpyAsync(dst0, src0, bytes0, hipMemcpyDeviceToHost, s));
        if (bytes1) TK_HIP(hipMemcpyAsync(dst1, src1, bytes1, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        return TK_OK;
    }
    TK_HIP(hipMemcpyAsync(slot.host(), src0, bytes0, hipMemcpyDeviceToHost, s));
    if (bytes1) TK_HIP(hipMemcpyAsync(slot.host() + off1, src1, bytes1, hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    std::memcpy(dst0, slot.host(), bytes0);
    if (bytes1) std::memcpy(dst1, slot.host() + off1, bytes1);
    return TK_OK;
}

// FP64 path: the block subspace iteration runs until its Ritz pairs pass the residual test of
// launch_eig_check (|| G u_j - lam_j u_j || <= max(EIG_TAU lam_j, EIG_CFLOOR sqrt(n) u ||G||_F)),
// EIG_ROUND_ITERS more iterations per failed test, at most EIG_MAX_ROUNDS rounds; the flags are
// read back after each test.  A problem still failing at the cap sets w.noconv (the call then
// returns TK_ENOCONV with its result).  The block Q of the last iteration is the warm start of
// the next round, so every round continues the same iteration.
constexpr double EIG_TAU = 1e-12;
constexpr double EIG_CFLOOR = 4.0;
constexpr int EIG_ROUND_ITERS = 2;
constexpr int EIG_MAX_ROUNDS = 16;
tk_status eig_converge(const EigBatch& b, Work& w, hipStream_t s)
{
    if (b.span_only || b.p >= b.n || b.count > 64 || !w.ctx) return TK_OK;
    for (int round = 0;; ++round) {
        TK_LAUNCH(launch_eig_check(b, EIG_TAU, EIG_CFLOOR, w.eflags, w.eres, s));
        int fl[64];
        tk_status st = readback(w.ctx, s, w.eflags, sizeof(int) * (size_t)b.count, fl);
        if (st != TK_OK) return st;
        bool all = true;
        for (int c = 0; c < b.count; ++c) all = all && fl[c] == 1;
        if (all) return TK_OK;
        if (round == EIG_MAX_ROUNDS) {
            w.noconv = true;
            return TK_OK;
        }
        EigBatch rb = b;
        rb.warm = b.Q;
        rb.sW = (long)b.n * b.p;
        rb.rw = b.p;
        rb.ldw = b.p;
        rb.trace = nullptr;
        ProfScope ps(TK_PROF_EIG, s);
        TK_LAUNCH(launch_eig(rb, EIG_ROUND_ITERS, s));
    }
}

// Leading R_k eigenvectors of the three Grams in w.G (stride nmax^2), HOSVD start.
tk_status eig_modes(const Plan& P, Work& w, int nmax, hipStream_t s)
{
    // With the eps rule on a float path the factors end up rotated to the core's HOSVD basis,
    // so the HOSVD start only has to span the leading subspace: an R-column block iterated
    // SPAN_ITERS_F32 times (its leading k-dimensional part converges like (lambda_{R+1} /
    // lambda_k)^iters for the eps rank k << R), without the Rayleigh-Ritz rotation.
    const bool span = P.eps_mode && P.prec != TK_FP64;
    // one launch for the three modes when they share n, p and R
    if (P.cubic && P.R[0] == P.R[1] && P.R[1] == P.R[2] && P.p[0] == P.p[1] && P.p[1] == P.p[2]) {
        EigBatch b{};
        b.count = 3; b.n = P.n[0]; b.p = P.p[0]; b.r = P.R[0]; b.rw = 0; b.ldw = 0;
        if (span && P.R[0] < P.n[0]) { b.p = P.R[0]; b.span_only = 1; }
        b.G = w.G; b.sG = (long)nmax * nmax;
        b.Q = w.Q; b.Y = w.Y; b.H = w.H; b.Vs = w.Vs;
        // the factors are written in place when layout_work packed them back to back, else into a
        // staging area and copied
        const long nr = (long)P.n[0] * P.R[0];
        const bool packed = w.U[1] == w.U[0] + nr && w.U[2] == w.U[1] + nr && w.U32[1] == w.U32[0] + nr &&
                            w.U32[2] == w.U32[1] + nr;
        b.U = packed ? w.U[0] : w.Y; b.sU = nr; b.ldu = P.R[0];
        if (packed && P.prec != TK_FP64) b.U32 = w.U32[0];
        b.lam = w.lam; b.sL = 64;
        b.trace = w.trace; b.sTrace = 1;
        b.nb = w.bt.nb; b.bs = w.bt.bs;
        b.cholqr = w.ctx ? w.ctx->cholqr : CholQr{};
        // the eigensolver writes U after its last use of Y, so U may alias Y
        {
            ProfScope ps(TK_PROF_EIG, s);
            TK_LAUNCH(launch_eig(b, b.span_only ? SPAN_ITERS_F32 : (P.prec == TK_FP64 ? COLD_ITERS : COLD_ITERS_F32), s));
        }
        if (P.prec == TK_FP64) {
            tk_status st = eig_converge(b, w, s);
            if (st != TK_OK) return st;
        }
        if (packed) {
            w.u32_fresh = (b.U32 != nullptr);
        } else {
            for (int k = 0; k < 3; ++k)
                TK_LAUNCH(launch_copy_f64(w.Y + (long)k * nr, w.U[k], nr, s, w.bt));
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            EigBatch b{};
            b.count = 1; b.n = P.n[k]; b.p = P.p[k]; b.r = P.R[k];
            b.G = w.G + (long)k * nmax * nmax; b.sG = 0;
            b.Q = w.Q; b.Y = w.Y; b.H = w.H; b.Vs = w.Vs;
            b.U = w.U[k]; b.sU = 0; b.ldu = P.R[k];
            b.lam = w.lam + 64 * k; b.sL = 64;
            b.trace = w.trace + k; b.sTrace = 1;
            b.nb = w.bt.nb; b.bs = w.bt.bs;
            b.cholqr = w.ctx ? w.ctx->cholqr : CholQr{};
            if (span && P.R[k] < P.n[k]) { b.p = P.R[k]; b.span_only = 1; }
            {
                ProfScope ps(TK_PROF_EIG, s);
                TK_LAUNCH(launch_eig(b, b.span_only ? SPAN_ITERS_F32 : (P.prec == TK_FP64 ? COLD_ITERS : COLD_ITERS_F32), s));
            }
            if (P.prec == TK_FP64) {
                tk_status st = eig_converge(b, w, s);
                if (st != TK_OK) return st;
            }
        }
    }
    return TK_OK;
}

// Leading R_k eigenvectors of one symmetric n_k x n_k matrix Gs, warm-started from w.U[k];
// u32 (optional) receives the FP32 copy of the new factor.
tk_status eig_update(const Plan& P, Work& w, int k, const double* Gs, hipStream_t s, float* u32)
{
    EigBatch b{};
    // warm start from the current factor.  Float paths: the block is the factor itself
    // (orthonormal, no QR) and one power step per HOOI update; FP64: oversampled block and
    // converged eigenvectors, so every HOOI step is exact as in the oracle.  With the eps rule
    // on a float path the factors are rotated to the core's HOSVD basis at the end, so a HOOI
    // update only has to deliver the subspace: the power-stepped block itself, orthonormalised.
    // (also for n <= EIG_PMAX: a full n x n Jacobi costs far more than one block step)
    b.count = 1; b.n = P.n[k]; b.r = P.R[k];
    const bool span = P.eps_mode && P.prec != TK_FP64 && P.R[k] < P.n[k];
    b.p = span ? P.R[k] : (P.n[k] <= EIG_PMAX) ? P.n[k] : (P.prec == TK_FP64 ? P.p[k] : P.R[k]);
    b.span_only = span ? 1 : 0;
    b.rw = P.R[k]; b.ldw = P.R[k]; b.warm = w.U[k]; b.sW = 0;
    b.G = Gs; b.sG = 0;
    b.Q = w.Q; b.Y = w.Y; b.H = w.H; b.Vs = w.Vs;
    // span-only: the last QR writes U[k] itself (the start block has read it by then); otherwise
    // a staging area, copied to U[k] afterwards
    b.U = span ? w.U[k] : w.Y + (long)P.n[k] * P.p[k];
    b.sU = 0; b.ldu = P.R[k];
    b.lam = w.lam + 64 * k; b.sL = 64;
    b.trace = nullptr;
    b.nb = w.bt.nb; b.bs = w.bt.bs;
    b.U32 = u32;
    b.cholqr = w.ctx ? w.ctx->cholqr : CholQr{};
    {
        ProfScope ps(TK_PROF_EIG, s);
        TK_LAUNCH(launch_eig(b, P.prec == TK_FP64 ? WARM_ITERS : WARM_ITERS_F32, s));
    }
    if (P.prec == TK_FP64) {
        tk_status st = eig_converge(b, w, s);
        if (st != TK_OK) return st;
    }
    if (!span) TK_LAUNCH(launch_copy_f64(b.U, w.U[k], (long)P.n[k] * P.R[k], s, w.bt));
    return TK_OK;
}

template <typename Real>
tk_status refresh_u32(const Plan& P, Work& w, int k, hipStream_t s)
{
    if (sizeof(Real) == 4) TK_LAUNCH(launch_convert_f64_to_f32(w.U[k], w.U32[k], (long)P.n[k] * P.R[k], s, w.bt));
    return TK_OK;
}

// T = A x_3 U3^T  (rows = n0 n1, r = R2)
template <typename Real>
tk_status ttm_last(const Plan& P, Work& w, const Real* A, hipStream_t s)
{
    long rows = (long)P.n[0] * P.n[1];
    ProfScope ps(TK_PROF_TTM, s);
    if (sizeof(Real) == 4) {
        TK_LAUNCH(launch_ttm_last_f32((const float*)A, rows, P.n[2], w.U32[2], P.R[2], (float*)w.T, s, w.bt));
    } else {
        GemmArgs g = gemm((int)rows, P.R[2], P.n[2], 1, A, 0, P.n[2], 1, w.U[2], 0, P.R[2], 1, w.T, 0, P.R[2], 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
    }
    return TK_OK;
}

// S = A x_1 U1^T  (R0 x n1 n2)
template <typename Real>
tk_status ttm_first(const Plan& P, Work& w, const Real* A, hipStream_t s)
{
    long cols = (long)P.n[1] * P.n[2];
    ProfScope ps(TK_PROF_TTM, s);
    if (sizeof(Real) == 4) {
        TK_LAUNCH(launch_ttm_first_f32((const float*)A, P.n[0], cols, w.U32[0], P.R[0], (float*)w.S, s, w.bt));
    } else {
        GemmArgs g = gemm(P.R[0], (int)cols, P.n[0], 1, w.U[0], 0, 1, P.R[0], A, 0, cols, 1, w.S, 0, cols, 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
    }
    return TK_OK;
}

template <typename Real>
hipError_t gemm_rd(const GemmArgs& g, const Work& w, hipStream_t s)   // Real operand A, double B, double C
{
    return wgemm<Real, double, double>(g, w, s);
}
template <typename Real>
hipError_t gemm_dr(const GemmArgs& g, const Work& w, hipStream_t s)   // double A, Real B, double C
{
    return wgemm<double, Real, double>(g, w, s);
}

// B1[i0][b][c] = sum_i1 U2[i1][b] T[i0][i1][c]
template <typename Real>
tk_status single_hole_1(const Plan& P, Work& w, hipStream_t s)
{
    const int n0 = P.n[0], n1 = P.n[1], R1 = P.R[1], R2 = P.R[2];
    GemmArgs g = gemm(R1, R2, n1, n0, w.U[1], 0, 1, R1, w.T, (long)n1 * R2, R2, 1, w.B, (long)R1 * R2, R2, 1);
    TK_LAUNCH(gemm_dr<Real>(g, w, s));
    return TK_OK;
}

// small Gram of a row-major n x K unfolding stored in w.B -> Gs (n x n)
// G = mode-`mode` Gram of the small FP64 tensor B (dims d, C-order): split-K FP64 MFMA tiles
// with a fixed-order reduction, as for the Grams of A.
tk_status small_gram(const int d[3], int mode, const double* B, double* G, void* work, hipStream_t s, Bat bt)
{
    TK_LAUNCH(launch_gram(B, d, mode, TK_FP64, G, work, s, bt));
    return TK_OK;
}

template <typename Real>
tk_status hooi_sweep(const Plan& P, Work& w, const Real* A, int nmax, hipStream_t s)
{
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
    const int R0 = P.R[0], R1 = P.R[1], R2 = P.R[2];
    double* Gs = w.G;   // reuse the first Gram slot
    tk_status st;
    // ---- mode 1: B1 = A x_2 U2^T x_3 U3^T
    if ((st = ttm_last<Real>(P, w, A, s)) != TK_OK) return st;
    if ((st = single_hole_1<Real>(P, w, s)) != TK_OK) return st;
    {
        const int d[3] = {n0, R1, R2};
        if ((st = small_gram(d, 0, w.B, Gs, w.gram_work, s, w.bt)) != TK_OK) return st;
    }
    if ((st = eig_update(P, w, 0, Gs, s, sizeof(Real) == 4 ? w.U32[0] : nullptr)) != TK_OK) return st;
    // ---- mode 2: B2[i1][a][c] = sum_i0 U1[i0][a] T[i0][i1][c]  (T still holds A x_3 U3^T)
    {
        GemmArgs g = gemm(R0, R2, n0, n1, w.U[0], 0, 1, R0, w.T, R2, (long)n1 * R2, 1, w.B, (long)R0 * R2, R2, 1);
        TK_LAUNCH(gemm_dr<Real>(g, w, s));
    }
    {
        const int d[3] = {n1, R0, R2};
        if ((st = small_gram(d, 0, w.B, Gs, w.gram_work, s, w.bt)) != TK_OK) return st;
    }
    if ((st = eig_update(P, w, 1, Gs, s, sizeof(Real) == 4 ? w.U32[1] : nullptr)) != TK_OK) return st;
    // ---- mode 3: S = A x_1 U1^T, B3[a][i2][b] = sum_i1 S[a][i1][i2] U2[i1][b]
    if ((st = ttm_first<Real>(P, w, A, s)) != TK_OK) return st;
    {
        GemmArgs g = gemm(n2, R1, n1, R0, w.S, (long)n1 * n2, 1, n2, w.U[1], 0, R1, 1, w.B, (long)n2 * R1, R1, 1);
        TK_LAUNCH(gemm_rd<Real>(g, w, s));
    }
    {
        // Gs[i2][i2'] = sum_a sum_b B3[a][i2][b] B3[a][i2'][b]: the mode-2 Gram of B3 (R0 x n2 x R1)
        const int d[3] = {R0, n2, R1};
        if ((st = small_gram(d, 1, w.B, Gs, w.gram_work, s, w.bt)) != TK_OK) return st;
    }
    if ((st = eig_update(P, w, 2, Gs, s, sizeof(Real) == 4 ? w.U32[2] : nullptr)) != TK_OK) return st;
    // ---- core[a][b][c] = sum_i2 B3[a][i2][b] U3[i2][c]
    {
        GemmArgs g = gemm(R1, R2, n2, R0, w.B, (long)n2 * R1, 1, R1, w.U[2], 0, R2, 1, w.core, (long)R1 * R2, R2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
    }
    (void)nmax;
    return TK_OK;
}

// HOSVD core: G = A x_1 U1^T x_2 U2^T x_3 U3^T via T and B1.
template <typename Real>
tk_status hosvd_core(const Plan& P, Work& w, const Real* A, hipStream_t s)
{
    tk_status st;
    if ((st = ttm_last<Real>(P, w, A, s)) != TK_OK) return st;
    if ((st = single_hole_1<Real>(P, w, s)) != TK_OK) return st;
    const int n0 = P.n[0], R0 = P.R[0], R1 = P.R[1], R2 = P.R[2];
    GemmArgs g = gemm(R0, R1 * R2, n0, 1, w.U[0], 0, 1, R0, w.B, 0, (long)R1 * R2, 1, w.core, 0, (long)R1 * R2, 1);
    TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
    return TK_OK;
}

// scal[0] = ||A||^2, scal[1] = ||A - core x_1 U1 x_2 U2 x_3 U3||^2 (factors n_k x R_k, FP64).
template <typename Real>
tk_status recon_norm(const Plan& P, Work& w, const Real* A, double* const Uf[3], const double* corep, hipStream_t s)
{
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
    const int R0 = P.R[0], R1 = P.R[1], R2 = P.R[2];
    // M1[i0][b][c] = sum_a U1[i0][a] core[a][b][c]
    {
        GemmArgs g = gemm(n0, R1 * R2, R0, 1, Uf[0], 0, R0, 1, corep, 0, (long)R1 * R2, 1, w.M1, 0, (long)R1 * R2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
    }
    // H[i0][i1][c] = sum_b U2[i1][b] M1[i0][b][c]   (FP64)
    {
        GemmArgs g = gemm(n1, R2, R1, n0, Uf[1], 0, R1, 1, w.M1, (long)R1 * R2, R2, 1, w.Hrec, (long)n1 * R2, R2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
    }
    long rows = (long)n0 * n1;
    ProfScope ps(TK_PROF_NORM, s);
    if (sizeof(Real) == 4) {
        int parts = recon_diff_parts(rows);
        TK_LAUNCH(launch_recon_diff_f32((const float*)A, rows, n2, w.Hrec, Uf[2], R2, w.partials, s, w.bt));
        TK_LAUNCH(launch_reduce_partials(w.partials, parts, 2, w.scal, s, w.bt));
    } else {
        GemmArgs g = gemm((int)rows, n2, R2, 1, w.Hrec, 0, R2, 1, Uf[2], 0, 1, R2, w.Ahat, 0, n2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
        int parts = 1024;
        TK_LAUNCH(launch_diff_norm<double>((const double*)A, w.Ahat, rows * n2, w.partials, parts, s, w.bt));
        TK_LAUNCH(launch_reduce_partials(w.partials, parts, 2, w.scal, s, w.bt));
    }
    // the partials are (a2, d2) per work-group: scal[0] = a2, scal[1] = d2
    return TK_OK;
}

// eps truncation of a rank-R result by the HOSVD of its core (float paths): the eigenvectors
// of the three core Grams rotate the factors and the core to the core's HOSVD basis, and the
// eps rule on their eigenvalues (with the measured d2 = ||A - A_R||^2) picks the ranks.
tk_status core_truncate(const Plan& P, Work& w, hipStream_t s)
{
    const int R0 = P.R[0], R1 = P.R[1], R2 = P.R[2];
    const int Rm = std::max(R0, std::max(R1, R2));
    const long RR = (long)Rm * Rm;
    // core Grams (R_k x R_k, leading dimension R_k, at Gc + k RR)
    {
        const int d[3] = {R0, R1, R2};
        tk_status st;
        for (int k = 0; k < 3; ++k)
            if ((st = small_gram(d, k, w.core, w.Gc + k * RR, w.gram_work, s, w.bt)) != TK_OK) return st;
    }
    // full eigendecompositions (p = n = R_k); one launch for the three modes when the ranks agree
    if (R0 == R1 && R1 == R2) {
        EigBatch b{};
        b.count = 3; b.n = R0; b.p = R0; b.r = R0;
        b.G = w.Gc; b.sG = RR;
        b.Q = w.tQ; b.Y = w.tY; b.H = w.tH; b.Vs = w.tVs;     // problem strides R0^2 == RR
        b.U = w.Vc; b.sU = RR; b.ldu = R0;
        b.lam = w.lamc; b.sL = 64;
        b.trace = nullptr;
        b.nb = w.bt.nb; b.bs = w.bt.bs;
        b.jacobi_tol = CORE_JACOBI_TOL;
        TK_LAUNCH(launch_eig(b, 0, s));
    } else {
        for (int k = 0; k < 3; ++k) {
            EigBatch b{};
            b.count = 1; b.n = P.R[k]; b.p = P.R[k]; b.r = P.R[k];
            b.G = w.Gc + k * RR; b.sG = 0;
            b.Q = w.tQ + k * RR; b.Y = w.tY + k * RR; b.H = w.tH + k * RR; b.Vs = w.tVs + k * RR;
            b.U = w.Vc + k * RR; b.sU = 0; b.ldu = P.R[k];
            b.lam = w.lamc + 64 * k; b.sL = 64;
            b.trace = nullptr;
            b.nb = w.bt.nb; b.bs = w.bt.bs;
            b.jacobi_tol = CORE_JACOBI_TOL;
            TK_LAUNCH(launch_eig(b, 0, s));
        }
    }
    // ranks: budget = (eps^2 a2 - d2) / 3 per mode (one launch for the three modes when their
    // rank caps agree)
    if (P.R[0] == P.R[1] && P.R[1] == P.R[2]) {
        TK_LAUNCH(launch_rank_rule(w.lamc, 64, P.R[0], 3, nullptr, 0, w.scal, 1, P.eps * P.eps, w.ranks, w.ranks + 3,
                                   s, w.bt));
    } else {
        for (int k = 0; k < 3; ++k)
            TK_LAUNCH(launch_rank_rule(w.lamc + 64 * k, 64, P.R[k], 1, nullptr, 0, w.scal, 1, P.eps * P.eps,
                                       w.ranks + k, w.ranks + 3 + k, s, w.bt));
    }
    // rotate factors: Urot_k = U_k V_k
    for (int k = 0; k < 3; ++k) {
        GemmArgs g = gemm(P.n[k], P.R[k], P.R[k], 1, w.U[k], 0, P.R[k], 1, w.Vc + k * RR, 0, P.R[k], 1, w.Urot[k], 0,
                          P.R[k], 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
        // sign rule on the rotated factor; the flips go into V_k so that the core follows
        TK_LAUNCH(launch_signfix_pair(w.Urot[k], P.R[k], P.n[k], w.Vc + k * RR, P.R[k], P.R[k], P.R[k], s, w.bt));
    }
    // rotate core: coreB = core x_1 V1^T x_2 V2^T x_3 V3^T
    {
        GemmArgs g = gemm(R0, R1 * R2, R0, 1, w.Vc, 0, 1, R0, w.core, 0, (long)R1 * R2, 1, w.coreA, 0, (long)R1 * R2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g, w, s)));
        GemmArgs g1 = gemm(R1, R2, R1, R0, w.Vc + RR, 0, 1, R1, w.coreA, (long)R1 * R2, R2, 1, w.coreB, (long)R1 * R2,
                           R2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g1, w, s)));
        GemmArgs g2 = gemm(R0 * R1, R2, R2, 1, w.coreB, 0, R2, 1, w.Vc + 2 * RR, 0, R2, 1, w.coreA, 0, R2, 1);
        TK_LAUNCH((wgemm<double, double, double>(g2, w, s)));
    }
    // the error of the truncated result is measured against A afterwards (its caller), so the
    // core's discarded energy is not formed here
    return TK_OK;
}

// held: a reservation of the caller that covers the result (its share is handed over).
tk_status alloc_result(tk_ctx* ctx, const int n[3], const int r[3], hipStream_t s, tk_tucker** out,
                       Reservation* held = nullptr)
{
    tk_tucker* t = new (std::nothrow) tk_tucker();
    if (!t) return fail(TK_ENOMEM, "host allocation failed");
    t->ctx = ctx;
    size_t bytes = result_bytes(n, r);
    if (!(held && held->hand_over(bytes)) && !reserve(ctx, bytes)) {
        delete t;
        return fail(TK_ENOMEM, "result (%zu bytes) exceeds the remaining HBM budget", bytes);
    }
    t->bytes = bytes;
    // results live long and are small: they come from the device heap, not from the
    // stream-ordered pool of the (large, short-lived) workspaces, which they would fragment;
    // the block of a freed result of the same size class (at most twice the size) is reused
    void* blk = nullptr;
    size_t blk_bytes = 0;
    {
        std::lock_guard<std::mutex> g(ctx->rc_mu);
        auto it = ctx->rcache.lower_bound(bytes);
        if (it != ctx->rcache.end() && it->first <= 2 * bytes) {
            blk = it->second;
            blk_bytes = it->first;
            ctx->rcache_bytes -= it->first;
            ctx->idle.fetch_sub(it->first);
            ctx->rcache.erase(it);
        }
    }
    if (!blk) {
        hipError_t e = hipMalloc(&blk, bytes);
        if (e != hipSuccess) {
            release(ctx, bytes);
            delete t;
            return fail(TK_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
        blk_bytes = bytes;
    }
    // a reused block larger than the result is charged at its full size (or not reused)
    if (blk_bytes > bytes) {
        if (reserve(ctx, blk_bytes - bytes, false)) {
            bytes = blk_bytes;
        } else {
            (void)hipFree(blk);
            blk = nullptr;
            hipError_t e = hipMalloc(&blk, bytes);
            if (e != hipSuccess) {
                release(ctx, bytes);
                delete t;
                return fail(TK_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
            }
            blk_bytes = bytes;
        }
        t->bytes = bytes;
    }
    t->block = blk;
    t->block_bytes = blk_bytes;
    t->stream = s;
    Arena ar;
    ar.base = (char*)blk;
    for (int k = 0; k < 3; ++k) {
        t->n[k] = n[k];
        t->r[k] = r[k];
        t->U[k] = ar.take<double>((size_t)n[k] * r[k]);
        t->U32[k] = ar.take<float>((size_t)n[k] * r[k]);
    }
    t->core = ar.take<double>((size_t)r[0] * r[1] * r[2]);
    t->core32 = ar.take<float>((size_t)r[0] * r[1] * r[2]);
    {
        std::lock_guard<std::mutex> g(ctx->life_mu);
        ++ctx->live_results;
    }
    *out = t;
    return TK_OK;
}

void free_result(tk_tucker* t)
{
    if (!t) return;
    tk_ctx* ctx = t->ctx;
    if (t->block) {
        // the result may have been read on any stream: its block is released (kept for the
        // next result, or freed) once the device is idle
        hipSetDevice(ctx->device);
        hipDeviceSynchronize();
        bool kept = false;
        {
            std::lock_guard<std::mutex> g(ctx->life_mu);
            if (!ctx->closing) {
                std::lock_guard<std::mutex> g2(ctx->rc_mu);
                if (ctx->rcache.size() < tk_ctx::kResultCache &&
                    ctx->rcache_bytes + t->block_bytes <= tk_ctx::kResultCacheBytes) {
                    ctx->rcache.emplace(t->block_bytes, t->block);
                    ctx->rcache_bytes += t->block_bytes;
                    ctx->idle.fetch_add(t->block_bytes);
                    kept = true;
                }
            }
        }
        if (!kept) hipFree(t->block);
    }
    release(ctx, t->bytes);
    delete t;
    bool last = false;
    {
        std::lock_guard<std::mutex> g(ctx->life_mu);
        last = (--ctx->live_results == 0) && ctx->closing;
    }
    if (last) delete ctx;
}

// Results of a destroyed context can only be freed.
bool usable(const tk_tucker* t)
{
    if (!t) return false;
    std::lock_guard<std::mutex> g(t->ctx->life_mu);
    return !t->ctx->closing;
}

tk_status fill_result_from(tk_tucker* t, const double* const Usrc[3], const int ldU[3], const double* core,
                           const int Rc[3], hipStream_t s)
{
    for (int k = 0; k < 3; ++k) {
        TK_HIP(hipMemcpy2DAsync(t->U[k], sizeof(double) * t->r[k], Usrc[k], sizeof(double) * ldU[k],
                                sizeof(double) * t->r[k], t->n[k], hipMemcpyDeviceToDevice, s));
        TK_LAUNCH(launch_convert_f64_to_f32(t->U[k], t->U32[k], (long)t->n[k] * t->r[k], s));
    }
    TK_LAUNCH((launch_copy_block<double, double>(core, Rc[1], Rc[2], t->core, t->r[0], t->r[1], t->r[2], s)));
    TK_LAUNCH((launch_copy_block<double, float>(core, Rc[1], Rc[2], t->core32, t->r[0], t->r[1], t->r[2], s)));
    return TK_OK;
}

// Replay of a captured pipeline: the launches of `pipeline` are captured once per shape,
// options, batch size and workspace address and replayed afterwards, with the grid evaluation
// node updated to this call's kernel parameters.
template <typename Real, typename F>
tk_status run_captured(tk_ctx* ctx, const Plan& P, int nb, void* base, const tk_grid* grid, const KernelParams* kps,
                       const Work& w, hipStream_t s, F& pipeline)
{
    std::array<long, 19> key{};
    long epsbits = 0;
    std::memcpy(&epsbits, &P.eps, sizeof(epsbits));
    const long vals[19] = {P.n[0], P.n[1], P.n[2], P.R[0], P.R[1], P.R[2], P.p[0], P.p[1], P.p[2], P.prec,
                           epsbits, P.sweeps, P.gsplit[0], P.gsplit[1], P.gsplit[2], nb,
                           (long)(intptr_t)base, (long)sizeof(Real), P.eps_mode ? 1 : 0};
    for (int i = 0; i < 19; ++i) key[i] = vals[i];
    GridEvalNode nd;
    const GridAxes ax = axes_of(grid);
    if (sizeof(Real) == 4) grid_eval_node_f32((float*)w.A, ax, kps, w.bt, &nd);
    else grid_eval_node_f64((double*)w.A, ax, kps, w.bt, &nd);
    std::lock_guard<std::mutex> g(ctx->graph_mu);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 64) {
            for (auto& kv : ctx->graphs) {
                (void)hipGraphExecDestroy(kv.second.ex);
                (void)hipGraphDestroy(kv.second.g);
            }
            ctx->graphs.clear();
        }
        // captured on a stream of its own (the caller's may be the null stream, which cannot
        // capture); the graph then runs on the caller's stream
        tk_ctx::GraphEntry e;
        hipStream_t cs = nullptr;
        TK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (be != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return fail(TK_EHIP, "stream capture: %s", hipGetErrorString(be));
        }
        const tk_status st = pipeline(cs);
        const hipError_t ce = hipStreamEndCapture(cs, &e.g);
        (void)hipStreamDestroy(cs);
        if (st != TK_OK) {
            if (e.g) (void)hipGraphDestroy(e.g);
            return st;
        }
        if (ce != hipSuccess) return fail(TK_EHIP, "stream capture: %s", hipGetErrorString(ce));
        size_t cnt = 0;
        TK_HIP(hipGraphGetNodes(e.g, nullptr, &cnt));
        std::vector<hipGraphNode_t> nodes(cnt);
        TK_HIP(hipGraphGetNodes(e.g, nodes.data(), &cnt));
        for (hipGraphNode_t node : nodes) {
            hipGraphNodeType t;
            if (hipGraphNodeGetType(node, &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(node, &kp) == hipSuccess && kp.func == nd.p.func) {
                e.grid_node = node;
                break;
            }
        }
        if (!e.grid_node) {
            (void)hipGraphDestroy(e.g);
            return fail(TK_EHIP, "captured pipeline has no grid evaluation node");
        }
        hipError_t ie = hipGraphInstantiate(&e.ex, e.g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(e.g);
            return fail(TK_EHIP, "graph instantiation: %s", hipGetErrorString(ie));
        }
        it = ctx->graphs.emplace(key, e).first;
    } else {
        TK_HIP(hipGraphExecKernelNodeSetParams(it->second.ex, it->second.grid_node, &nd.p));
    }
    TK_HIP(hipGraphLaunch(it->second.ex, s));
    return TK_OK;
}

// Bytes of nb workspaces of plan P laid out back to back (stride ws), plus the gather area of
// the final readback.
size_t batch_layout(const Plan& P, bool own_A, int nb, size_t* ws)
{
    Arena plan;
    Work w;
    layout_work(plan, P, own_A, w);
    *ws = align_up(plan.off, 256);
    return *ws * (size_t)nb + align_up((size_t)nb * 64, 256);
}

// The compression pipeline for nb problems of one shape: problem b samples kps[b] on `grid`
// (A_in: one caller tensor instead, nb == 1).  The problems' workspaces lie ws bytes apart and
// every launch covers all of them (grid z), each problem running the work-groups it runs alone.
// outs[b] / sts[b]: the result and TK_OK or TK_ENOCONV (eps not met; the result is returned
// anyway).  Any other error is returned for the whole call, with no results.
// A chunk of an uneven batch whose workspace the batch laid out (and charged) beforehand, with
// the problems' tensors already evaluated there by the batch's persistent grid launch.
struct BatchSlot {
    void* base;
};

template <typename Real>
tk_status compress_impl(tk_ctx* ctx, const KernelParams* kps, int nb, const void* A_in, const tk_grid* grid, Plan P,
                        hipStream_t s, tk_tucker** outs, tk_status* sts, const BatchSlot* slot = nullptr)
{
    const bool own_A = (A_in == nullptr);
    if (nb < 1 || nb > BATCH_MAX || (!own_A && nb != 1)) return fail(TK_EINVAL, "batch of %d problems", nb);
    if (nb > 1 && (P.prec == TK_FP64 || P.converge))
        return fail(TK_EINVAL, "the FP64 path and converged HOOI read back between steps: one problem per call");
    if (slot && (!own_A || sizeof(Real) != 4)) return fail(TK_EINVAL, "batch slot: float tensors of the batch only");
    for (int b = 0; b < nb; ++b) { outs[b] = nullptr; sts[b] = TK_OK; }
    size_t ws = 0;
    const size_t total = batch_layout(P, own_A, nb, &ws);
    const size_t need = (slot ? 0 : total) + (size_t)nb * result_bytes(P.n, P.R);
    Reservation res(ctx, need);
    if (!res.take()) return fail(TK_ENOMEM, "compress needs %zu bytes; budget %zu, in use %zu", need, ctx->budget,
                                 ctx->in_use.load());
    Ws wsp;   // (unused with a batch slot: the batch owns that workspace)
    void* base = nullptr;
    if (slot) {
        base = slot->base;
    } else {
        hipError_t he = ws_get(ctx, s, 0, total, wsp);
        if (he != hipSuccess) return fail(TK_ENOMEM, "workspace of %zu bytes: %s", total, hipGetErrorString(he));
        base = wsp.p;
    }
    Arena ar;
    ar.base = (char*)base;
    Work w;
    layout_work(ar, P, own_A, w);
    w.bt.nb = nb;
    w.bt.bs = (long)ws;
    w.ctx = ctx;
    char* gather = (char*)base + ws * (size_t)nb;
    const int nmax = std::max(P.n[0], std::max(P.n[1], P.n[2]));
    const Real* A = own_A ? (const Real*)w.A : (const Real*)A_in;

    // the launches of the pipeline, from the grid evaluation to the final error (the FP64 eps
    // path reads ranks back in between)
    // kernels without a fast closed form: the radial-table route, except in a captured graph (whose
    // grid node is updated per call to the direct kernel)
    bool table_route = false;
    RadialGrid rg{};
    auto pipeline = [&](hipStream_t s) -> tk_status {
        tk_status st;
        if (own_A && !slot) {
            GridAxes ax = axes_of(grid);
            ProfScope ps(TK_PROF_GRID, s);
            if (table_route)
                TK_LAUNCH(launch_grid_eval_radial(w.A, (int)sizeof(Real), ax, kps, rg, w.rtab, s, w.bt));
            else if (sizeof(Real) == 4) TK_LAUNCH(launch_grid_eval_f32((float*)w.A, ax, kps, s, w.bt));
            else TK_LAUNCH(launch_grid_eval_f64((double*)w.A, ax, kps, s, w.bt));
        }
        if (P.init_U[0]) {
            // ---- given start factors (multigrid): no Gram; ||A||^2 for the convergence test
            for (int k = 0; k < 3; ++k)
                TK_LAUNCH(launch_copy_f64(P.init_U[k], w.U[k], (long)P.n[k] * P.R[k], s));
            TK_LAUNCH(launch_dot<Real>(A, A, (long)P.n[0] * P.n[1] * P.n[2], w.partials, 1024, w.trace, s));
        } else {
            // ---- HOSVD: Grams (one launch for the three modes when all take the large-tile
            // kernel) and leading eigenvectors
            if (gram3_eligible(P.n, P.prec, P.gsplit)) {
                ProfScope ps(TK_PROF_GRAM, s);
                TK_LAUNCH(launch_gram3(A, P.n, P.prec, w.G, (long)nmax * nmax, w.gram_work, s, w.bt, P.gsplit));
            } else {
                for (int k = 0; k < 3; ++k) {
                    ProfScope ps(TK_PROF_GRAM, s);
                    TK_LAUNCH(launch_gram(A, P.n, k, P.prec, w.G + (long)k * nmax * nmax, w.gram_work, s, w.bt,
                                          P.gsplit[k]));
                }
            }
            if ((st = eig_modes(P, w, nmax, s)) != TK_OK) return st;
        }

        if (P.eps_mode && P.prec == TK_FP64) {
            // rank rule on the Gram eigenvalues: tail(r) = trace - sum_{i<r} lambda_i
            TK_HIP(hipMemcpyAsync(w.scal, w.trace, sizeof(double), hipMemcpyDeviceToDevice, s));   // ||A||^2
            TK_LAUNCH(launch_rank_rule(w.lam, 64, P.R[0], 1, w.trace, 1, w.scal, 0, P.eps * P.eps, w.ranks + 0,
                                       w.ranks + 3, s));
            TK_LAUNCH(launch_rank_rule(w.lam + 64, 64, P.R[1], 1, w.trace + 1, 1, w.scal, 0, P.eps * P.eps, w.ranks + 1,
                                       w.ranks + 4, s));
            TK_LAUNCH(launch_rank_rule(w.lam + 128, 64, P.R[2], 1, w.trace + 2, 1, w.scal, 0, P.eps * P.eps,
                                       w.ranks + 2, w.ranks + 5, s));
            int hr[6];
            if ((st = readback(ctx, s, w.ranks, sizeof(hr), hr)) != TK_OK) return st;
            // continue with the selected ranks: the leading columns of the factors are kept
            Plan Q = P;
            for (int k = 0; k < 3; ++k) Q.R[k] = hr[k];
            for (int k = 0; k < 3; ++k) {
                if (Q.R[k] != P.R[k]) {
                    TK_HIP(hipMemcpy2DAsync(w.Urot[k], sizeof(double) * Q.R[k], w.U[k], sizeof(double) * P.R[k],
                                            sizeof(double) * Q.R[k], P.n[k], hipMemcpyDeviceToDevice, s));
                    TK_HIP(hipMemcpyAsync(w.U[k], w.Urot[k], sizeof(double) * Q.R[k] * P.n[k], hipMemcpyDeviceToDevice, s));
                }
                Q.p[k] = (P.n[k] <= EIG_PMAX) ? P.n[k] : std::min(Q.R[k] + 8, EIG_PMAX);
            }
            P = Q;
        }
        if (!w.u32_fresh)
            for (int k = 0; k < 3; ++k)
                if ((st = refresh_u32<Real>(P, w, k, s)) != TK_OK) return st;

        // ---- HOOI sweeps, then the core
        if (P.sweeps == 0) {
            if ((st = hosvd_core<Real>(P, w, A, s)) != TK_OK) return st;
        } else if (P.converge) {
            // sweeps until the core norm stops changing: | ||G|| - ||G_prev|| | <= tol ||A||, the
            // first ||G_prev|| being that of the HOSVD core (norms read back after each sweep)
            const long ncore = (long)P.R[0] * P.R[1] * P.R[2];
            double na2 = 0.0, g2 = 0.0;
            if ((st = readback(ctx, s, w.trace, sizeof(double), &na2)) != TK_OK) return st;
            if ((st = hosvd_core<Real>(P, w, A, s)) != TK_OK) return st;
            TK_LAUNCH(launch_dot<double>(w.core, w.core, ncore, w.partials, 64, w.scal + 12, s));
            if ((st = readback(ctx, s, w.scal + 12, sizeof(double), &g2)) != TK_OK) return st;
            double prev = std::sqrt(g2);
            for (int it = 0; it < P.sweeps; ++it) {
                if ((st = hooi_sweep<Real>(P, w, A, nmax, s)) != TK_OK) return st;
                TK_LAUNCH(launch_dot<double>(w.core, w.core, ncore, w.partials, 64, w.scal + 12, s));
                if ((st = readback(ctx, s, w.scal + 12, sizeof(double), &g2)) != TK_OK) return st;
                const double cur = std::sqrt(g2);
                if (std::fabs(cur - prev) <= CONVERGE_TOL * std::sqrt(na2)) break;
                prev = cur;
            }
        } else {
            for (int it = 0; it < P.sweeps; ++it)
                if ((st = hooi_sweep<Real>(P, w, A, nmax, s)) != TK_OK) return st;
        }
        // ---- reconstruction error
        if ((st = recon_norm<Real>(P, w, A, w.U, w.core, s)) != TK_OK) return st;

        const bool trunc = P.eps_mode && P.prec != TK_FP64;
        if (trunc) {
            // ranks from the core HOSVD with the (conservative) error bound, then the error of the
            // truncated result measured directly against A
            if ((st = core_truncate(P, w, s)) != TK_OK) return st;
            TK_LAUNCH(launch_mask_rank(w.Urot, P.n, P.R, w.coreA, w.ranks, s, w.bt));
            if ((st = recon_norm<Real>(P, w, A, w.Urot, w.coreA, s)) != TK_OK) return st;
            TK_LAUNCH(launch_final_err(w.scal, s, w.bt, true));
        } else {
            TK_LAUNCH(launch_final_err(w.scal, s, w.bt, true));   // no truncation: t2 = 0
        }
        return TK_OK;
    };
    tk_status st;
    const bool capturable = own_A && wsp.cached && P.prec != TK_FP64 && !P.converge && !P.init_U[0] &&
                            !g_prof_on.load();
    if (own_A && !slot && !(ctx->graphs_on && capturable)) table_route = radial_plan(axes_of(grid), kps, nb, &rg);
    if (ctx->graphs_on && capturable) {
        if ((st = run_captured<Real>(ctx, P, nb, base, grid, kps, w, s, pipeline)) != TK_OK) return st;
    } else if ((st = pipeline(s)) != TK_OK) {
        return st;
    }
    const bool trunc = P.eps_mode && P.prec != TK_FP64;
    const double* Usrc[3] = {w.U[0], w.U[1], w.U[2]};
    const double* csrc = w.core;
    if (trunc) {
        for (int k = 0; k < 3; ++k) Usrc[k] = w.Urot[k];
        csrc = w.coreA;
    }
    // ---- per problem: ranks (6 ints, padded to 8) and scal[0..3] (4 doubles)
    std::vector<int> hr((size_t)nb * 8);
    std::vector<double> hs((size_t)nb * 4);
    if (nb == 1) {
        int r6[6] = {P.R[0], P.R[1], P.R[2], 1, 1, 1};
        if (trunc) { if ((st = readback(ctx, s, w.ranks, sizeof(r6), r6, w.scal, 4 * sizeof(double), hs.data())) != TK_OK) return st; }
        else if ((st = readback(ctx, s, w.scal, 4 * sizeof(double), hs.data())) != TK_OK) return st;
        std::memcpy(hr.data(), r6, sizeof(r6));
    } else {
        int* granks = (int*)gather;
        double* gscal = (double*)(gather + (size_t)nb * 32);
        TK_LAUNCH(launch_gather_u32(w.ranks, (long)ws, 8, granks, nb, s));
        TK_LAUNCH(launch_gather_u32(w.scal, (long)ws, 8, gscal, nb, s));
        TK_HIP(hipMemcpyAsync(hr.data(), granks, (size_t)nb * 32, hipMemcpyDeviceToHost, s));
        TK_HIP(hipMemcpyAsync(hs.data(), gscal, (size_t)nb * 32, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        if (!trunc)
            for (int b = 0; b < nb; ++b)
                for (int k = 0; k < 3; ++k) hr[(size_t)b * 8 + k] = P.R[k];
    }
    auto drop_all = [&]() {
        for (int b = 0; b < nb; ++b) { free_result(outs[b]); outs[b] = nullptr; }
    };
    // all results first, then one launch copies every problem's factors and core into them
    ExtractArgs ea{};
    ea.nb = nb;
    ea.bs = (long)ws;
    ea.core_src = csrc;
    for (int k = 0; k < 3; ++k) {
        ea.n[k] = P.n[k];
        ea.ld[k] = P.R[k];
        ea.Rc[k] = P.R[k];
        ea.Usrc[k] = Usrc[k];
    }
    for (int b = 0; b < nb; ++b) {
        int final_r[3];
        for (int k = 0; k < 3; ++k) final_r[k] = hr[(size_t)b * 8 + k];
        tk_tucker* t = nullptr;
        if ((st = alloc_result(ctx, P.n, final_r, s, &t, &res)) != TK_OK) {
            drop_all();
            return st;
        }
        outs[b] = t;
        ResultDst& d = ea.dst[b];
        for (int k = 0; k < 3; ++k) {
            d.U[k] = t->U[k];
            d.U32[k] = t->U32[k];
            d.r[k] = final_r[k];
        }
        d.core = t->core;
        d.core32 = t->core32;
    }
    if (launch_extract_results(ea, s) != hipSuccess) {
        drop_all();
        return fail(TK_EHIP, "result extraction: %s", hipGetErrorString(hipGetLastError()));
    }
    for (int b = 0; b < nb; ++b) {
        tk_tucker* t = outs[b];
        for (int k = 0; k < 3; ++k) t->b[k] = grid->b[k];
        t->layout = grid->layout;
        t->prec = P.prec;
        t->rel_err = hs[(size_t)b * 4 + 3];
        t->norm_a = std::sqrt(hs[(size_t)b * 4 + 0]);
        if ((P.eps_mode && !(t->rel_err <= P.eps)) || w.noconv) sts[b] = TK_ENOCONV;
    }
    // the results are complete when the call returns, for work on any stream
    if (hipStreamSynchronize(s) != hipSuccess) {
        drop_all();
        return fail(TK_EHIP, "compress: %s", hipGetErrorString(hipGetLastError()));
    }
    if (nb == 1 && sts[0] == TK_ENOCONV)
        return fail(TK_ENOCONV, "eps=%g not reached: error %g at ranks (%d,%d,%d)", P.eps, outs[0]->rel_err,
                    outs[0]->r[0], outs[0]->r[1], outs[0]->r[2]);
    return TK_OK;
}

tk_status compress_any(tk_ctx* ctx, const tk_kernel* kernel, const void* A_in, const tk_grid* grid,
                       const tk_opts* opts, void* stream, tk_tucker** out)
{
    if (!ctx || !out) return fail(TK_EINVAL, "ctx/out is NULL");
    *out = nullptr;
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    KernelParams kp{};
    if (!A_in && (st = check_kernel(kernel, &kp)) != TK_OK) return st;
    Plan P;
    if ((st = make_plan(grid, opts, &P)) != TK_OK) return st;
    apply_tuning(ctx, &P);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(TK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    (void)hipGetLastError();   // drop errors left by earlier, unrelated HIP calls
    hipStream_t s = (hipStream_t)stream;
    tk_status one = TK_OK;
    if (P.prec == TK_FP64) return compress_impl<double>(ctx, &kp, 1, A_in, grid, P, s, out, &one);
    return compress_impl<float>(ctx, &kp, 1, A_in, grid, P, s, out, &one);
}

// nb <= BATCH_MAX problems on one grid with one set of options, launched together.  outs[i] /
// sts[i] as for compress_impl.
tk_status compress_group(tk_ctx* ctx, const tk_kernel* const* kernels, int nb, const tk_grid* grid,
                         const tk_opts* opts, hipStream_t s, tk_tucker** outs, tk_status* sts,
                         const BatchSlot* slot = nullptr)
{
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    KernelParams kps[BATCH_MAX];
    if (nb < 1 || nb > BATCH_MAX) return fail(TK_EINVAL, "batch of %d problems", nb);
    for (int b = 0; b < nb; ++b)
        if ((st = check_kernel(kernels[b], &kps[b])) != TK_OK) return st;
    Plan P;
    if ((st = make_plan(grid, opts, &P)) != TK_OK) return st;
    apply_tuning(ctx, &P);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(TK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    (void)hipGetLastError();
    if (P.prec == TK_FP64) return compress_impl<double>(ctx, kps, nb, nullptr, grid, P, s, outs, sts);
    return compress_impl<float>(ctx, kps, nb, nullptr, grid, P, s, outs, sts, slot);
}

// Can problems with these options share launches?  (The FP64 path reads the eigensolver's
// convergence flags -- and in eps mode the ranks -- back between steps, and converged HOOI the
// core norm, so their problems run one per call.)
bool groupable(const tk_opts* o) { return o->prec != TK_FP64 && o->hooi_sweeps != TK_HOOI_CONVERGE; }

bool cov_geometry(const tk_tucker* t, int off[3], int m[3])
{
    for (int k = 0; k < 3; ++k) {
        if (t->layout == TK_OFFSET) { off[k] = 0; m[k] = t->n[k]; }
        else if (t->n[k] % 2 == 1) { off[k] = (t->n[k] - 1) / 2; m[k] = (t->n[k] + 1) / 2; }
        else return false;
    }
    return true;
}

size_t matvec_work_bytes(const tk_tucker* t, int esz)
{
    int off[3], m[3];
    cov_geometry(t, off, m);
    size_t M3 = (size_t)m[0] * m[1] * m[2];
    Arena ar;
    ar.take<char>((size_t)t->r[0] * t->r[1] * t->n[2] * esz);    // W generators
    ar.take<char>((size_t)t->r[0] * M3 * esz);                   // Z1
    ar.take<char>((size_t)t->r[1] * M3 * esz);                   // P
    ar.take<double>(2048);                                       // dot partials + result
    return ar.off;
}

template <typename T>
tk_status matvec_impl(tk_ctx* ctx, const tk_tucker* t, const T* z, T* y, hipStream_t s, double* dot_out)
{
    int off[3], m[3];
    if (!cov_geometry(t, off, m)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    const int r0 = t->r[0], r1 = t->r[1], r2 = t->r[2];
    const long M3 = (long)m[0] * m[1] * m[2];
    size_t need = matvec_work_bytes(t, sizeof(T));
    Reservation res(ctx, need);
    if (!res.take()) return fail(TK_ENOMEM, "matvec needs %zu bytes; budget %zu, in use %zu", need, ctx->budget,
                                 ctx->in_use.load());
    Ws wsp;
    hipError_t he = ws_get(ctx, s, 0, need, wsp);
    if (he != hipSuccess) return fail(TK_ENOMEM, "workspace of %zu bytes: %s", need, hipGetErrorString(he));
    void* base = wsp.p;
    Arena ar;
    ar.base = (char*)base;
    T* W = ar.take<T>((size_t)r0 * r1 * t->n[2]);
    T* Z1 = ar.take<T>((size_t)r0 * M3);
    T* Pb = ar.take<T>((size_t)r1 * M3);
    double* dots = ar.take<double>(2048);
    const T* U0 = sizeof(T) == 4 ? (const T*)t->U32[0] : (const T*)t->U[0];
    const T* U1 = sizeof(T) == 4 ? (const T*)t->U32[1] : (const T*)t->U[1];
    const T* U2 = sizeof(T) == 4 ? (const T*)t->U32[2] : (const T*)t->U[2];
    const T* core = sizeof(T) == 4 ? (const T*)t->core32 : (const T*)t->core;
    // W[a][b][i] = sum_c core[a][b][c] U3[i][c]  (generators of the mode-3 Toeplitz factors)
    {
        GemmArgs g = gemm(r0 * r1, t->n[2], r2, 1, core, 0, r2, 1, U2, 0, 1, r2, W, 0, t->n[2], 1);
        TK_LAUNCH((launch_gemm<T, T, T>(g, s)));
    }
    // Z1[a] = T(U1[:, a]) along mode 1
    {
        ToepLeftArgs a{};
        a.M = m[0]; a.N = (int)((long)m[1] * m[2]); a.K = m[0]; a.nb = 1;
        a.gen = U0; a.gs_idx = r0; a.gs_col = 1; a.gstride_g = 1; a.gstride_b = 0;
        a.glen = t->n[0]; a.glen_pad = (t->n[0] + 1) & ~1; a.off = off[0];
        a.In = z; a.sIs = 0; a.sIg = 0; a.sIb = 0; a.sIi = (long)m[1] * m[2];
        a.Out = Z1; a.sOs = 0; a.sOg = M3; a.sOi = (long)m[1] * m[2];
        a.accumulate = 0;
        ProfScope ps(TK_PROF_TOEP_LEFT, s);
        TK_LAUNCH(launch_toep_left<T>(a, 1, r0, s));
    }
    for (int a0 = 0; a0 < r0; ++a0) {
        // P[(i0, i1)][b][i2'] = sum_i2 Z1[a][i0][i1][i2] T(w_ab)[i2][i2']
        ToepRightArgs rr{};
        rr.R = (long)m[0] * m[1]; rr.K = m[2]; rr.m = m[2]; rr.nb = r1;
        rr.gen = W + (long)a0 * r1 * t->n[2]; rr.gs_idx = 1; rr.gs_col = t->n[2]; rr.glen = t->n[2]; rr.off = off[2];
        rr.In = Z1 + (long)a0 * M3; rr.ldi = m[2];
        rr.Out = Pb; rr.ldo = (long)r1 * m[2];
        {
            ProfScope ps(TK_PROF_TOEP_RIGHT, s);
            TK_LAUNCH(launch_toep_right<T>(rr, s));
        }
        // y[i0][i1'][:] (+)= sum_b sum_i1 T(U2[:, b])[i1'][i1] P[i0][i1][b][:]
        ToepLeftArgs l{};
        l.M = m[1]; l.N = m[2]; l.K = m[1]; l.nb = r1;
        l.gen = U1; l.gs_idx = r1; l.gs_col = 1; l.gstride_g = 0; l.gstride_b = 1;
        l.glen = t->n[1]; l.glen_pad = (t->n[1] + 1) & ~1; l.off = off[1];
        l.In = Pb; l.sIs = (long)m[1] * r1 * m[2]; l.sIg = 0; l.sIb = m[2]; l.sIi = (long)r1 * m[2];
        l.Out = y; l.sOs = (long)m[1] * m[2]; l.sOg = 0; l.sOi = m[2];
        l.accumulate = a0 > 0;
        ProfScope ps(TK_PROF_TOEP_LEFT, s);
        TK_LAUNCH(launch_toep_left<T>(l, m[0], 1, s));
    }
    if (dot_out) {
        TK_LAUNCH(launch_dot<T>(z, y, M3, dots, 1024, dots + 1024, s));
        tk_status rs = readback(ctx, s, dots + 1024, sizeof(double), dot_out);
        if (rs != TK_OK) return rs;
    }
    return TK_OK;
}

int next_pow2(int x)
{
    int L = 1;
    while (L < x) L <<= 1;
    return L;
}

int ilog2(int L)
{
    int l = 0;
    while ((1 << l) < L) ++l;
    return l;
}

// y = C z by the 3-D DFT (see k_fft.hip); FP32 data.  A matvec is a preamble (the Fourier-side
// factors and the core contracted with two of them, small kernels) and five passes over the
// data; a batch of quadratic forms runs its preambles on a side stream and the passes of all
// items back to back.
struct MvGeom {
    int off[3], m[3], L[3], lg[3], r[3];
    int H2, H2p, r2p;
};

bool mv_geom(const tk_tucker* t, MvGeom* g)
{
    if (!cov_geometry(t, g->off, g->m)) return false;
    for (int k = 0; k < 3; ++k) {
        g->L[k] = next_pow2(std::max(2 * g->m[k] - 1, 2));
        g->lg[k] = ilog2(g->L[k]);
        g->r[k] = t->r[k];
    }
    g->H2 = g->L[2] / 2 + 1;
    g->H2p = (g->H2 + 15) & ~15;     // row pitch of the half spectra: whole 128-byte lines per 16 fibres
    g->r2p = (g->r[2] + 3) & ~3;
    return true;
}

// per-item buffers: twiddles, Fourier-side factors, Hs[f1][f0][c], Uh3[f2][c], dot partials
struct MvPre {
    float2* tw[3];
    double *Uh0, *Uh1, *Uh2, *M1, *dots;
    float *Hs, *Uh3;
};
void lay_pre(Arena& ar, const MvGeom& g, MvPre* b)
{
    for (int k = 0; k < 3; ++k) b->tw[k] = ar.take<float2>((size_t)g.L[k]);
    b->Uh0 = ar.take<double>((size_t)g.L[0] * g.r[0]);
    b->Uh1 = ar.take<double>((size_t)g.L[1] * g.r[1]);
    b->Uh2 = ar.take<double>((size_t)g.H2 * g.r[2]);
    b->M1 = ar.take<double>((size_t)g.L[0] * g.r[1] * g.r[2]);
    b->Hs = ar.take<float>((size_t)g.L[0] * g.L[1] * g.r2p);
    b->Uh3 = ar.take<float>((size_t)g.H2 * g.r2p);
    b->dots = ar.take<double>(2048);
}
// the half spectra between the passes (shared by the items of a batch, which run in turn)
size_t mv_a1_elems(const MvGeom& g) { return (size_t)g.m[0] * g.m[1] * g.H2p; }
size_t mv_a2_elems(const MvGeom& g) { return (size_t)g.m[0] * g.L[1] * g.H2p; }

tk_status mv_preamble(const tk_tucker* t, const MvGeom& g, const MvPre& b, hipStream_t s)
{
    ProfScope ps(TK_PROF_SMALL, s);
    for (int k = 0; k < 3; ++k) TK_LAUNCH(launch_twiddles(b.tw[k], g.L[k], s));
    // Fourier-side factors and Hs[f1][f0][c] = sum_ab G_abc Uh1[f0][a] Uh2[f1][b] (c padded to r2p)
    const int r0 = g.r[0], r1 = g.r[1], r2 = g.r[2];
    FourierAxes fa;
    fa.ax[0] = FourierAxis{t->U[0], r0, g.off[0], g.m[0], g.L[0], g.L[0], b.Uh0};
    fa.ax[1] = FourierAxis{t->U[1], r1, g.off[1], g.m[1], g.L[1], g.L[1], b.Uh1};
    fa.ax[2] = FourierAxis{t->U[2], r2, g.off[2], g.m[2], g.L[2], g.H2, b.Uh2};
    TK_LAUNCH(launch_fourier_factors(fa, s));
    GemmArgs gm = gemm(g.L[0], r1 * r2, r0, 1, b.Uh0, 0, r0, 1, t->core, 0, (long)r1 * r2, 1, b.M1, 0, (long)r1 * r2, 1);
    TK_LAUNCH((launch_gemm<double, double, double>(gm, s)));
    TK_LAUNCH(launch_spectral_core(b.Uh1, b.M1, g.L[0], g.L[1], r1, r2, g.r2p, b.Hs, s));
    TK_LAUNCH(launch_f64_to_f32_padded(b.Uh2, g.H2, r2, g.r2p, b.Uh3, s));
    return TK_OK;
}

// The five passes.  dot_dst (device, optional): z . y, summed by the last pass (y_out may then
// be NULL: y is not stored).
tk_status mv_passes(const MvGeom& g, const MvPre& b, float2* A1, float2* A2, const float* z, float* y,
                    double* dot_dst, hipStream_t s)
{
    const int* m = g.m;
    const int* L = g.L;
    const int* lg = g.lg;
    const int H2 = g.H2, H2p = g.H2p;
    FftPassArgs a{};
    {
        ProfScope ps(TK_PROF_FFT, s);
        // P1: axis 2 forward, real rows of m2 -> H2 complex
        a = FftPassArgs{};
        a.L = L[2]; a.logL = lg[2];
        a.n_inner = m[0] * m[1]; a.len_in = m[2]; a.len_out = H2;
        a.s_in_o = 0; a.s_in_i = m[2]; a.s_in_k = 1; a.s_out_o = 0; a.s_out_i = H2p; a.s_out_k = 1;
        a.in = z; a.out = A1; a.in_real = 1; a.out_real = 0; a.mode = 0; a.scale = 1.f; a.tw = b.tw[2];
        TK_LAUNCH(launch_fft_pass(a, 1, s));
        // P2: axis 1 forward, fibres (i0, f2) over i1
        a = FftPassArgs{};
        a.L = L[1]; a.logL = lg[1];
        a.n_inner = H2; a.len_in = m[1]; a.len_out = L[1];
        a.s_in_o = (long)m[1] * H2p; a.s_in_i = 1; a.s_in_k = H2p;
        a.s_out_o = (long)L[1] * H2p; a.s_out_i = 1; a.s_out_k = H2p;
        a.in = A1; a.out = A2; a.mode = 0; a.scale = 1.f; a.tw = b.tw[1];
        TK_LAUNCH(launch_fft_pass(a, m[0], s));
    }
    {
        ProfScope ps(TK_PROF_FFT_AXIS0, s);
        // P3: axis 0 forward, times chat, inverse; fibres (f1, f2) over i0, in place
        a = FftPassArgs{};
        a.L = L[0]; a.logL = lg[0];
        a.n_inner = H2; a.len_in = m[0]; a.len_out = m[0];
        a.s_in_o = H2p; a.s_in_i = 1; a.s_in_k = (long)L[1] * H2p;
        a.s_out_o = H2p; a.s_out_i = 1; a.s_out_k = (long)L[1] * H2p;
        a.in = A2; a.out = A2; a.mode = 3; a.scale = 1.f;
        a.Hs = b.Hs; a.Uh3 = b.Uh3; a.r2p = g.r2p; a.tw = b.tw[0];
        TK_LAUNCH(launch_fft_pass(a, L[1], s));
    }
    {
        ProfScope ps(TK_PROF_FFT, s);
        // P4: axis 1 inverse, keep i1 < m1
        a = FftPassArgs{};
        a.L = L[1]; a.logL = lg[1];
        a.n_inner = H2; a.len_in = L[1]; a.len_out = m[1];
        a.s_in_o = (long)L[1] * H2p; a.s_in_i = 1; a.s_in_k = H2p;
        a.s_out_o = (long)m[1] * H2p; a.s_out_i = 1; a.s_out_k = H2p;
        a.in = A2; a.out = A1; a.mode = 1; a.scale = 1.f; a.tw = b.tw[1];
        TK_LAUNCH(launch_fft_pass(a, m[0], s));
        // P5: axis 2 inverse from the half spectrum, real part, keep i2 < m2, scale
        a = FftPassArgs{};
        a.L = L[2]; a.logL = lg[2];
        a.n_inner = m[0] * m[1]; a.len_in = H2; a.len_out = m[2];
        a.s_in_o = 0; a.s_in_i = H2p; a.s_in_k = 1; a.s_out_o = 0; a.s_out_i = m[2]; a.s_out_k = 1;
        a.in = A1; a.out = y; a.no_store = y ? 0 : 1; a.out_real = 1; a.mode = 2; a.tw = b.tw[2];
        a.scale = (float)(1.0 / ((double)L[0] * L[1] * L[2]));
        if (dot_dst) {
            // z . y summed while y is formed: one FP64 partial per work-group, then added in order
            a.dot_z = z; a.dot_part = b.dots; a.dot_cap = 1024;
        }
        unsigned blocks = 0;
        TK_LAUNCH(launch_fft_pass(a, 1, s, &blocks));
        if (dot_dst) TK_LAUNCH(launch_reduce_partials(b.dots, (int)blocks, 1, dot_dst, s));
    }
    return TK_OK;
}

// The workspace of one matvec: per-item buffers, then the two half spectra.
void mv_lay(Arena& ar, const MvGeom& g, MvPre* b, float2** A1, float2** A2)
{
    lay_pre(ar, g, b);
    *A1 = ar.take<float2>(mv_a1_elems(g));
    *A2 = ar.take<float2>(mv_a2_elems(g));
}

// One matvec (y != NULL) or quadratic form (dot_out != NULL; y may then be NULL).
// plan_bytes != nullptr: only report the workspace the call needs (nothing runs).
tk_status matvec_fft(tk_ctx* ctx, const tk_tucker* t, const float* z, float* y, hipStream_t s, double* dot_out,
                     size_t* plan_bytes = nullptr)
{
    MvGeom g;
    if (!mv_geom(t, &g)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    auto lay = [&](Arena& ar, MvPre* b, float2** A1, float2** A2) { mv_lay(ar, g, b, A1, A2); };
    Arena plan;
    MvPre b;
    float2 *A1, *A2;
    lay(plan, &b, &A1, &A2);
    if (plan_bytes) {
        *plan_bytes = plan.off;
        return TK_OK;
    }
    Reservation res(ctx, plan.off);
    if (!res.take()) return fail(TK_ENOMEM, "matvec needs %zu bytes; budget %zu, in use %zu", plan.off, ctx->budget,
                                 ctx->in_use.load());
    Ws wsp;
    hipError_t he = ws_get(ctx, s, 0, plan.off, wsp);
    if (he != hipSuccess) return fail(TK_ENOMEM, "workspace of %zu bytes: %s", plan.off, hipGetErrorString(he));
    Arena ar;
    ar.base = (char*)wsp.p;
    lay(ar, &b, &A1, &A2);
    tk_status st;
    if ((st = mv_preamble(t, g, b, s)) != TK_OK) return st;
    if ((st = mv_passes(g, b, A1, A2, z, y, dot_out ? b.dots + 1024 : nullptr, s)) != TK_OK) return st;
    if (dot_out) {
        tk_status rs = readback(ctx, s, b.dots + 1024, sizeof(double), dot_out);
        if (rs != TK_OK) return rs;
    }
    return TK_OK;
}

// Quadratic forms of `count` results on the FFT path: the preambles on a side stream (each
// followed by an event), the passes of the items in turn on s, sharing one pair of spectrum
// buffers, the values gathered and read back once.  Same kernels and launch shapes as
// matvec_fft, so each value is bitwise the single call's.
tk_status quadform_fft_batch(tk_ctx* ctx, int count, const tk_tucker* const* ts, const void* const* z_devs,
                             void* const* y_devs, hipStream_t s, hipStream_t side, double* out)
{
    std::vector<MvGeom> g(count);
    size_t a1 = 0, a2 = 0;
    for (int i = 0; i < count; ++i) {
        if (!mv_geom(ts[i], &g[i])) return fail(TK_ELAYOUT, "item %d: even-sized centred grid has no origin node", i);
        a1 = std::max(a1, mv_a1_elems(g[i]));
        a2 = std::max(a2, mv_a2_elems(g[i]));
    }
    std::vector<MvPre> b(count);
    float2 *A1, *A2;
    double* gather;
    auto lay = [&](Arena& ar) {
        for (int i = 0; i < count; ++i) lay_pre(ar, g[i], &b[i]);
        A1 = ar.take<float2>(a1);
        A2 = ar.take<float2>(a2);
        gather = ar.take<double>((size_t)count);
    };
    Arena plan;
    lay(plan);
    Reservation res(ctx, plan.off);
    if (!res.take()) return fail(TK_ENOMEM, "quadratic forms need %zu bytes; budget %zu, in use %zu", plan.off,
                                 ctx->budget, ctx->in_use.load());
    Ws wsp;
    hipError_t he = ws_get(ctx, s, 0, plan.off, wsp);
    if (he != hipSuccess) return fail(TK_ENOMEM, "workspace of %zu bytes: %s", plan.off, hipGetErrorString(he));
    Arena ar;
    ar.base = (char*)wsp.p;
    lay(ar);
    std::vector<hipEvent_t> ev(count + 1, nullptr);
    tk_status st = TK_OK;
    auto run = [&]() -> tk_status {
        for (auto& e : ev) TK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // the preambles start after the work queued on s
        TK_HIP(hipEventRecord(ev[count], s));
        TK_HIP(hipStreamWaitEvent(side, ev[count], 0));
        tk_status r;
        for (int i = 0; i < count; ++i) {
            if ((r = mv_preamble(ts[i], g[i], b[i], side)) != TK_OK) return r;
            TK_HIP(hipEventRecord(ev[i], side));
        }
        for (int i = 0; i < count; ++i) {
            TK_HIP(hipStreamWaitEvent(s, ev[i], 0));
            if ((r = mv_passes(g[i], b[i], A1, A2, (const float*)z_devs[i], y_devs ? (float*)y_devs[i] : nullptr,
                               gather + i, s)) != TK_OK)
                return r;
        }
        return readback(ctx, s, gather, sizeof(double) * count, out);
    };
    st = run();
    if (st != TK_OK) (void)hipStreamSynchronize(side);   // no preamble left running on the workspace
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

// The FFT form keeps the third factor's columns (padded to a multiple of 4) in one register
// tile of at most LIB_RMAX; results of a higher third rank (FP64 compressions up to EIG_PMAX,
// loaded files) take the dense form, which has no rank limit.
bool use_fft(const tk_ctx* ctx, const tk_tucker* t, int io)
{
    return io == TK_FP32 && ctx->matvec_method != TK_MV_DENSE && ((t->r[2] + 3) & ~3) <= LIB_RMAX;
}

}  // namespace

// ==========================================================================================
// C ABI
// ==========================================================================================
extern "C" {

const char* tk_version(void) { return "tk-mi355x 0.1 (gfx950)"; }

tk_status tk_profile_enable(int on)
{
    g_prof_on.store(on != 0);
    return TK_OK;
}

tk_status tk_profile_select(unsigned mask)
{
    g_prof_mask.store(mask);
    return TK_OK;
}

tk_status tk_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventSynchronize(r.b);
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof.clear();
    return TK_OK;
}

tk_status tk_profile_read(int cls, long long* launches, double* total_ms)
{
    if (cls < 0 || cls >= TK_PROF_COUNT || !launches || !total_ms) return fail(TK_EINVAL, "bad profile query");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    long long n = 0;
    double ms = 0.0;
    for (auto& r : g_prof) {
        if (r.cls != cls) continue;
        TK_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        TK_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return TK_OK;
}

const char* tk_last_error(void) { return g_last_error.c_str(); }

const char* tk_strerror(tk_status s)
{
    switch (s) {
    case TK_OK: return "TK_OK";
    case TK_EINVAL: return "TK_EINVAL";
    case TK_EUNSUPPORTED: return "TK_EUNSUPPORTED";
    case TK_ELAYOUT: return "TK_ELAYOUT";
    case TK_ENOMEM: return "TK_ENOMEM";
    case TK_EHIP: return "TK_EHIP";
    case TK_ENOCONV: return "TK_ENOCONV";
    }
    return "TK_UNKNOWN";
}

tk_status tk_ctx_create(int device, size_t hbm_budget_bytes, tk_ctx** out)
{
    if (!out) return fail(TK_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return fail(TK_EHIP, "no HIP device");
    if (device < 0 || device >= count) return fail(TK_EINVAL, "device %d out of range (%d devices)", device, count);
    TK_HIP(hipSetDevice(device));
    size_t freeb = 0, total = 0;
    TK_HIP(hipMemGetInfo(&freeb, &total));
    hipMemPool_t pool;
    TK_HIP(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t thr = UINT64_MAX;
    TK_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
    // memory freed on one stream goes to another only once the free has completed: reuse that
    // follows event dependencies would make a worker's next allocation wait for the kernels
    // another worker still runs on memory it has just released
    int off = 0;
    TK_HIP(hipMemPoolSetAttribute(pool, hipMemPoolReuseFollowEventDependencies, &off));
    TK_HIP(hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowOpportunistic, &off));
    TK_HIP(hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &off));
    TK_HIP(eig_set_attributes());
    TK_HIP(kron_set_attributes());
    TK_HIP(fft_set_attributes());
    void* scr = nullptr;
    TK_HIP(scratch_address(device, &scr));
    tk_ctx* c = new (std::nothrow) tk_ctx();
    if (!c) return fail(TK_ENOMEM, "host allocation failed");
    c->device = device;
    c->scratch = scr;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)freeb);
    const size_t slot_bytes = (size_t)tk_ctx::kSlots * tk_ctx::kSlotBytes;
    if (hipHostMalloc((void**)&c->pinned, slot_bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->dev_slots, slot_bytes) != hipSuccess) {
        if (c->pinned) (void)hipHostFree(c->pinned);
        delete c;
        return fail(TK_ENOMEM, "staging buffers (%zu bytes)", slot_bytes);
    }
    *out = c;
    return TK_OK;
}

void tk_ctx_destroy(tk_ctx* ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->dev_slots) (void)hipFree(ctx->dev_slots);
    ctx->pinned = nullptr;
    ctx->dev_slots = nullptr;
    {
        std::lock_guard<std::mutex> g(ctx->graph_mu);
        for (auto& kv : ctx->graphs) {
            (void)hipGraphExecDestroy(kv.second.ex);
            (void)hipGraphDestroy(kv.second.g);
        }
        ctx->graphs.clear();
    }
    {
        std::lock_guard<std::mutex> g(ctx->ws_mu);
        for (auto& kv : ctx->ws)
            if (kv.second.ptr) (void)hipFreeAsync(kv.second.ptr, nullptr);
        ctx->ws.clear();
    }
    hipDeviceSynchronize();
    for (hipStream_t st : ctx->streams) (void)hipStreamDestroy(st);
    ctx->streams.clear();
    bool now = false;
    {
        std::lock_guard<std::mutex> g(ctx->life_mu);
        ctx->closing = true;
        std::lock_guard<std::mutex> g2(ctx->rc_mu);
        for (auto& kv : ctx->rcache) (void)hipFree(kv.second);
        ctx->rcache.clear();
        ctx->rcache_bytes = 0;
        ctx->idle.store(0);
        now = (ctx->live_results == 0);
    }
    if (now) delete ctx;
}

tk_status tk_autotune(tk_ctx* ctx, const tk_grid* grid, int prec, void* hip_stream, int nsplit_out[3],
                      double ms_out[3])
{
    if (!ctx || !grid) return fail(TK_EINVAL, "NULL argument");
    if (prec < TK_FP64 || prec > TK_BF16X3) return fail(TK_EINVAL, "unknown precision %d", prec);
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    const int* n = grid->n;
    const size_t N = (size_t)n[0] * n[1] * n[2];
    const size_t esz = prec == TK_FP64 ? 8 : 4;
    const int nmax = std::max(n[0], std::max(n[1], n[2]));
    size_t wb = 0;
    for (int k = 0; k < 3; ++k) wb = std::max(wb, gram_work_bytes(n, k, prec));   // the largest candidate
    const size_t need = align_up(N * esz, 256) + align_up(sizeof(double) * nmax * nmax, 256) + wb;
    Reservation res(ctx, need);
    if (!res.take()) return fail(TK_ENOMEM, "autotune needs %zu bytes", need);
    Ws wsp;
    TK_HIP(ws_get(ctx, s, 0, need, wsp));
    char* base = (char*)wsp.p;
    void* A = base;
    double* G = (double*)(base + align_up(N * esz, 256));
    void* work = base + align_up(N * esz, 256) + align_up(sizeof(double) * nmax * nmax, 256);
    // a Matern 3/2 covariance on the grid (the timing does not depend on the values)
    tk_kernel kk{};
    kk.family = TK_MATERN; kk.nu = 1.5; kk.ell = 0.3; kk.sigma2 = 1.0; kk.alpha = 1.0; kk.p = 1.0;
    KernelParams kp{};
    if ((st = check_kernel(&kk, &kp)) != TK_OK) return st;
    GridAxes ax = axes_of(grid);
    if (esz == 4) TK_LAUNCH(launch_grid_eval_f32((float*)A, ax, &kp, s));
    else TK_LAUNCH(launch_grid_eval_f64((double*)A, ax, &kp, s));
    hipEvent_t e0, e1;
    TK_HIP(hipEventCreate(&e0));
    TK_HIP(hipEventCreate(&e1));
    for (int k = 0; k < 3; ++k) {
        int cand[GRAM_MAX_CANDIDATES];
        const int nc = gram_split_candidates(n, k, prec, cand);
        int best = cand[0];
        float best_ms = 1e30f;
        for (int c = 0; c < nc; ++c) {
            TK_LAUNCH(launch_gram(A, n, k, prec, G, work, s, Bat(), cand[c]));   // warm-up
            TK_HIP(hipEventRecord(e0, s));
            for (int rep = 0; rep < 5; ++rep) TK_LAUNCH(launch_gram(A, n, k, prec, G, work, s, Bat(), cand[c]));
            TK_HIP(hipEventRecord(e1, s));
            TK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            TK_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= 5.f;
            if (ms < best_ms) { best_ms = ms; best = cand[c]; }
        }
        {
            std::lock_guard<std::mutex> g(ctx->tune_mu);
            ctx->tune[{n[0], n[1], n[2], k, prec}] = best;
        }
        if (nsplit_out) nsplit_out[k] = best;
        if (ms_out) ms_out[k] = best_ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return TK_OK;
}

tk_status tk_autotune_save(tk_ctx* ctx, const char* path)
{
    if (!ctx || !path) return fail(TK_EINVAL, "NULL argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(TK_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    std::fprintf(f, "{\"format\": \"tk-autotune-1\", \"entries\": [");
    bool first = true;
    for (const auto& kv : ctx->tune) {
        std::fprintf(f, "%s\n  {\"n\": [%d, %d, %d], \"mode\": %d, \"prec\": %d, \"nsplit\": %d}", first ? "" : ",",
                     kv.first[0], kv.first[1], kv.first[2], kv.first[3], kv.first[4], kv.second);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? TK_OK : fail(TK_EINVAL, "cannot write %s", path);
}

tk_status tk_autotune_load(tk_ctx* ctx, const char* path)
{
    if (!ctx || !path) return fail(TK_EINVAL, "NULL argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(TK_EINVAL, "cannot read %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    if (text.find("\"tk-autotune-1\"") == std::string::npos) return fail(TK_EINVAL, "%s is not an autotune file", path);
    std::map<std::array<int, 5>, int> add;
    size_t pos = 0;
    while ((pos = text.find("{\"n\":", pos)) != std::string::npos) {
        int a, b, c, mode, prec, ns;
        const size_t end = text.find('}', pos);
        if (end == std::string::npos) break;
        const std::string obj = text.substr(pos, end - pos + 1);
        if (std::sscanf(obj.c_str(), "{\"n\": [%d, %d, %d], \"mode\": %d, \"prec\": %d, \"nsplit\": %d}", &a, &b, &c,
                        &mode, &prec, &ns) != 6 ||
            a < 1 || b < 1 || c < 1 || mode < 0 || mode > 2 || prec < TK_FP64 || prec > TK_BF16X3 || ns < 1)
            return fail(TK_EINVAL, "%s: bad entry %s", path, obj.c_str());
        add[{a, b, c, mode, prec}] = ns;
        pos = end;
    }
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    for (const auto& kv : add) ctx->tune[kv.first] = kv.second;
    return TK_OK;
}

tk_status tk_ctx_release_stream(tk_ctx* ctx, void* hip_stream)
{
    if (!ctx) return fail(TK_EINVAL, "ctx is NULL");
    TK_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> g(ctx->ws_mu);
    for (int slot = 0; slot < 2; ++slot) {
        auto it = ctx->ws.find({s, slot});
        if (it == ctx->ws.end()) continue;
        if (it->second.busy) return fail(TK_EINVAL, "a call on this stream is still running");
        if (it->second.ptr) (void)hipFreeAsync(it->second.ptr, s);
        ctx->idle.fetch_sub(it->second.bytes);
        ctx->ws.erase(it);
    }
    return TK_OK;
}

tk_status tk_ctx_set_graphs(tk_ctx* ctx, int on)
{
    if (!ctx) return fail(TK_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> g(ctx->graph_mu);
    ctx->graphs_on = on != 0;
    return TK_OK;
}

tk_status tk_ctx_set_cholqr(tk_ctx* ctx, double floor, double one_pass, double accept2)
{
    if (!ctx || !(floor == floor) || !(one_pass == one_pass) || !(accept2 == accept2))
        return fail(TK_EINVAL, "ctx is NULL or a threshold is NaN");
    std::lock_guard<std::mutex> g(ctx->graph_mu);
    ctx->cholqr = CholQr{floor > 0.0 ? floor : 0.0, one_pass, accept2};
    // captured pipelines hold the old threshold in their launches
    for (auto& kv : ctx->graphs) {
        (void)hipGraphExecDestroy(kv.second.ex);
        (void)hipGraphDestroy(kv.second.g);
    }
    ctx->graphs.clear();
    return TK_OK;
}

tk_status tk_ctx_set_workers(tk_ctx* ctx, int workers)
{
    if (!ctx || workers < 1 || workers > 16) return fail(TK_EINVAL, "workers must be in 1..16");
    ctx->workers = workers;
    return TK_OK;
}

tk_status tk_set_matvec_method(tk_ctx* ctx, int method)
{
    if (!ctx || method < TK_MV_AUTO || method > TK_MV_DENSE) return fail(TK_EINVAL, "bad matvec method");
    ctx->matvec_method = method;
    return TK_OK;
}

tk_status tk_ctx_budget(const tk_ctx* ctx, size_t* budget_bytes, size_t* in_use_bytes)
{
    if (!ctx) return fail(TK_EINVAL, "ctx is NULL");
    if (budget_bytes) *budget_bytes = ctx->budget;
    if (in_use_bytes) *in_use_bytes = ctx->in_use.load();
    return TK_OK;
}

tk_status tk_estimate_bytes(const tk_grid* grid, const tk_opts* opts, size_t* peak_bytes)
{
    if (!peak_bytes) return fail(TK_EINVAL, "peak_bytes is NULL");
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    Plan P;
    if ((st = make_plan(grid, opts, &P)) != TK_OK) return st;
    *peak_bytes = estimate(P, true);
    return TK_OK;
}

tk_status tk_compress(tk_ctx* ctx, const tk_kernel* kernel, const tk_grid* grid, const tk_opts* opts,
                      void* hip_stream, tk_tucker** out)
{
    if (!kernel) return fail(TK_EINVAL, "kernel is NULL");
    return compress_any(ctx, kernel, nullptr, grid, opts, hip_stream, out);
}

tk_status tk_compress_tensor(tk_ctx* ctx, const void* A_dev, const tk_grid* grid, const tk_opts* opts,
                             void* hip_stream, tk_tucker** out)
{
    if (!A_dev) return fail(TK_EINVAL, "A_dev is NULL");
    return compress_any(ctx, nullptr, A_dev, grid, opts, hip_stream, out);
}

tk_status tk_compress_multigrid(tk_ctx* ctx, const tk_kernel* kernel, const tk_grid* grid, int levels,
                                const tk_opts* opts, void* hip_stream, tk_tucker** out)
{
    if (!ctx || !kernel || !grid || !opts || !out) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    KernelParams kp{};
    if ((st = check_kernel(kernel, &kp)) != TK_OK) return st;
    if (levels < 0 || levels > 8) return fail(TK_EINVAL, "levels=%d: 0..8", levels);
    // points per axis per level, coarsest first: each coarser level keeps (n + 1) / 2 points
    std::vector<std::array<int, 3>> sz((size_t)levels + 1);
    for (int k = 0; k < 3; ++k) {
        int n = grid->n[k];
        for (int l = levels; l >= 0; --l) {
            sz[(size_t)l][k] = n;
            n = (n + 1) / 2;
        }
        if (sz[0][k] < 2) return fail(TK_EINVAL, "axis %d: %d levels leave fewer than 2 points", k, levels);
    }
    Plan Pchk;
    if ((st = make_plan(grid, opts, &Pchk)) != TK_OK) return st;
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    // coarsest level: the plain compression (HOSVD, its ALS sweeps, eps rule or fixed ranks)
    tk_grid g0 = *grid;
    for (int k = 0; k < 3; ++k) g0.n[k] = sz[0][k];
    tk_opts o0 = *opts;
    if (o0.hooi_sweeps == TK_HOOI_CONVERGE && Pchk.prec != TK_FP64) o0.hooi_sweeps = -1;
    tk_tucker* t = nullptr;
    st = compress_any(ctx, kernel, nullptr, &g0, &o0, s, &t);
    if (st != TK_OK && st != TK_ENOCONV) return st;
    for (int l = 1; l <= levels; ++l) {
        tk_grid gl = *grid;
        for (int k = 0; k < 3; ++k) gl.n[k] = sz[(size_t)l][k];
        tk_grid gp = *grid;
        for (int k = 0; k < 3; ++k) gp.n[k] = sz[(size_t)l - 1][k];
        const GridAxes ac = axes_of(&gp), af = axes_of(&gl);
        // fixed ranks from the coarsest level, the sweeps of the options (at least one)
        tk_opts ol = *opts;
        ol.eps = 0.0;
        for (int k = 0; k < 3; ++k) ol.ranks[k] = t->r[k];
        if (ol.hooi_sweeps == 0) ol.hooi_sweeps = 1;
        Plan P;
        if ((st = make_plan(&gl, &ol, &P)) != TK_OK) { free_result(t); return st; }
        // interpolated, orthonormalised start factors in the stream's second workspace slot
        size_t ib = 0;
        for (int k = 0; k < 3; ++k) ib += align_up(sizeof(double) * (size_t)gl.n[k] * P.R[k], 256);
        Reservation res(ctx, ib);
        if (!res.take()) { free_result(t); return fail(TK_ENOMEM, "multigrid start factors (%zu bytes)", ib); }
        Ws iw;
        hipError_t he = ws_get(ctx, s, 1, ib, iw);
        if (he != hipSuccess) { free_result(t); return fail(TK_ENOMEM, "multigrid start factors: %s", hipGetErrorString(he)); }
        char* p = (char*)iw.p;
        for (int k = 0; k < 3; ++k) {
            double* Uk = (double*)p;
            p += align_up(sizeof(double) * (size_t)gl.n[k] * P.R[k], 256);
            he = launch_interp_factor(t->U[k], gp.n[k], ac.x0[k], ac.h[k], Uk, gl.n[k], af.x0[k], af.h[k], P.R[k], s);
            if (he == hipSuccess) he = launch_qr(Uk, Uk, 1, gl.n[k], P.R[k], s);
            if (he != hipSuccess) { free_result(t); return fail(TK_EHIP, "multigrid prolongation: %s", hipGetErrorString(he)); }
            P.init_U[k] = Uk;
        }
        // the coarse result was last used by the prolongation on s
        if (hipStreamSynchronize(s) != hipSuccess) { free_result(t); return fail(TK_EHIP, "multigrid: stream error"); }
        free_result(t);
        t = nullptr;
        apply_tuning(ctx, &P);
        tk_status lst = TK_OK;
        st = (P.prec == TK_FP64) ? compress_impl<double>(ctx, &kp, 1, nullptr, &gl, P, s, &t, &lst)
                                 : compress_impl<float>(ctx, &kp, 1, nullptr, &gl, P, s, &t, &lst);
        if (st != TK_OK) return st;
        if (lst != TK_OK && lst != TK_ENOCONV) { free_result(t); return lst; }
        if (lst == TK_ENOCONV && l == levels) st = TK_ENOCONV;
    }
    *out = t;
    if (opts->eps > 0 && !(t->rel_err <= opts->eps)) return fail(TK_ENOCONV, "multigrid: E=%g > eps=%g", t->rel_err, opts->eps);
    return st;
}

// Sec. 3.4: the sinc-quadrature canonical tensor of a half-integer Matern (R = 2M + 1 terms,
// side matrices Q_l) and its Tucker form by canonical-to-Tucker: the RHOSVD start (leading
// eigenvectors of Q_l Q_l^T) and `sweeps` ALS sweeps on the canonical data, where the
// single-hole Gram of mode a is Q_a (P_j^T P_j o P_m^T P_m) Q_a^T with P_l = V_l^T Q_l; core
// G_(0) = P_0 KR(P_1, P_2); error against the canonical tensor from ||CP||^2 - ||G||^2.  No full
// tensor is formed: everything is a product of the n_l x R side matrices.
tk_status tk_compress_sinc(tk_ctx* ctx, const tk_kernel* kernel, const tk_grid* grid, int M, double C0,
                           const int ranks[3], int sweeps, void* hip_stream, tk_tucker** out)
{
    if (!ctx || !kernel || !grid || !ranks || !out) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    KernelParams kp{};
    if ((st = check_kernel(kernel, &kp)) != TK_OK) return st;
    if (kernel->family != TK_MATERN || kp.half < 0)
        return fail(TK_EUNSUPPORTED, "sinc canonical tensor: Matern nu in {1/2, 3/2, 5/2} only");
    if (kp.axs[0] != 1.0 || kp.axs[1] != 1.0 || kp.axs[2] != 1.0)
        return fail(TK_EUNSUPPORTED, "sinc canonical tensor: isotropic distance only");
    if (M < 1 || M > 256) return fail(TK_EINVAL, "M=%d: 1..256", M);
    if (!std::isfinite(C0) || C0 <= 0) return fail(TK_EINVAL, "C0 must be finite and > 0");
    if (sweeps < 0 || sweeps > CONVERGE_MAX_SWEEPS) return fail(TK_EINVAL, "sweeps=%d: 0..%d", sweeps, CONVERGE_MAX_SWEEPS);
    const int R = 2 * M + 1;
    int r[3];
    for (int k = 0; k < 3; ++k) {
        r[k] = ranks[k];
        if (r[k] < 1) return fail(TK_EINVAL, "ranks[%d]=%d", k, r[k]);
        r[k] = std::min(r[k], std::min(grid->n[k], R));
        if (r[k] > LIB_RMAX) return fail(TK_EUNSUPPORTED, "rank %d exceeds %d", r[k], LIB_RMAX);
    }
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    const int* n = grid->n;
    const int nmax = std::max(n[0], std::max(n[1], n[2]));
    const int rmax = std::max(r[0], std::max(r[1], r[2]));
    const int pmax = (nmax <= EIG_PMAX) ? nmax : std::min(rmax + 8, EIG_PMAX);
    double *t, *w, *Q[3], *Gq[3], *S, *P[3], *Ga, *Gb, *Wg, *T1, *KR, *core, *V[3], *eQ, *eY, *eH, *eVs, *lam, *scal;
    int* eflags;
    double* eres;
    auto lay = [&](Arena& ar) {
        t = ar.take<double>(R);
        w = ar.take<double>(R);
        for (int k = 0; k < 3; ++k) Q[k] = ar.take<double>((size_t)n[k] * R);
        for (int k = 0; k < 3; ++k) Gq[k] = ar.take<double>((size_t)R * R);
        S = ar.take<double>((size_t)nmax * nmax);
        for (int k = 0; k < 3; ++k) P[k] = ar.take<double>((size_t)r[k] * R);
        Ga = ar.take<double>((size_t)R * R);
        Gb = ar.take<double>((size_t)R * R);
        Wg = ar.take<double>((size_t)R * R);
        T1 = ar.take<double>((size_t)nmax * R);
        KR = ar.take<double>((size_t)R * r[1] * r[2]);
        core = ar.take<double>((size_t)r[0] * r[1] * r[2]);
        for (int k = 0; k < 3; ++k) V[k] = ar.take<double>((size_t)n[k] * r[k]);
        eQ = ar.take<double>((size_t)nmax * pmax);
        eY = ar.take<double>((size_t)nmax * pmax);
        eH = ar.take<double>((size_t)pmax * pmax);
        eVs = ar.take<double>((size_t)pmax * pmax);
        lam = ar.take<double>(64);
        scal = ar.take<double>(16);
        eflags = ar.take<int>(64);
        eres = ar.take<double>(EIG_CHECK_DOUBLES);   // one eigenproblem at a time
    };
    Arena plan;
    lay(plan);
    Reservation res(ctx, plan.off);
    if (!res.take()) return fail(TK_ENOMEM, "sinc compression needs %zu bytes", plan.off);
    Ws wsp;
    TK_HIP(ws_get(ctx, s, 0, plan.off, wsp));
    Arena ar;
    ar.base = (char*)wsp.p;
    lay(ar);
    Work wk{};
    wk.ctx = ctx;
    wk.eflags = eflags;
    wk.eres = eres;
    // leading r_a eigenvectors of the n_a x n_a matrix S into V[a] (FP64, iterated to the
    // residual test like every FP64 eigensolve)
    auto eig_into = [&](int a) -> tk_status {
        EigBatch b{};
        b.count = 1; b.n = n[a]; b.r = r[a];
        b.p = (n[a] <= EIG_PMAX) ? n[a] : std::min(r[a] + 8, EIG_PMAX);
        b.G = S; b.sG = (long)n[a] * n[a];
        b.Q = eQ; b.Y = eY; b.H = eH; b.Vs = eVs;
        b.U = V[a]; b.sU = (long)n[a] * r[a]; b.ldu = r[a];
        b.lam = lam; b.sL = 64;
        TK_LAUNCH(launch_eig(b, COLD_ITERS, s));
        return eig_converge(b, wk, s);
    };
    const double h = C0 * std::log((double)M) / (double)M;
    const double c = kp.inv_len;            // sqrt(2 nu) / ell
    TK_LAUNCH(launch_sinc_nodes(M, h, c, kp.half, kp.sigma2, t, w, s));
    const GridAxes ax = axes_of(grid);
    TK_LAUNCH(launch_sinc_factors(ax, R, t, w, Q, s));
    // RHOSVD start: S = Q_a Q_a^T
    for (int a = 0; a < 3; ++a) {
        GemmArgs g = gemm(n[a], n[a], R, 1, Q[a], 0, R, 1, Q[a], 0, 1, R, S, 0, n[a], 1);
        TK_LAUNCH((launch_gemm<double, double, double>(g, s)));
        if ((st = eig_into(a)) != TK_OK) return st;
    }
    // P_l = V_l^T Q_l (r_l x R)
    auto project = [&](int l) -> tk_status {
        GemmArgs g = gemm(r[l], R, n[l], 1, V[l], 0, 1, r[l], Q[l], 0, R, 1, P[l], 0, R, 1);
        TK_LAUNCH((launch_gemm<double, double, double>(g, s)));
        return TK_OK;
    };
    for (int l = 0; l < 3; ++l)
        if ((st = project(l)) != TK_OK) return st;
    for (int sw = 0; sw < sweeps; ++sw) {
        for (int a = 0; a < 3; ++a) {
            const int j = a == 0 ? 1 : 0, m = a == 2 ? 1 : 2;
            // Wg = (P_j^T P_j) o (P_m^T P_m)
            GemmArgs gj = gemm(R, R, r[j], 1, P[j], 0, 1, R, P[j], 0, R, 1, Ga, 0, R, 1);
            TK_LAUNCH((launch_gemm<double, double, double>(gj, s)));
            GemmArgs gm = gemm(R, R, r[m], 1, P[m], 0, 1, R, P[m], 0, R, 1, Gb, 0, R, 1);
            TK_LAUNCH((launch_gemm<double, double, double>(gm, s)));
            TK_LAUNCH(launch_hadamard(Ga, Gb, Wg, (long)R * R, s));
            // S = (Q_a Wg) Q_a^T
            GemmArgs g1 = gemm(n[a], R, R, 1, Q[a], 0, R, 1, Wg, 0, R, 1, T1, 0, R, 1);
            TK_LAUNCH((launch_gemm<double, double, double>(g1, s)));
            GemmArgs g2 = gemm(n[a], n[a], R, 1, T1, 0, R, 1, Q[a], 0, 1, R, S, 0, n[a], 1);
            TK_LAUNCH((launch_gemm<double, double, double>(g2, s)));
            if ((st = eig_into(a)) != TK_OK) return st;
            if ((st = project(a)) != TK_OK) return st;
        }
    }
    // core G_(0) = P_0 KR(P_1, P_2)
    TK_LAUNCH(launch_khatri_rao(P[1], P[2], R, r[1], r[2], KR, s));
    GemmArgs gc = gemm(r[0], r[1] * r[2], R, 1, P[0], 0, R, 1, KR, 0, (long)r[1] * r[2], 1, core, 0,
                       (long)r[1] * r[2], 1);
    TK_LAUNCH((launch_gemm<double, double, double>(gc, s)));
    // ||CP||^2 = sum_{k,k'} prod_l (Q_l^T Q_l)[k][k'],  ||G||^2
    for (int l = 0; l < 3; ++l) {
        GemmArgs g = gemm(R, R, n[l], 1, Q[l], 0, 1, R, Q[l], 0, R, 1, Gq[l], 0, R, 1);
        TK_LAUNCH((launch_gemm<double, double, double>(g, s)));
    }
    TK_LAUNCH(launch_triple_sum(Gq[0], Gq[1], Gq[2], (long)R * R, scal, s));
    const long ncore = (long)r[0] * r[1] * r[2];
    TK_LAUNCH(launch_dot<double>(core, core, ncore, scal + 4, 8, scal + 1, s));
    double sc[2];
    if ((st = readback(ctx, s, scal, sizeof(sc), sc)) != TK_OK) return st;
    tk_tucker* tt = nullptr;
    if ((st = alloc_result(ctx, n, r, s, &tt)) != TK_OK) return st;
    for (int k = 0; k < 3; ++k) {
        TK_LAUNCH(launch_copy_f64(V[k], tt->U[k], (long)n[k] * r[k], s, Bat()));
        TK_LAUNCH(launch_convert_f64_to_f32(tt->U[k], tt->U32[k], (long)n[k] * r[k], s, Bat()));
    }
    TK_LAUNCH(launch_copy_f64(core, tt->core, ncore, s, Bat()));
    TK_LAUNCH(launch_convert_f64_to_f32(tt->core, tt->core32, ncore, s, Bat()));
    TK_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 3; ++k) tt->b[k] = grid->b[k];
    tt->layout = grid->layout;
    tt->prec = TK_FP64;
    tt->norm_a = std::sqrt(sc[0]);
    tt->rel_err = std::sqrt(std::max(sc[0] - sc[1], 0.0) / sc[0]);
    *out = tt;
    if (wk.noconv) return fail(TK_ENOCONV, "sinc compression: an eigensolve did not pass its residual test");
    return TK_OK;
}

tk_status tk_compress_group(tk_ctx* ctx, int count, const tk_kernel* kernels, const tk_grid* grid,
                            const tk_opts* opts, void* hip_stream, tk_tucker** outs, int* statuses)
{
    if (!ctx || !kernels || !grid || !opts || !outs || !statuses) return fail(TK_EINVAL, "NULL argument");
    if (count < 1 || count > BATCH_MAX) return fail(TK_EINVAL, "count=%d: 1..%d problems per group", count, BATCH_MAX);
    for (int i = 0; i < count; ++i) { outs[i] = nullptr; statuses[i] = TK_OK; }
    tk_status st[BATCH_MAX];
    tk_status r;
    if (count == 1 || !groupable(opts)) {
        for (int i = 0; i < count; ++i) {
            r = compress_any(ctx, &kernels[i], nullptr, grid, opts, hip_stream, &outs[i]);
            if (r == TK_ENOCONV) { statuses[i] = TK_ENOCONV; continue; }
            if (r != TK_OK) {
                std::string m = g_last_error;
                for (int j = 0; j < i; ++j) { free_result(outs[j]); outs[j] = nullptr; }
                return fail(r, "%s", m.c_str());
            }
        }
        return TK_OK;
    }
    const tk_kernel* ks[BATCH_MAX];
    for (int i = 0; i < count; ++i) ks[i] = &kernels[i];
    r = compress_group(ctx, ks, count, grid, opts, (hipStream_t)hip_stream, outs, st);
    if (r != TK_OK) return r;
    for (int i = 0; i < count; ++i) statuses[i] = st[i];
    return TK_OK;
}

tk_status tk_compress_batch(tk_ctx* ctx, int count, const tk_kernel* kernels, const tk_grid* grids,
                            const tk_opts* opts, void* hip_stream, tk_tucker** outs)
{
    if (!ctx || !kernels || !grids || !opts || !outs || count < 0) return fail(TK_EINVAL, "bad batch arguments");
    for (int i = 0; i < count; ++i) outs[i] = nullptr;
    if (count == 0) return TK_OK;
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    // work units: problems on the same grid share launches (chunks of at most BATCH_MAX, near
    // equal in size), the largest units first
    struct Unit {
        std::vector<int> idx;
        double cost;
    };
    std::vector<Unit> units;
    {
        std::vector<int> order(count);
        for (int i = 0; i < count; ++i) order[i] = i;
        auto same_grid = [&](int i, int j) {
            const tk_grid &a = grids[i], &b = grids[j];
            for (int k = 0; k < 3; ++k)
                if (a.n[k] != b.n[k] || a.b[k] != b.b[k]) return false;
            return a.layout == b.layout;
        };
        // every result of the batch stays allocated until the call returns
        size_t all_results = 0;
        for (int i = 0; i < count; ++i) {
            Plan P;
            if (make_plan(&grids[i], opts, &P) == TK_OK) all_results += result_bytes(P.n, P.R);
        }
        std::vector<char> taken(count, 0);
        for (int i = 0; i < count; ++i) {
            if (taken[i]) continue;
            std::vector<int> g{i};
            taken[i] = 1;
            if (groupable(opts))
                for (int j = i + 1; j < count; ++j)
                    if (!taken[j] && same_grid(i, j)) { g.push_back(j); taken[j] = 1; }
            const int m = (int)g.size();
            // the largest chunk whose workspaces fit the budget beside all the batch's results
            int cap = 1;
            if (m > 1) {
                Plan P;
                if (make_plan(&grids[i], opts, &P) == TK_OK) {
                    for (int nb = std::min(m, BATCH_MAX); nb > 1; --nb) {
                        size_t wsz = 0;
                        const size_t need = batch_layout(P, true, nb, &wsz) + all_results;
                        if (need <= ctx->budget) { cap = nb; break; }
                    }
                }
            }
            // a group is also split into its share of the worker streams (in proportion to its
            // problems, at least 3 per part): the latency-bound steps of one part (eigensolver
            // panels, small products) then overlap the streaming steps of the others
            const int share = (int)(((long)ctx->workers * m + count - 1) / count);
            const int nchunk = std::max((m + cap - 1) / cap, std::min(share, m / 3));
            const double per = (double)grids[i].n[0] * grids[i].n[1] * grids[i].n[2];
            for (int c = 0, pos = 0; c < nchunk; ++c) {
                const int len = m / nchunk + (c < m % nchunk ? 1 : 0);
                Unit u;
                u.idx.assign(g.begin() + pos, g.begin() + pos + len);
                u.cost = per * len;
                units.push_back(std::move(u));
                pos += len;
            }
        }
        std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.cost > y.cost; });
    }
    const int nunits = (int)units.size();
    const int W = std::min(nunits, ctx->workers);
    std::vector<hipStream_t> ws(W);
    {
        std::lock_guard<std::mutex> g(ctx->pool_mu);
        while ((int)ctx->streams.size() < W) {
            hipStream_t st;
            TK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            ctx->streams.push_back(st);
        }
        for (int i = 0; i < W; ++i) ws[i] = ctx->streams[i];
    }
    // ---- float tensors: one persistent launch evaluates the grids of every unit, of every size,
    // into a workspace the batch lays out for all units at once (when it fits the budget; the
    // units then run on their slots without a grid launch of their own)
    std::vector<BatchSlot> slots;
    Reservation batch_res(ctx, 0);
    Ws batch_ws;
    std::vector<GridJob> jobs;     // host copies stay alive until the call returns
    std::vector<int> first;
    if (count > 1 && groupable(opts) && opts->prec != TK_FP64) {
        std::vector<size_t> off(nunits), wsz(nunits);
        size_t tot = 0;
        bool ok = true;
        for (int u = 0; u < nunits && ok; ++u) {
            Plan P;
            ok = make_plan(&grids[units[u].idx[0]], opts, &P) == TK_OK;
            if (!ok) break;
            apply_tuning(ctx, &P);
            off[u] = tot;
            tot += align_up(batch_layout(P, true, (int)units[u].idx.size(), &wsz[u]), 256);
        }
        for (int u = 0; u < nunits && ok; ++u)
            for (size_t b = 0; b < units[u].idx.size() && ok; ++b) {
                const int i = units[u].idx[b];
                KernelParams kp{};
                ok = check_kernel(&kernels[i], &kp) == TK_OK;
                if (ok) jobs.push_back(grid_job_f32(nullptr, axes_of(&grids[i]), kp));
                if (ok) jobs.back().A = reinterpret_cast<float*>(off[u] + b * wsz[u]);   // offset for now
            }
        // largest grids first, so that their planes start first
        std::stable_sort(jobs.begin(), jobs.end(), [](const GridJob& a, const GridJob& b) {
            return (long)a.g.n[0] * a.g.n[1] * a.g.n[2] > (long)b.g.n[0] * b.g.n[1] * b.g.n[2];
        });
        first.assign(jobs.size() + 1, 0);
        for (size_t j = 0; j < jobs.size(); ++j) first[j + 1] = first[j] + grid_job_items(jobs[j]);
        const size_t tab = align_up(sizeof(GridJob) * jobs.size(), 256) + align_up(sizeof(int) * first.size(), 256) + 256;
        if (ok && !jobs.empty() && batch_res.take_bytes(tot + tab) &&
            ws_get(ctx, (hipStream_t)hip_stream, 1, tot + tab, batch_ws) == hipSuccess) {
            char* base = (char*)batch_ws.p;
            for (GridJob& j : jobs) j.A = reinterpret_cast<float*>(base + reinterpret_cast<size_t>(j.A));
            GridJob* jobs_dev = (GridJob*)(base + tot);
            int* first_dev = (int*)(base + tot + align_up(sizeof(GridJob) * jobs.size(), 256));
            unsigned* counter = (unsigned*)(base + tot + tab - 256);
            hipStream_t cs = (hipStream_t)hip_stream;
            TK_HIP(hipMemcpyAsync(jobs_dev, jobs.data(), sizeof(GridJob) * jobs.size(), hipMemcpyHostToDevice, cs));
            TK_HIP(hipMemcpyAsync(first_dev, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, cs));
            TK_HIP(hipMemsetAsync(counter, 0, sizeof(unsigned), cs));
            {
                ProfScope ps(TK_PROF_GRID, cs);
                TK_LAUNCH(launch_grid_eval_f32_queue(jobs_dev, (int)jobs.size(), first_dev, first.back(), counter, cs));
            }
            slots.resize(nunits);
            for (int u = 0; u < nunits; ++u) slots[u].base = base + off[u];
        }
    }
    // the items start after the work already queued on the caller's stream
    hipEvent_t fork;
    TK_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    TK_HIP(hipEventRecord(fork, (hipStream_t)hip_stream));
    std::atomic<int> next{0};
    std::mutex mu;
    std::condition_variable cv;
    int running = 0;
    long finished = 0;
    std::vector<tk_status> st(count, TK_OK);
    std::vector<std::string> msg(count);
    auto worker = [&](int wi) {
        if (hipSetDevice(ctx->device) != hipSuccess) return;
        hipStream_t s = ws[wi];
        if (hipStreamWaitEvent(s, fork, 0) != hipSuccess) return;
        for (;;) {
            const int ui = next.fetch_add(1);
            if (ui >= nunits) break;
            const Unit& u = units[ui];
            const int nb = (int)u.idx.size();
            std::vector<const tk_kernel*> ks(nb);
            std::vector<tk_tucker*> os(nb, nullptr);
            std::vector<tk_status> ss(nb, TK_OK);
            for (int b = 0; b < nb; ++b) ks[b] = &kernels[u.idx[b]];
            for (;;) {
                long seen;
                {
                    std::lock_guard<std::mutex> g(mu);
                    ++running;
                    seen = finished;
                }
                tk_status r;
                if (!slots.empty()) {
                    r = compress_group(ctx, ks.data(), nb, &grids[u.idx[0]], opts, s, os.data(), ss.data(),
                                       &slots[ui]);
                } else if (nb == 1) {
                    r = compress_any(ctx, ks[0], nullptr, &grids[u.idx[0]], opts, s, &os[0]);
                    if (r == TK_ENOCONV) { ss[0] = TK_ENOCONV; r = TK_OK; }
                } else {
                    r = compress_group(ctx, ks.data(), nb, &grids[u.idx[0]], opts, s, os.data(), ss.data());
                }
                bool retry = false;
                {
                    std::lock_guard<std::mutex> g(mu);
                    --running;
                    // out of budget while others hold memory: wait for one of them, then retry
                    retry = (r == TK_ENOMEM && (running > 0 || finished != seen));
                    if (!retry) ++finished;
                }
                cv.notify_all();
                if (retry) {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return finished != seen || running == 0; });
                    continue;
                }
                for (int b = 0; b < nb; ++b) {
                    const int i = u.idx[b];
                    outs[i] = os[b];
                    st[i] = (r != TK_OK) ? r : ss[b];
                    if (r != TK_OK) msg[i] = g_last_error;
                    else if (ss[b] == TK_ENOCONV) msg[i] = "eps not reached";
                }
                break;
            }
        }
    };
    std::vector<std::thread> th;
    th.reserve(W);
    for (int i = 0; i < W; ++i) th.emplace_back(worker, i);
    for (auto& t : th) t.join();
    (void)hipEventDestroy(fork);
    for (int i = 0; i < count; ++i) {
        if (outs[i] == nullptr && st[i] == TK_OK) {
            st[i] = TK_EHIP;
            msg[i] = "worker could not start (hipSetDevice / hipStreamWaitEvent failed)";
        }
        if (st[i] != TK_OK && st[i] != TK_ENOCONV) {
            for (int j = 0; j < count; ++j) { free_result(outs[j]); outs[j] = nullptr; }
            return fail(st[i], "batch item %d: %s", i, msg[i].c_str());
        }
    }
    return TK_OK;
}

tk_status tk_tucker_info(const tk_tucker* t, int n[3], int ranks[3], double* rel_err_fro, double* norm_a,
                         int* layout)
{
    if (!t) return fail(TK_EINVAL, "t is NULL");
    for (int k = 0; k < 3; ++k) {
        if (n) n[k] = t->n[k];
        if (ranks) ranks[k] = t->r[k];
    }
    if (rel_err_fro) *rel_err_fro = t->rel_err;
    if (norm_a) *norm_a = t->norm_a;
    if (layout) *layout = t->layout;
    return TK_OK;
}

tk_status tk_tucker_get(const tk_tucker* t, double* U_host[3], double* core_host)
{
    if (!t) return fail(TK_EINVAL, "t is NULL");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    TK_HIP(hipSetDevice(t->ctx->device));
    (void)hipGetLastError();
    // results are complete when the call that made them returns
    for (int k = 0; k < 3; ++k)
        if (U_host && U_host[k])
            TK_HIP(hipMemcpy(U_host[k], t->U[k], sizeof(double) * t->n[k] * t->r[k], hipMemcpyDeviceToHost));
    if (core_host)
        TK_HIP(hipMemcpy(core_host, t->core, sizeof(double) * t->r[0] * t->r[1] * t->r[2], hipMemcpyDeviceToHost));
    return TK_OK;
}

tk_status tk_tucker_device(const tk_tucker* t, const double* U_dev[3], const double** core_dev)
{
    if (!t) return fail(TK_EINVAL, "t is NULL");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    for (int k = 0; k < 3; ++k)
        if (U_dev) U_dev[k] = t->U[k];
    if (core_dev) *core_dev = t->core;
    return TK_OK;
}

tk_status tk_reconstruct(tk_ctx* ctx, const tk_tucker* t, void* A_dev, int io, void* hip_stream)
{
    if (!ctx || !t || !A_dev) return fail(TK_EINVAL, "NULL argument");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    if (io != TK_FP64 && io != TK_FP32) return fail(TK_EINVAL, "io must be TK_FP64 or TK_FP32");
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    const int* n = t->n;
    const int* r = t->r;
    size_t need = sizeof(double) * ((size_t)n[0] * r[1] * r[2] + (size_t)n[0] * n[1] * r[2]) + 1024;
    Reservation res(ctx, need);
    if (!res.take()) return fail(TK_ENOMEM, "reconstruct needs %zu bytes", need);
    void* base = nullptr;
    Ws wsp;
    TK_HIP(ws_get(ctx, s, 0, need, wsp));
    base = wsp.p;
    Arena ar;
    ar.base = (char*)base;
    double* M1 = ar.take<double>((size_t)n[0] * r[1] * r[2]);
    double* H = ar.take<double>((size_t)n[0] * n[1] * r[2]);
    GemmArgs g = gemm(n[0], r[1] * r[2], r[0], 1, t->U[0], 0, r[0], 1, t->core, 0, (long)r[1] * r[2], 1, M1, 0,
                      (long)r[1] * r[2], 1);
    TK_LAUNCH((launch_gemm<double, double, double>(g, s)));
    GemmArgs g1 = gemm(n[1], r[2], r[1], n[0], t->U[1], 0, r[1], 1, M1, (long)r[1] * r[2], r[2], 1, H,
                       (long)n[1] * r[2], r[2], 1);
    TK_LAUNCH((launch_gemm<double, double, double>(g1, s)));
    GemmArgs g2 = gemm(n[0] * n[1], n[2], r[2], 1, H, 0, r[2], 1, t->U[2], 0, 1, r[2], A_dev, 0, n[2], 1);
    if (io == TK_FP64) TK_LAUNCH((launch_gemm<double, double, double>(g2, s)));
    else TK_LAUNCH((launch_gemm<double, double, float>(g2, s)));
    return TK_OK;
}

tk_status tk_cov_dims(const tk_tucker* t, int m[3])
{
    if (!t || !m) return fail(TK_EINVAL, "NULL argument");
    int off[3];
    if (!cov_geometry(t, off, m)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    return TK_OK;
}

tk_status tk_kron_matvec(tk_ctx* ctx, const tk_tucker* t, const void* z_dev, void* y_dev, int io, void* hip_stream)
{
    if (!ctx || !t || !z_dev || !y_dev) return fail(TK_EINVAL, "NULL argument");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    if (z_dev == y_dev) return fail(TK_EINVAL, "y must not alias z");
    if (io != TK_FP64 && io != TK_FP32) return fail(TK_EINVAL, "io must be TK_FP64 or TK_FP32");
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    if (io == TK_FP64 && ctx->matvec_method == TK_MV_FFT) return fail(TK_EINVAL, "the FFT matvec is FP32 only");
    if (use_fft(ctx, t, io))
        return matvec_fft(ctx, t, (const float*)z_dev, (float*)y_dev, (hipStream_t)hip_stream, nullptr);
    if (io == TK_FP32)
        return matvec_impl<float>(ctx, t, (const float*)z_dev, (float*)y_dev, (hipStream_t)hip_stream, nullptr);
    return matvec_impl<double>(ctx, t, (const double*)z_dev, (double*)y_dev, (hipStream_t)hip_stream, nullptr);
}

// The FFT matvec of tk_kron_matvec on the device's fixed scratch area: the same kernels and
// launch shapes (so the same y, bit for bit), no allocation, no budget charge.  Nothing in the
// workspace needs to start at zero (every buffer is written before it is read), so the contents
// a previous call left behind do not matter; two calls that overlap on one device race.
tk_status tk_kron_matvec_noalloc(tk_ctx* ctx, const tk_tucker* t, const float* z_dev, float* y_dev,
                                 void* hip_stream)
{
    if (!ctx || !t || !z_dev || !y_dev) return fail(TK_EINVAL, "NULL argument");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    if ((const void*)z_dev == (const void*)y_dev) return fail(TK_EINVAL, "y must not alias z");
    if (!ctx->scratch) return fail(TK_EHIP, "no scratch address on device %d", ctx->device);
    MvGeom g;
    if (!mv_geom(t, &g)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    if (g.r2p > LIB_RMAX)
        return fail(TK_EUNSUPPORTED, "third rank %d exceeds %d (the FFT matvec's register tile)", g.r[2], LIB_RMAX);
    Arena plan;
    MvPre b;
    float2 *A1, *A2;
    mv_lay(plan, g, &b, &A1, &A2);
    if (plan.off > NOALLOC_SCRATCH_BYTES)
        return fail(TK_ENOMEM, "operator %dx%dx%d at ranks (%d,%d,%d) needs %zu bytes of workspace; the "
                    "no-allocation scratch holds %zu (up to 64 points per axis)", g.m[0], g.m[1], g.m[2], g.r[0],
                    g.r[1], g.r[2], plan.off, NOALLOC_SCRATCH_BYTES);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    Arena ar;
    ar.base = (char*)ctx->scratch;
    mv_lay(ar, g, &b, &A1, &A2);
    tk_status st;
    if ((st = mv_preamble(t, g, b, s)) != TK_OK) return st;
    return mv_passes(g, b, A1, A2, z_dev, y_dev, nullptr, s);
}

tk_status tk_quadratic_form(tk_ctx* ctx, const tk_tucker* t, const void* z_dev, int io, void* hip_stream,
                            double* out, void* y_dev)
{
    if (!ctx || !t || !z_dev || !out) return fail(TK_EINVAL, "NULL argument");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    if (io != TK_FP64 && io != TK_FP32) return fail(TK_EINVAL, "io must be TK_FP64 or TK_FP32");
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    int off[3], m[3];
    if (!cov_geometry(t, off, m)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    void* ybuf = y_dev;
    size_t esz = io == TK_FP32 ? 4 : 8;
    size_t ybytes = esz * (size_t)m[0] * m[1] * m[2];
    const bool fft = use_fft(ctx, t, io);       // the FFT path sums z . y without storing y
    Reservation res(ctx, (y_dev || fft) ? 0 : ybytes);
    Ws yws;
    if (!y_dev && !fft) {
        if (!res.take()) return fail(TK_ENOMEM, "quadratic form needs %zu bytes", ybytes);
        hipError_t he = ws_get(ctx, s, 1, ybytes, yws);
        if (he != hipSuccess) return fail(TK_ENOMEM, "y of %zu bytes: %s", ybytes, hipGetErrorString(he));
        ybuf = yws.p;
    }
    tk_status st;
    if (io == TK_FP64 && ctx->matvec_method == TK_MV_FFT) st = fail(TK_EINVAL, "the FFT matvec is FP32 only");
    else if (fft)
        st = matvec_fft(ctx, t, (const float*)z_dev, (float*)ybuf, s, out);
    else if (io == TK_FP32)
        st = matvec_impl<float>(ctx, t, (const float*)z_dev, (float*)ybuf, s, out);
    else
        st = matvec_impl<double>(ctx, t, (const double*)z_dev, (double*)ybuf, s, out);
    return st;
}

tk_status tk_quadratic_form_batch(tk_ctx* ctx, int count, const tk_tucker* const* ts, const void* const* z_devs,
                                  int io, void* hip_stream, double* out, void* const* y_devs)
{
    if (!ctx || !ts || !z_devs || !out || count < 0) return fail(TK_EINVAL, "bad batch arguments");
    if (count == 0) return TK_OK;
    for (int i = 0; i < count; ++i)
        if (!ts[i] || !z_devs[i]) return fail(TK_EINVAL, "item %d: NULL result or vector", i);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    if (io != TK_FP64 && io != TK_FP32) return fail(TK_EINVAL, "io must be TK_FP64 or TK_FP32");
    bool all_fft = true;
    for (int i = 0; i < count; ++i) all_fft = all_fft && use_fft(ctx, ts[i], io);
    if (all_fft) {
        for (int i = 0; i < count; ++i)
            if (!usable(ts[i])) return fail(TK_EINVAL, "item %d: result of a destroyed context", i);
        hipStream_t side;
        {
            std::lock_guard<std::mutex> g(ctx->pool_mu);
            if (ctx->streams.empty()) {
                hipStream_t st;
                TK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
                ctx->streams.push_back(st);
            }
            side = ctx->streams[0];
        }
        return quadform_fft_batch(ctx, count, ts, z_devs, y_devs, (hipStream_t)hip_stream, side, out);
    }
    const int W = std::min(count, ctx->workers);
    std::vector<hipStream_t> ws(W);
    {
        std::lock_guard<std::mutex> g(ctx->pool_mu);
        while ((int)ctx->streams.size() < W) {
            hipStream_t st;
            TK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            ctx->streams.push_back(st);
        }
        for (int i = 0; i < W; ++i) ws[i] = ctx->streams[i];
    }
    // the items start after the work already queued on the caller's stream
    hipEvent_t fork;
    TK_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    TK_HIP(hipEventRecord(fork, (hipStream_t)hip_stream));
    std::atomic<int> next{0};
    std::vector<tk_status> st(count, TK_OK);
    std::vector<std::string> msg(count);
    auto worker = [&](int wi) {
        if (hipSetDevice(ctx->device) != hipSuccess) return;
        hipStream_t s = ws[wi];
        if (hipStreamWaitEvent(s, fork, 0) != hipSuccess) return;
        for (;;) {
            const int i = next.fetch_add(1);
            if (i >= count) break;
            st[i] = tk_quadratic_form(ctx, ts[i], z_devs[i], io, s, &out[i], y_devs ? y_devs[i] : nullptr);
            if (st[i] != TK_OK) msg[i] = g_last_error;
        }
    };
    std::vector<std::thread> th;
    th.reserve(W);
    for (int i = 0; i < W; ++i) th.emplace_back(worker, i);
    for (auto& t : th) t.join();
    (void)hipEventDestroy(fork);
    for (int i = 0; i < count; ++i)
        if (st[i] != TK_OK) return fail(st[i], "batch item %d: %s", i, msg[i].c_str());
    return TK_OK;
}

tk_status tk_estimate_matvec_bytes(tk_ctx* ctx, const tk_tucker* t, int io, size_t* bytes)
{
    if (!ctx || !t || !bytes) return fail(TK_EINVAL, "NULL argument");
    if (io != TK_FP64 && io != TK_FP32) return fail(TK_EINVAL, "io must be TK_FP64 or TK_FP32");
    int off[3], m[3];
    if (!cov_geometry(t, off, m)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    if (use_fft(ctx, t, io)) return matvec_fft(ctx, t, nullptr, nullptr, nullptr, nullptr, bytes);
    *bytes = matvec_work_bytes(t, io == TK_FP32 ? 4 : 8);
    return TK_OK;
}

tk_status tk_trace(tk_ctx* ctx, const tk_tucker* t, void* hip_stream, double* out)
{
    if (!ctx || !t || !out) return fail(TK_EINVAL, "NULL argument");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    int off[3], m[3];
    if (!cov_geometry(t, off, m)) return fail(TK_ELAYOUT, "even-sized centred grid has no origin node");
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    Slot slot(ctx);
    if (slot.i < 0) return fail(TK_EHIP, "trace: all %d staging slots busy", tk_ctx::kSlots);
    double scale = (double)m[0] * m[1] * m[2];
    hipError_t e = launch_cov_trace(t->core, t->r[0], t->r[1], t->r[2], t->U[0] + (long)off[0] * t->r[0],
                                    t->U[1] + (long)off[1] * t->r[1], t->U[2] + (long)off[2] * t->r[2], scale,
                                    (double*)slot.dev(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(slot.host(), slot.dev(), sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) std::memcpy(out, slot.host(), sizeof(double));
    if (e != hipSuccess) return fail(TK_EHIP, "trace: %s", hipGetErrorString(e));
    return TK_OK;
}

tk_status tk_tucker_save(const tk_tucker* t, const char* path)
{
    if (!t || !path) return fail(TK_EINVAL, "NULL argument");
    if (!usable(t)) return fail(TK_EINVAL, "result of a destroyed context");
    std::vector<std::vector<double>> U(3);
    for (int k = 0; k < 3; ++k) U[k].resize((size_t)t->n[k] * t->r[k]);
    std::vector<double> core((size_t)t->r[0] * t->r[1] * t->r[2]);
    double* Up[3] = {U[0].data(), U[1].data(), U[2].data()};
    tk_status st = tk_tucker_get(t, Up, core.data());
    if (st != TK_OK) return st;
    FILE* f = fopen(path, "wb");
    if (!f) return fail(TK_EINVAL, "cannot open %s for writing", path);
    const char magic[8] = {'T', 'K', 'T', 'U', 'C', 'K', '0', '1'};
    int32_t hdr[8] = {1, t->n[0], t->n[1], t->n[2], t->r[0], t->r[1], t->r[2], t->layout};
    double meta[5] = {t->b[0], t->b[1], t->b[2], t->rel_err, t->norm_a};
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(meta, sizeof(meta), 1, f) == 1;
    for (int k = 0; k < 3 && ok; ++k) ok = fwrite(U[k].data(), sizeof(double), U[k].size(), f) == U[k].size();
    if (ok) ok = fwrite(core.data(), sizeof(double), core.size(), f) == core.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(TK_EINVAL, "write to %s failed", path);
    return TK_OK;
}

tk_status tk_tucker_load(tk_ctx* ctx, const char* path, tk_tucker** out)
{
    if (!ctx || !path || !out) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(TK_EINVAL, "cannot open %s", path);
    char magic[8];
    int32_t hdr[8];
    double meta[5];
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "TKTUCK01", 8) == 0 && fread(hdr, sizeof(hdr), 1, f) == 1 &&
              fread(meta, sizeof(meta), 1, f) == 1 && hdr[0] == 1;
    int n[3] = {hdr[1], hdr[2], hdr[3]}, r[3] = {hdr[4], hdr[5], hdr[6]};
    for (int k = 0; k < 3 && ok; ++k) ok = n[k] >= 1 && n[k] <= NMAX && r[k] >= 1 && r[k] <= n[k] && r[k] <= EIG_PMAX;
    ok = ok && (hdr[7] == TK_CENTERED || hdr[7] == TK_OFFSET);
    std::vector<std::vector<double>> U(3);
    std::vector<double> core;
    if (ok) {
        for (int k = 0; k < 3 && ok; ++k) {
            U[k].resize((size_t)n[k] * r[k]);
            ok = fread(U[k].data(), sizeof(double), U[k].size(), f) == U[k].size();
        }
        core.resize((size_t)r[0] * r[1] * r[2]);
        if (ok) ok = fread(core.data(), sizeof(double), core.size(), f) == core.size();
    }
    fclose(f);
    if (!ok) return fail(TK_EINVAL, "%s is not a valid result file", path);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    tk_tucker* t = nullptr;
    tk_status st = alloc_result(ctx, n, r, nullptr, &t);
    if (st != TK_OK) return st;
    for (int k = 0; k < 3; ++k) {
        hipError_t e = hipMemcpy(t->U[k], U[k].data(), sizeof(double) * U[k].size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_convert_f64_to_f32(t->U[k], t->U32[k], (long)U[k].size(), nullptr);
        if (e != hipSuccess) { free_result(t); return fail(TK_EHIP, "load: %s", hipGetErrorString(e)); }
    }
    hipError_t e = hipMemcpy(t->core, core.data(), sizeof(double) * core.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_convert_f64_to_f32(t->core, t->core32, (long)core.size(), nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { free_result(t); return fail(TK_EHIP, "load: %s", hipGetErrorString(e)); }
    for (int k = 0; k < 3; ++k) t->b[k] = meta[k];
    t->layout = hdr[7];
    t->rel_err = meta[3];
    t->norm_a = meta[4];
    *out = t;
    return TK_OK;
}

void tk_tucker_free(tk_tucker* t) { free_result(t); }

tk_status tk_normal_fill(tk_ctx* ctx, uint32_t seed, uint32_t stream_id, float* z_dev, size_t count,
                         void* hip_stream)
{
    if (!ctx || (!z_dev && count)) return fail(TK_EINVAL, "NULL argument");
    if (count > ((size_t)1 << 32)) return fail(TK_EINVAL, "count %zu above 2^32", count);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    TK_LAUNCH(launch_philox_normal(seed, stream_id, (long)count, z_dev, (hipStream_t)hip_stream));
    return TK_OK;
}

tk_status tk_philox4x32(tk_ctx* ctx, const uint32_t key[2], uint64_t counter0, size_t nblocks, uint32_t* out_dev,
                        void* hip_stream)
{
    if (!ctx || !key || (!out_dev && nblocks)) return fail(TK_EINVAL, "NULL argument");
    if (((uintptr_t)out_dev & 15) != 0) return fail(TK_EINVAL, "out_dev must be 16-byte aligned");
    if (nblocks > ((size_t)1 << 31)) return fail(TK_EINVAL, "nblocks %zu above 2^31", nblocks);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    TK_LAUNCH(launch_philox_words(key[0], key[1], (unsigned long long)counter0, (long)nblocks, out_dev,
                                  (hipStream_t)hip_stream));
    return TK_OK;
}

tk_status tk_grid_eval(tk_ctx* ctx, const tk_kernel* kernel, const tk_grid* grid, int prec, void* A_dev,
                       void* hip_stream)
{
    if (!ctx || !A_dev) return fail(TK_EINVAL, "NULL argument");
    tk_status st;
    if ((st = check_grid(grid)) != TK_OK) return st;
    KernelParams kp{};
    if ((st = check_kernel(kernel, &kp)) != TK_OK) return st;
    if (prec < TK_FP64 || prec > TK_BF16X3) return fail(TK_EINVAL, "unknown precision %d", prec);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    GridAxes ax = axes_of(grid);
    hipStream_t s = (hipStream_t)hip_stream;
    RadialGrid rg{};
    if (radial_plan(ax, &kp, 1, &rg)) {
        const size_t bytes = sizeof(double) * (size_t)rg.T;
        Reservation res(ctx, bytes);
        if (!res.take()) return fail(TK_ENOMEM, "radial table of %zu bytes", bytes);
        Ws wsp;
        hipError_t e = ws_get(ctx, s, 0, bytes, wsp);
        if (e != hipSuccess) return fail(TK_ENOMEM, "workspace: %s", hipGetErrorString(e));
        TK_LAUNCH(launch_grid_eval_radial(A_dev, prec == TK_FP64 ? 8 : 4, ax, &kp, rg, (double*)wsp.p, s));
        return TK_OK;
    }
    if (prec == TK_FP64) TK_LAUNCH(launch_grid_eval_f64((double*)A_dev, ax, &kp, s));
    else TK_LAUNCH(launch_grid_eval_f32((float*)A_dev, ax, &kp, s));
    return TK_OK;
}

tk_status tk_gram(tk_ctx* ctx, const void* A_dev, const int n[3], int mode, int prec, double* G_dev, void* hip_stream)
{
    if (!ctx || !A_dev || !n || !G_dev) return fail(TK_EINVAL, "NULL argument");
    if (mode < 0 || mode > 2) return fail(TK_EINVAL, "mode %d", mode);
    if (prec < TK_FP64 || prec > TK_BF16X3) return fail(TK_EINVAL, "unknown precision %d", prec);
    for (int k = 0; k < 3; ++k)
        if (n[k] < 1 || n[k] > NMAX) return fail(TK_EINVAL, "n[%d]=%d", k, n[k]);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    size_t wb = gram_work_bytes(n, mode, prec);
    Reservation res(ctx, wb);
    if (!res.take()) return fail(TK_ENOMEM, "gram needs %zu bytes", wb);
    Ws wsp;
    TK_HIP(ws_get(ctx, s, 0, wb, wsp));
    hipError_t e = launch_gram(A_dev, n, mode, prec, G_dev, wsp.p, s);
    if (e != hipSuccess) return fail(TK_EHIP, "gram launch: %s", hipGetErrorString(e));
    return TK_OK;
}

tk_status tk_eig_topr(tk_ctx* ctx, int count, int n, int r, const double* G_dev, double* lambda_dev, double* U_dev,
                      void* hip_stream)
{
    if (!ctx || !G_dev || !lambda_dev || !U_dev) return fail(TK_EINVAL, "NULL argument");
    if (count < 1 || n < 1 || n > NMAX || r < 1 || r > n) return fail(TK_EINVAL, "bad sizes");
    if (r > LIB_RMAX) return fail(TK_EUNSUPPORTED, "r=%d exceeds %d", r, LIB_RMAX);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    int p = (n <= EIG_PMAX) ? n : std::min(r + 8, EIG_PMAX);
    size_t need = sizeof(double) * ((size_t)count * (2 * (size_t)n * p + 2 * (size_t)p * p + 64) +
                                    64 * (size_t)EIG_CHECK_DOUBLES) + 8192;
    Reservation res(ctx, need);
    if (!res.take()) return fail(TK_ENOMEM, "eig needs %zu bytes", need);
    Ws wsp;
    TK_HIP(ws_get(ctx, s, 0, need, wsp));
    Arena ar;
    ar.base = (char*)wsp.p;
    EigBatch b{};
    b.count = count; b.n = n; b.p = p; b.r = r;
    b.G = G_dev; b.sG = (long)n * n;
    b.Q = ar.take<double>((size_t)count * n * p);
    b.Y = ar.take<double>((size_t)count * n * p);
    b.H = ar.take<double>((size_t)count * p * p);
    b.Vs = ar.take<double>((size_t)count * p * p);
    b.U = U_dev; b.sU = (long)n * r; b.ldu = r;
    b.lam = lambda_dev; b.sL = r;
    hipError_t e = launch_eig(b, COLD_ITERS, s);
    if (e != hipSuccess) return fail(TK_EHIP, "eig launch: %s", hipGetErrorString(e));
    // iterate until the Ritz pairs pass the residual test, in groups of at most 64 problems
    Work w{};
    w.ctx = ctx;
    w.eflags = ar.take<int>(64);
    w.eres = ar.take<double>(64 * (size_t)EIG_CHECK_DOUBLES);
    for (int c0 = 0; c0 < count; c0 += 64) {
        EigBatch bc = b;
        bc.count = std::min(64, count - c0);
        bc.G = b.G + (long)c0 * b.sG;
        bc.Q = b.Q + (long)c0 * n * p;
        bc.Y = b.Y + (long)c0 * n * p;
        bc.H = b.H + (long)c0 * p * p;
        bc.Vs = b.Vs + (long)c0 * p * p;
        bc.U = b.U + (long)c0 * b.sU;
        bc.lam = b.lam + (long)c0 * b.sL;
        tk_status st = eig_converge(bc, w, s);
        if (st != TK_OK) return st;
    }
    TK_HIP(hipStreamSynchronize(s));
    if (w.noconv) return fail(TK_ENOCONV, "eigensolver: residual test not met after %d rounds", EIG_MAX_ROUNDS);
    return TK_OK;
}

// ------------------------------------------------------------------------------------------
// Separable covariance C = C_1 (x) C_2 (x) C_3 (Sec. 4, "Separable covariance matrices")
// ------------------------------------------------------------------------------------------
}  // extern "C"

struct tk_kron1 {
    tk_ctx* ctx = nullptr;
    int n[3] = {0, 0, 0};
    void* block = nullptr;        // L_k, then (after the first solve) C_k^-1 and scratch
    size_t bytes = 0;             // charged to the context's budget
    double* L[3] = {nullptr, nullptr, nullptr};
    double* Cinv[3] = {nullptr, nullptr, nullptr};
    void* inv_block = nullptr;    // L_k^-1 and C_k^-1, formed at the first solve
    double logdet = 0.0;
    double logdet_k[3] = {0, 0, 0};
};

namespace {

// Lazily form C_k^-1 = L_k^-T L_k^-1 (n_k <= 1024) for the solves.
tk_status kron1_inverses(tk_kron1* k, hipStream_t s)
{
    if (k->Cinv[0]) return TK_OK;
    for (int a = 0; a < 3; ++a)
        if (k->n[a] > NMAX) return fail(TK_EUNSUPPORTED, "solve: axis %d has %d > %d points", a, k->n[a], NMAX);
    size_t need = 0;
    for (int a = 0; a < 3; ++a) need += 2 * align_up(sizeof(double) * (size_t)k->n[a] * k->n[a], 256);
    if (!reserve(k->ctx, need)) return fail(TK_ENOMEM, "inverse factors need %zu bytes", need);
    void* blk = nullptr;
    hipError_t e = hipMalloc(&blk, need);
    if (e != hipSuccess) { release(k->ctx, need); return fail(TK_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e)); }
    char* p = (char*)blk;
    for (int a = 0; a < 3; ++a) {
        const int n = k->n[a];
        double* Li = (double*)p;
        p += align_up(sizeof(double) * (size_t)n * n, 256);
        double* Ci = (double*)p;
        p += align_up(sizeof(double) * (size_t)n * n, 256);
        TK_LAUNCH(launch_trinv(k->L[a], n, Li, Ci, s));   // Ci (n x n) is free until the product below
        // C^-1 = Li^T Li
        GemmArgs g = gemm(n, n, n, 1, Li, 0, 1, n, Li, 0, n, 1, Ci, 0, n, 1);
        TK_LAUNCH((launch_gemm<double, double, double>(g, s)));
        k->Cinv[a] = Ci;
    }
    TK_HIP(hipStreamSynchronize(s));
    k->inv_block = blk;
    k->bytes += need;
    return TK_OK;
}

// y = x x_1 M_1 x_2 M_2 x_3 M_3 (M_k: n_k x n_k row-major, applied along mode k) through two
// scratch volumes; the result lands in y.
tk_status kron1_apply(const int n[3], double* const M[3], const double* x, double* y, double* tmp, hipStream_t s)
{
    const long N12 = (long)n[1] * n[2], N01 = (long)n[0] * n[1];
    // mode 1: tmp[i0][.] = sum_j M0[i0][j] x[j][.]
    GemmArgs g0 = gemm(n[0], (int)N12, n[0], 1, M[0], 0, n[0], 1, x, 0, N12, 1, tmp, 0, N12, 1);
    TK_LAUNCH((launch_gemm<double, double, double>(g0, s)));
    // mode 2: y[i0][i1][.] = sum_j M1[i1][j] tmp[i0][j][.]   (batch over i0)
    GemmArgs g1 = gemm(n[1], n[2], n[1], n[0], M[1], 0, n[1], 1, tmp, N12, n[2], 1, y, N12, n[2], 1);
    TK_LAUNCH((launch_gemm<double, double, double>(g1, s)));
    // mode 3: tmp[r][i2] = sum_j y[r][j] M2[i2][j]
    GemmArgs g2 = gemm((int)N01, n[2], n[2], 1, y, 0, n[2], 1, M[2], 0, 1, n[2], tmp, 0, n[2], 1);
    TK_LAUNCH((launch_gemm<double, double, double>(g2, s)));
    TK_HIP(hipMemcpyAsync(y, tmp, sizeof(double) * (size_t)N01 * n[2], hipMemcpyDeviceToDevice, s));
    return TK_OK;
}

}  // namespace

extern "C" {

tk_status tk_kron1_create(tk_ctx* ctx, const tk_kernel kernels[3], const tk_grid* grid, const double nugget[3],
                          void* hip_stream, tk_kron1** out)
{
    if (!ctx || !kernels || !grid || !out) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    if (!grid) return fail(TK_EINVAL, "grid is NULL");
    KernelParams kp[3];
    tk_status st;
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1 || grid->n[a] > KRON1_NMAX)
            return fail(TK_EUNSUPPORTED, "axis %d: %d points (1..%d)", a, grid->n[a], KRON1_NMAX);
        if (!std::isfinite(grid->b[a]) || grid->b[a] <= 0) return fail(TK_EINVAL, "grid b[%d] must be > 0", a);
        if ((st = check_kernel(&kernels[a], &kp[a])) != TK_OK) return st;
        const double ng = nugget ? nugget[a] : 0.0;
        if (!std::isfinite(ng) || ng < 0) return fail(TK_EINVAL, "nugget[%d] must be finite and >= 0", a);
    }
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    size_t bytes = 0;
    for (int a = 0; a < 3; ++a) bytes += align_up(sizeof(double) * (size_t)grid->n[a] * grid->n[a], 256);
    size_t wb = 0;
    for (int a = 0; a < 3; ++a) wb = std::max(wb, cholesky_work_bytes(grid->n[a]));
    Reservation res(ctx, bytes + wb + 256);
    if (!res.take()) return fail(TK_ENOMEM, "separable covariance needs %zu bytes", bytes + wb);
    tk_kron1* k = new (std::nothrow) tk_kron1();
    if (!k) return fail(TK_ENOMEM, "host allocation failed");
    k->ctx = ctx;
    hipError_t e = hipMalloc(&k->block, bytes);
    if (e != hipSuccess) { delete k; return fail(TK_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e)); }
    Ws wsp;
    e = ws_get(ctx, s, 0, wb + 256, wsp);
    if (e != hipSuccess) { hipFree(k->block); delete k; return fail(TK_ENOMEM, "workspace: %s", hipGetErrorString(e)); }
    int* info = (int*)wsp.p;
    double* ld = (double*)((char*)wsp.p + 64);
    void* work = (char*)wsp.p + 256;
    char* p = (char*)k->block;
    const GridAxes ax = axes_of(grid);
    int hinfo[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        const int n = grid->n[a];
        k->n[a] = n;
        k->L[a] = (double*)p;
        p += align_up(sizeof(double) * (size_t)n * n, 256);
        const double h = (n > 1) ? ax.h[a] : 0.0;
        TK_HIP(hipMemsetAsync(info + a, 0, sizeof(int), s));
        tk_status ls = TK_OK;
        if (launch_cov1d(k->L[a], n, ax.x0[a], h, kp[a], nugget ? nugget[a] : 0.0, s) != hipSuccess ||
            launch_cholesky(k->L[a], n, work, info + a, s) != hipSuccess ||
            launch_logdet_chol(k->L[a], n, ld + a, s) != hipSuccess)
            ls = fail(TK_EHIP, "separable covariance factor %d: %s", a, hipGetErrorString(hipGetLastError()));
        if (ls != TK_OK) { hipFree(k->block); delete k; return ls; }
    }
    double hld[3];
    TK_HIP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    TK_HIP(hipMemcpyAsync(hld, ld, sizeof(hld), hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    for (int a = 0; a < 3; ++a)
        if (hinfo[a] != 0) {
            hipFree(k->block);
            delete k;
            return fail(TK_EINVAL, "axis %d: the covariance factor is not positive definite (pivot %d); add a nugget",
                        a, hinfo[a] - 1);
        }
    const double N = (double)grid->n[0] * grid->n[1] * grid->n[2];
    k->logdet = 0.0;
    for (int a = 0; a < 3; ++a) {
        k->logdet_k[a] = hld[a];
        k->logdet += (N / grid->n[a]) * hld[a];
    }
    k->bytes = bytes;
    res.hand_over(bytes);
    *out = k;
    return TK_OK;
}

tk_status tk_kron1_logdet(const tk_kron1* k, double* out, double logdet_axis[3])
{
    if (!k || !out) return fail(TK_EINVAL, "NULL argument");
    *out = k->logdet;
    if (logdet_axis)
        for (int a = 0; a < 3; ++a) logdet_axis[a] = k->logdet_k[a];
    return TK_OK;
}

tk_status tk_kron1_factor(const tk_kron1* k, int axis, double* L_host)
{
    if (!k || !L_host || axis < 0 || axis > 2) return fail(TK_EINVAL, "bad argument");
    TK_HIP(hipSetDevice(k->ctx->device));
    TK_HIP(hipMemcpy(L_host, k->L[axis], sizeof(double) * (size_t)k->n[axis] * k->n[axis], hipMemcpyDeviceToHost));
    return TK_OK;
}

tk_status tk_kron1_apply(tk_ctx* ctx, tk_kron1* k, int op, const double* z_dev, double* y_dev, void* hip_stream)
{
    if (!ctx || !k || !z_dev || !y_dev) return fail(TK_EINVAL, "NULL argument");
    if (z_dev == y_dev) return fail(TK_EINVAL, "y must not alias z");
    if (op != TK_KRON1_SOLVE && op != TK_KRON1_CHOL) return fail(TK_EINVAL, "unknown operation %d", op);
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    tk_status st;
    if (op == TK_KRON1_SOLVE && (st = kron1_inverses(k, s)) != TK_OK) return st;
    const size_t N = (size_t)k->n[0] * k->n[1] * k->n[2];
    Reservation res(ctx, sizeof(double) * N);
    if (!res.take()) return fail(TK_ENOMEM, "scratch of %zu bytes", sizeof(double) * N);
    Ws wsp;
    hipError_t e = ws_get(ctx, s, 0, sizeof(double) * N, wsp);
    if (e != hipSuccess) return fail(TK_ENOMEM, "workspace: %s", hipGetErrorString(e));
    double* M[3];
    for (int a = 0; a < 3; ++a) M[a] = (op == TK_KRON1_SOLVE) ? k->Cinv[a] : k->L[a];
    return kron1_apply(k->n, M, z_dev, y_dev, (double*)wsp.p, s);
}

tk_status tk_kron1_loglik(tk_ctx* ctx, tk_kron1* k, const double* z_dev, void* hip_stream, double* out,
                          double* quad_out)
{
    if (!ctx || !k || !z_dev || !out) return fail(TK_EINVAL, "NULL argument");
    TK_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)hip_stream;
    tk_status st;
    if ((st = kron1_inverses(k, s)) != TK_OK) return st;
    const size_t N = (size_t)k->n[0] * k->n[1] * k->n[2];
    const size_t need = 2 * sizeof(double) * N + sizeof(double) * 2048 + 256;
    Reservation res(ctx, need);
    if (!res.take()) return fail(TK_ENOMEM, "log-likelihood needs %zu bytes", need);
    Ws wsp;
    hipError_t e = ws_get(ctx, s, 0, need, wsp);
    if (e != hipSuccess) return fail(TK_ENOMEM, "workspace: %s", hipGetErrorString(e));
    double* w = (double*)wsp.p;
    double* tmp = w + N;
    double* parts = tmp + N;
    if ((st = kron1_apply(k->n, k->Cinv, z_dev, w, tmp, s)) != TK_OK) return st;
    TK_LAUNCH(launch_dot<double>(z_dev, w, (long)N, parts, 1024, parts + 1024, s));
    double q = 0.0;
    if ((st = readback(ctx, s, parts + 1024, sizeof(double), &q)) != TK_OK) return st;
    if (quad_out) *quad_out = q;
    *out = -0.5 * ((double)N * std::log(2.0 * M_PI) + k->logdet + q);
    return TK_OK;
}

void tk_kron1_free(tk_kron1* k)
{
    if (!k) return;
    hipSetDevice(k->ctx->device);
    hipDeviceSynchronize();
    if (k->block) hipFree(k->block);
    if (k->inv_block) hipFree(k->inv_block);
    release(k->ctx, k->bytes);
    delete k;
}

}  // extern "C"
