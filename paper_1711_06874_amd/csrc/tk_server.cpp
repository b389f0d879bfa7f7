// Request loop for mixed compress / covariance requests on resident results (C ABI in tk.h).
//
// Requests are queued in arrival order.  W worker threads, each with its own non-blocking HIP
// stream, take the first queued request that can run now: a compress request when its
// estimated peak bytes fit the context's HBM budget next to what is resident and what has been
// admitted, a follow-up (matvec, trace, quadratic form) when the compress it refers to has
// finished and its workspace fits.  A request that cannot run yet stays queued while later
// ones go ahead, so requests that arrive while others are on the GPU are admitted as workers
// and memory free up and their work overlaps on the device.  Compress results stay resident
// (owned by the server) until released.  Built on the public entry points only.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tk.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Resident {
    tk_tucker* t = nullptr;
    int users = 0;           // follow-ups running on it
    bool released = false;   // free once users drops to 0
};

struct Pending {
    long long id;
    tk_request r;
    Clock::time_point t_submit;
    size_t est = 0;          // admission estimate (0 until computed)
    hipEvent_t ready = nullptr;   // recorded on the submitter's stream; the worker waits for it
    bool solo = false;       // run alone (a group it was part of did not fit)
};

// Compress requests that may share launches: same grid, same options.
bool same_problem_shape(const tk_request& a, const tk_request& b)
{
    if (a.kind != TK_REQ_COMPRESS || b.kind != TK_REQ_COMPRESS) return false;
    for (int k = 0; k < 3; ++k)
        if (a.grid.n[k] != b.grid.n[k] || a.grid.b[k] != b.grid.b[k] || a.opts.ranks[k] != b.opts.ranks[k])
            return false;
    return a.grid.layout == b.grid.layout && a.opts.eps == b.opts.eps && a.opts.r_max == b.opts.r_max &&
           a.opts.hooi_sweeps == b.opts.hooi_sweeps && a.opts.prec == b.opts.prec;
}

}  // namespace

struct tk_server {
    tk_ctx* ctx = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> threads;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int group_max = 32;                           // compress requests one pass may take
    long long next_id = 1;
    int running = 0;
    size_t admitted = 0;                          // estimates of running requests
    std::deque<Pending> queue;
    std::map<long long, tk_result> done;          // finished, not yet collected
    std::map<long long, int> collected;           // tickets already returned by tk_server_wait
    std::map<long long, Resident> resident;       // compress results
    std::map<long long, int> compress_state;      // 0 queued/running, 1 resident, -1 failed or released
    Clock::time_point origin;
};

namespace {

double secs(const tk_server* sv, Clock::time_point t)
{
    return std::chrono::duration<double>(t - sv->origin).count();
}

void set_error(tk_result* res, const char* msg)
{
    std::snprintf(res->error, sizeof(res->error), "%s", msg ? msg : "");
}

// Can request p start now?  Sets p.est.  Caller holds the lock.  Returns 1 (run), 0 (wait),
// -1 (fails at once: sets *fail_status).
int admissible(tk_server* sv, Pending& p, tk_status* fail_status)
{
    size_t budget = 0, in_use = 0;
    tk_ctx_budget(sv->ctx, &budget, &in_use);
    if (p.r.kind == TK_REQ_COMPRESS) {
        if (p.est == 0) {
            size_t e = 0;
            if (tk_estimate_bytes(&p.r.grid, &p.r.opts, &e) != TK_OK) {
                *fail_status = TK_EINVAL;
                return -1;
            }
            p.est = e > 0 ? e : 1;
        }
    } else {
        auto st = sv->compress_state.find(p.r.target);
        if (st == sv->compress_state.end() || st->second < 0) {
            *fail_status = TK_EINVAL;         // unknown, failed or released target
            return -1;
        }
        if (st->second == 0) return 0;        // target still queued or running
        if (p.est == 0) {
            size_t e = 0;
            if (p.r.kind != TK_REQ_TRACE) {
                if (tk_estimate_matvec_bytes(sv->ctx, sv->resident[p.r.target].t, p.r.io, &e) != TK_OK) {
                    *fail_status = TK_EINVAL;
                    return -1;
                }
            }
            p.est = e > 0 ? e : 1;
        }
    }
    // nothing else running: try it even if the estimate says no (it fails cleanly with ENOMEM)
    if (sv->running == 0) return 1;
    return (in_use + sv->admitted + p.est <= budget) ? 1 : 0;
}

void run_one(tk_server* sv, const Pending& p, hipStream_t s, tk_result* res, tk_tucker** made)
{
    tk_status st = TK_OK;
    *made = nullptr;
    const tk_request& r = p.r;
    if (p.ready && hipStreamWaitEvent(s, p.ready, 0) != hipSuccess) {
        res->status = TK_EHIP;
        set_error(res, "hipStreamWaitEvent on the request's ready event failed");
        return;
    }
    if (r.kind == TK_REQ_COMPRESS) {
        st = tk_compress(sv->ctx, &r.kernel, &r.grid, &r.opts, s, made);
        if (*made) {
            int n[3], rk[3], lay;
            double e, na;
            tk_tucker_info(*made, n, rk, &e, &na, &lay);
            std::memcpy(res->ranks, rk, sizeof(rk));
            res->rel_err = e;
        }
    } else {
        tk_tucker* t;
        {
            std::lock_guard<std::mutex> g(sv->mu);
            t = sv->resident[r.target].t;
        }
        if (r.kind == TK_REQ_MATVEC) {
            st = tk_kron_matvec(sv->ctx, t, r.z_dev, r.y_dev, r.io, s);
            if (st == TK_OK && hipStreamSynchronize(s) != hipSuccess) st = TK_EHIP;
        } else if (r.kind == TK_REQ_TRACE) {
            st = tk_trace(sv->ctx, t, s, &res->value);
        } else {
            st = tk_quadratic_form(sv->ctx, t, r.z_dev, r.io, s, &res->value, r.y_dev);
        }
    }
    res->status = st;
    if (st != TK_OK) set_error(res, tk_last_error());
}

// Compress requests on one grid in one pass (tk_compress_group); res[b] per member.
void run_group(tk_server* sv, const std::vector<Pending>& g, hipStream_t s, std::vector<tk_result>& res,
               std::vector<tk_tucker*>& made)
{
    const int nb = (int)g.size();
    made.assign(nb, nullptr);
    for (const Pending& p : g)
        if (p.ready && hipStreamWaitEvent(s, p.ready, 0) != hipSuccess) {
            for (tk_result& r : res) {
                r.status = TK_EHIP;
                set_error(&r, "hipStreamWaitEvent on a request's ready event failed");
            }
            return;
        }
    std::vector<tk_kernel> ks(nb);
    for (int b = 0; b < nb; ++b) ks[b] = g[b].r.kernel;
    std::vector<int> sts(nb, TK_OK);
    const tk_status st = tk_compress_group(sv->ctx, nb, ks.data(), &g[0].r.grid, &g[0].r.opts, s, made.data(),
                                           sts.data());
    for (int b = 0; b < nb; ++b) {
        if (st != TK_OK) {
            res[b].status = st;
            set_error(&res[b], tk_last_error());
            made[b] = nullptr;
            continue;
        }
        res[b].status = sts[b];
        int n[3], rk[3], lay;
        double e, na;
        tk_tucker_info(made[b], n, rk, &e, &na, &lay);
        std::memcpy(res[b].ranks, rk, sizeof(rk));
        res[b].rel_err = e;
        if (sts[b] != TK_OK) set_error(&res[b], "eps not reached within r_max");
    }
}

void worker(tk_server* sv, int wi)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipStream_t s = sv->streams[wi];
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // first request (in arrival order) that can run now
        auto it = sv->queue.begin();
        int verdict = 0;
        tk_status fst = TK_OK;
        for (; it != sv->queue.end(); ++it) {
            verdict = admissible(sv, *it, &fst);
            if (verdict != 0) break;
        }
        if (it == sv->queue.end()) {
            if (sv->stop && sv->queue.empty()) return;
            sv->cv_work.wait(lk);
            continue;
        }
        Pending p = *it;
        sv->queue.erase(it);
        tk_result res{};
        res.kind = p.r.kind;
        res.t_submit = secs(sv, p.t_submit);
        if (verdict < 0) {
            if (p.ready) (void)hipEventDestroy(p.ready);
            res.status = fst;
            set_error(&res, p.r.kind == TK_REQ_COMPRESS ? "tk_estimate_bytes rejected the grid or options"
                                                        : "follow-up on an unknown, failed or released compress, "
                                                          "or its vectors were rejected");
            res.t_start = res.t_end = secs(sv, Clock::now());
            if (p.r.kind == TK_REQ_COMPRESS) sv->compress_state[p.id] = -1;
            sv->done[p.id] = res;
            sv->cv_done.notify_all();
            continue;
        }
        // continuous batching: queued compress requests on the same grid join this pass while
        // their estimates fit the budget
        std::vector<Pending> group{p};
        size_t est_sum = p.est;
        if (p.r.kind == TK_REQ_COMPRESS && !p.solo && sv->group_max > 1) {
            size_t budget = 0, in_use = 0;
            tk_ctx_budget(sv->ctx, &budget, &in_use);
            for (auto jt = sv->queue.begin(); jt != sv->queue.end() && (int)group.size() < sv->group_max;) {
                tk_status jf = TK_OK;
                if (!jt->solo && same_problem_shape(jt->r, p.r) && admissible(sv, *jt, &jf) == 1 &&
                    in_use + sv->admitted + est_sum + jt->est <= budget) {
                    est_sum += jt->est;
                    group.push_back(*jt);
                    jt = sv->queue.erase(jt);
                    continue;
                }
                ++jt;
            }
        }
        const int nb = (int)group.size();
        ++sv->running;
        sv->admitted += est_sum;
        if (p.r.kind != TK_REQ_COMPRESS) ++sv->resident[p.r.target].users;
        lk.unlock();
        std::vector<tk_result> rs(nb, res);
        for (int b = 0; b < nb; ++b) {
            rs[b].kind = group[b].r.kind;
            rs[b].t_submit = secs(sv, group[b].t_submit);
        }
        const double t0 = secs(sv, Clock::now());
        std::vector<tk_tucker*> made(nb, nullptr);
        if (nb == 1) run_one(sv, p, s, &rs[0], &made[0]);
        else run_group(sv, group, s, rs, made);
        const double t1 = secs(sv, Clock::now());
        for (tk_result& r : rs) { r.t_start = t0; r.t_end = t1; }
        std::vector<tk_tucker*> to_free;
        lk.lock();
        --sv->running;
        sv->admitted -= est_sum;
        if (rs[0].status == TK_ENOMEM && (sv->running > 0 || nb > 1)) {
            // memory went to requests admitted meanwhile (or the group was too large): queue
            // the requests again at the front, a group's members to run alone
            for (tk_tucker* t : made)
                if (t) to_free.push_back(t);
            if (p.r.kind != TK_REQ_COMPRESS) --sv->resident[p.r.target].users;
            for (int b = nb - 1; b >= 0; --b) {
                if (nb > 1) group[b].solo = true;
                sv->queue.push_front(group[b]);
            }
        } else {
            for (int b = 0; b < nb; ++b) {
                const Pending& q = group[b];
                if (q.ready) (void)hipEventDestroy(q.ready);
                if (q.r.kind == TK_REQ_COMPRESS) {
                    if (made[b] && (rs[b].status == TK_OK || rs[b].status == TK_ENOCONV)) {
                        sv->resident[q.id].t = made[b];
                        sv->compress_state[q.id] = 1;
                    } else {
                        if (made[b]) to_free.push_back(made[b]);
                        sv->compress_state[q.id] = -1;
                    }
                } else {
                    Resident& rsd = sv->resident[q.r.target];
                    if (--rsd.users == 0 && rsd.released) {
                        to_free.push_back(rsd.t);
                        sv->resident.erase(q.r.target);
                    }
                }
                sv->done[q.id] = rs[b];
            }
            sv->cv_done.notify_all();
        }
        sv->cv_work.notify_all();
        if (!to_free.empty()) {
            lk.unlock();
            for (tk_tucker* t : to_free) tk_tucker_free(t);
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

tk_status tk_server_create(tk_ctx* ctx, int workers, tk_server** out)
{
    if (!ctx || !out || workers < 1 || workers > 16) return TK_EINVAL;
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TK_EHIP;
    tk_server* sv = new (std::nothrow) tk_server();
    if (!sv) return TK_ENOMEM;
    sv->ctx = ctx;
    sv->origin = Clock::now();
    for (int i = 0; i < workers; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
            delete sv;
            return TK_EHIP;
        }
        sv->streams.push_back(s);
    }
    for (int i = 0; i < workers; ++i)
        sv->threads.emplace_back([sv, i, dev] {
            (void)hipSetDevice(dev);
            worker(sv, i);
        });
    *out = sv;
    return TK_OK;
}

tk_status tk_server_set_batching(tk_server* sv, int max_group)
{
    if (!sv || max_group < 1 || max_group > 32) return TK_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    sv->group_max = max_group;
    return TK_OK;
}

tk_status tk_server_submit(tk_server* sv, const tk_request* req, long long* ticket)
{
    if (!sv || !req || !ticket) return TK_EINVAL;
    if (req->kind < TK_REQ_COMPRESS || req->kind > TK_REQ_QUADFORM) return TK_EINVAL;
    if ((req->kind == TK_REQ_MATVEC && (!req->z_dev || !req->y_dev)) ||
        (req->kind == TK_REQ_QUADFORM && !req->z_dev))
        return TK_EINVAL;
    // only the vectors of a matvec or quadratic form are device inputs that the submitter may
    // still be producing; an event on its stream orders the request after that work
    hipEvent_t ready = nullptr;
    const bool vectors = req->kind == TK_REQ_MATVEC || req->kind == TK_REQ_QUADFORM;
    if (vectors && req->stream != TK_STREAM_READY) {
        if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return TK_EHIP;
        if (hipEventRecord(ready, (hipStream_t)req->stream) != hipSuccess) {
            (void)hipEventDestroy(ready);
            return TK_EHIP;
        }
    }
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) {
        if (ready) (void)hipEventDestroy(ready);
        return TK_EINVAL;
    }
    Pending p;
    p.id = sv->next_id++;
    p.r = *req;
    p.t_submit = Clock::now();
    p.ready = ready;
    if (req->kind == TK_REQ_COMPRESS) sv->compress_state[p.id] = 0;
    sv->queue.push_back(p);
    *ticket = p.id;
    sv->cv_work.notify_all();
    return TK_OK;
}

tk_status tk_server_wait(tk_server* sv, long long ticket, tk_result* out)
{
    if (!sv || !out) return TK_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (ticket < 1 || ticket >= sv->next_id || sv->collected.count(ticket)) return TK_EINVAL;
    for (;;) {
        auto it = sv->done.find(ticket);
        if (it != sv->done.end()) {
            *out = it->second;
            sv->done.erase(it);
            sv->collected[ticket] = 1;
            return TK_OK;
        }
        sv->cv_done.wait(lk);
    }
}

tk_status tk_server_tucker(tk_server* sv, long long compress_ticket, const tk_tucker** out)
{
    if (!sv || !out) return TK_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->resident.find(compress_ticket);
    if (it == sv->resident.end() || it->second.released) return TK_EINVAL;
    *out = it->second.t;
    return TK_OK;
}

tk_status tk_server_release(tk_server* sv, long long compress_ticket)
{
    if (!sv) return TK_EINVAL;
    tk_tucker* t = nullptr;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        auto it = sv->resident.find(compress_ticket);
        if (it == sv->resident.end() || it->second.released) return TK_EINVAL;
        sv->compress_state[compress_ticket] = -1;
        if (it->second.users > 0) {
            it->second.released = true;          // freed by the last follow-up using it
            return TK_OK;
        }
        t = it->second.t;
        sv->resident.erase(it);
    }
    tk_tucker_free(t);
    return TK_OK;
}

void tk_server_destroy(tk_server* sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    for (auto& th : sv->threads) th.join();
    for (auto& kv : sv->resident)
        if (kv.second.t) tk_tucker_free(kv.second.t);
    for (hipStream_t s : sv->streams) {
        (void)hipStreamSynchronize(s);
        (void)tk_ctx_release_stream(sv->ctx, s);
        (void)hipStreamDestroy(s);
    }
    delete sv;
}

}  // extern "C"
