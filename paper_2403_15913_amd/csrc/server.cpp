// Served form: a request loop over resident sparsity patterns.
//
// Each registered pattern's symbolic analysis is uploaded once and stays on
// the device. A request names a pattern and brings new values (W, J, Sigma)
// and a right-hand side: a refactor+solve with the pattern's analysis reused
// (section "Hybrid linear solver": the symbolic factorisation is computed
// once and only refactorisations follow). Requests wait in one FIFO queue.
// Worker threads, each with its own HIP stream and a fixed HBM arena of
// budget / workers bytes, repeatedly take the longest FIFO prefix that fits
// their arena (and max_wave), gather its inputs with one copy kernel, run
// the batched refactor + refined solve over all of them, and scatter the
// solutions back. Requests that arrive while a wave runs join the next wave
// of whichever worker frees up first, so waves from different workers
// overlap on the GPU (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/kkt.h"
#include "api_internal.hpp"

using namespace kkt;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SrvRequest {
    int64_t ticket = 0;
    int pat = 0;
    const Symbolic* sym = nullptr;
    const DevPattern* dpat = nullptr;
    size_t bytes = 0;
    const double *w = nullptr, *j = nullptr, *sx = nullptr, *ss = nullptr, *b = nullptr;
    double* x = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream: the inputs and x are ready after it
    double t_submit = 0, t_start = 0, t_done = 0;
    kkt_status status = KKT_OK;
    kkt_solve_info info{};
    bool done = false;
};

struct SrvWorker {
    hipStream_t st = nullptr;
    DevBuf arena;
    size_t cap = 0;
    Engine eng;
    DevBuf segs;
    CopySeg* hsegs = nullptr;  // pinned
    int seg_cap = 0;
    std::thread th;
    ~SrvWorker() {
        if (hsegs) (void)hipHostFree(hsegs);
        if (st) (void)hipStreamDestroy(st);
    }
};

}  // namespace

struct kkt_server {
    kkt_server_opts o{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<const Symbolic*> psym;
    std::vector<std::unique_ptr<DevPattern>> ppat;
    std::vector<size_t> pbytes;
    std::deque<SrvRequest*> queue;
    std::unordered_map<int64_t, std::unique_ptr<SrvRequest>> reqs;
    int64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::unique_ptr<SrvWorker>> workers;
    std::vector<hipEvent_t> ev_free;  // events for the requests' readiness, reused
    // statistics since the last reset
    std::vector<double> lat, qdel, svc;
    int64_t submitted = 0, completed = 0, rejected = 0, waves = 0, wave_reqs = 0;
    double t_first = -1.0, t_last = 0.0;
};

static void run_wave(kkt_server* S, SrvWorker* W, std::vector<SrvRequest*>& wave) {
    const int nq = (int)wave.size();
    std::vector<const Symbolic*> syms(nq);
    std::vector<const DevPattern*> pats(nq);
    for (int q = 0; q < nq; q++) {
        syms[q] = wave[q]->sym;
        pats[q] = wave[q]->dpat;
    }
    Engine& E = W->eng;
    kkt_status st = E.place(syms, pats, (char*)W->arena.p, W->cap, true, W->st, nullptr);
    std::vector<kkt_solve_info> infos(nq);
    std::vector<int> fst(nq, 0), bad(nq, -1);
    if (st == KKT_OK) {
        int ns = 0;
        auto seg = [&](const double* src, double* dst, int64_t len) {
            if (len > 0) W->hsegs[ns++] = CopySeg{src, dst, len};
        };
        for (int q = 0; q < nq; q++) {
            const SrvRequest* r = wave[q];
            const Symbolic& Y = *r->sym;
            seg(r->w, E.stage.w + E.w_ofs[q], Y.nnz_w);
            seg(r->j, E.stage.j + E.j_ofs[q], Y.nnz_j);
            seg(r->sx, E.stage.sx + E.n_ofs[q], Y.n);
            seg(r->ss, E.stage.ss + E.m_ofs[q], Y.m);
            seg(r->b, E.stage.b + E.n_ofs[q], Y.n);
        }
        // the gather reads the requests' arrays only after the work their
        // submitters had queued before submitting
        hipError_t e = hipSuccess;
        for (int q = 0; q < nq && e == hipSuccess; q++) e = hipStreamWaitEvent(W->st, wave[q]->ready, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(W->segs.p, W->hsegs, ns * sizeof(CopySeg), hipMemcpyHostToDevice, W->st);
        if (e != hipSuccess) st = hip_fail(e, "segment upload");
        if (st == KKT_OK) {
            launch_copy_segments((const CopySeg*)W->segs.p, ns, W->st);
            Calls C;
            std::memset(&C, 0, sizeof(C));
            C.w = E.stage.w; C.jv = E.stage.j; C.sx = E.stage.sx; C.ss = E.stage.ss; C.gamma = 0.0;
            st = E.refactor(C, W->st);
            if (st == KKT_OK) {
                Calls X;
                std::memset(&X, 0, sizeof(X));
                X.b = E.stage.b;
                X.x = E.stage.x;
                st = E.solve(X, S->o.refine_max_iter, S->o.refine_tol, infos.data(), W->st);
                // per-request factor status (the solve reports the worst of the wave)
                kkt_status rs = E.read_status(fst.data(), bad.data());
                if (rs == KKT_ERR_DEVICE || rs == KKT_ERR_OOM) st = rs;
                else if (st != KKT_ERR_DEVICE && st != KKT_ERR_OOM) st = KKT_OK;
            }
        }
        if (st == KKT_OK) {
            // the segment list is still read by the gather kernel until the
            // stream passes it; the solve above synchronised, so reuse is safe
            ns = 0;
            for (int q = 0; q < nq; q++) seg(E.stage.x + E.n_ofs[q], wave[q]->x, wave[q]->sym->n);
            hipError_t e2 = hipMemcpyAsync(W->segs.p, W->hsegs, ns * sizeof(CopySeg), hipMemcpyHostToDevice, W->st);
            if (e2 == hipSuccess) {
                launch_copy_segments((const CopySeg*)W->segs.p, ns, W->st);
                e2 = hipStreamSynchronize(W->st);
            }
            if (e2 != hipSuccess) st = hip_fail(e2, "result scatter");
        }
    }
    const double t = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    for (int q = 0; q < nq; q++) {
        SrvRequest* r = wave[q];
        r->t_done = t;
        r->info = infos[q];
        if (st != KKT_OK) r->status = st;
        else if (fst[q] != KKT_OK) r->status = fst[q];
        else r->status = infos[q].status;
        r->info.status = r->status;
        r->done = true;
        S->ev_free.push_back(r->ready);  // the worker's stream has passed the wait on it
        r->ready = nullptr;
        S->lat.push_back(r->t_done - r->t_submit);
        S->qdel.push_back(r->t_start - r->t_submit);
        S->svc.push_back(r->t_done - r->t_start);
        S->completed++;
    }
    S->waves++;
    S->wave_reqs += nq;
    S->t_last = std::max(S->t_last, t);
    S->cv_done.notify_all();
}

static void worker_loop(kkt_server* S, SrvWorker* W) {
    for (;;) {
        std::vector<SrvRequest*> wave;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->queue.empty()) {
                if (S->stop) return;
                continue;
            }
            if (S->o.linger_us > 0 && (int)S->queue.size() < S->o.max_wave && !S->stop) {
                const auto until = std::chrono::steady_clock::now() +
                                   std::chrono::microseconds((int64_t)S->o.linger_us);
                S->cv_work.wait_until(lk, until, [&] { return S->stop || (int)S->queue.size() >= S->o.max_wave; });
                if (S->queue.empty()) continue;
            }
            size_t bytes = 0;
            while (!S->queue.empty() && (int)wave.size() < S->o.max_wave) {
                SrvRequest* r = S->queue.front();
                if (bytes + r->bytes > W->cap) break;
                bytes += r->bytes;
                wave.push_back(r);
                S->queue.pop_front();
            }
            const double t = now_s();
            for (SrvRequest* r : wave) r->t_start = t;
            if (!S->queue.empty()) S->cv_work.notify_one();
        }
        if (!wave.empty()) run_wave(S, W, wave);
    }
}

extern "C" {

void kkt_server_opts_default(kkt_server_opts* o) {
    if (!o) return;
    o->hbm_budget = (int64_t)8 << 30;
    o->max_wave = 64;
    o->workers = 2;
    o->refine_max_iter = 10;
    o->refine_tol = 1e-14;
    o->linger_us = 0.0;
}

kkt_status kkt_server_create(const kkt_server_opts* opt, kkt_server** out) {
    if (!out) return fail(KKT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    kkt_server_opts o;
    kkt_server_opts_default(&o);
    if (opt) o = *opt;
    if (o.hbm_budget <= 0 || o.max_wave < 1 || o.workers < 1 || o.workers > 8 || o.refine_max_iter < 0 ||
        !(o.refine_tol >= 0.0) || !(o.linger_us >= 0.0))
        return fail(KKT_ERR_INVALID_ARG, "bad server options");
    kkt_status st = ensure_runtime();
    if (st) return st;
    std::unique_ptr<kkt_server> S(new (std::nothrow) kkt_server);
    if (!S) return fail(KKT_ERR_OOM, "host allocation");
    S->o = o;
    const size_t cap = (size_t)(o.hbm_budget / o.workers) & ~(size_t)255;
    const int seg_cap = 5 * o.max_wave + 8;
    for (int k = 0; k < o.workers; k++) {
        std::unique_ptr<SrvWorker> W(new SrvWorker);
        hipError_t e = hipStreamCreateWithFlags(&W->st, hipStreamNonBlocking);
        if (e == hipSuccess) e = W->arena.alloc(cap);
        if (e == hipSuccess) e = W->segs.alloc(seg_cap * sizeof(CopySeg));
        if (e == hipSuccess) e = hipHostMalloc((void**)&W->hsegs, seg_cap * sizeof(CopySeg), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "server worker setup");
        W->cap = cap;
        W->seg_cap = seg_cap;
        S->workers.push_back(std::move(W));
    }
    for (auto& W : S->workers) W->th = std::thread(worker_loop, S.get(), W.get());
    *out = S.release();
    return KKT_OK;
}

kkt_status kkt_server_register(kkt_server* S, const kkt_symbolic* sym, int32_t* pattern_id) {
    if (!S || !sym || !pattern_id) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    std::unique_ptr<DevPattern> dp(new (std::nothrow) DevPattern);
    if (!dp) return fail(KKT_ERR_OOM, "host allocation");
    hipError_t e = dp->build(sym->S);
    if (e != hipSuccess) return hip_fail(e, "pattern upload");
    const size_t need = instance_bytes(sym->S);
    std::lock_guard<std::mutex> lk(S->mu);
    if (need > S->workers[0]->cap) return fail(KKT_ERR_BUDGET, "one request of this pattern exceeds a worker's HBM share");
    S->psym.push_back(&sym->S);
    S->ppat.push_back(std::move(dp));
    S->pbytes.push_back(need);
    *pattern_id = (int32_t)S->psym.size() - 1;
    return KKT_OK;
}

kkt_status kkt_server_submit(kkt_server* S, int32_t pattern_id, const double* w_vals, const double* j_vals,
                             const double* sigma_x, const double* sigma_s, const double* b, double* x,
                             void* stream, int64_t* ticket) {
    if (!S || !ticket) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    std::unique_ptr<SrvRequest> r(new (std::nothrow) SrvRequest);
    if (!r) return fail(KKT_ERR_OOM, "host allocation");
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->ev_free.empty()) {
            ev = S->ev_free.back();
            S->ev_free.pop_back();
        }
    }
    hipError_t e = ev ? hipSuccess : hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)stream);
    if (e != hipSuccess) {
        if (ev) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->ev_free.push_back(ev);
        }
        return hip_fail(e, "request event");
    }
    r->ready = ev;
    std::lock_guard<std::mutex> lk(S->mu);
    auto give_back = [&] { S->ev_free.push_back(ev); };
    if (pattern_id < 0 || pattern_id >= (int)S->psym.size()) {
        give_back();
        return fail(KKT_ERR_INVALID_ARG, "unknown pattern id");
    }
    const Symbolic& Y = *S->psym[pattern_id];
    if ((Y.nnz_w > 0 && !w_vals) || (Y.nnz_j > 0 && !j_vals) || (Y.n > 0 && (!sigma_x || !b || !x)) ||
        (Y.m > 0 && !sigma_s)) {
        give_back();
        return fail(KKT_ERR_INVALID_ARG, "NULL request array");
    }
    r->ticket = S->next_ticket++;
    r->pat = pattern_id;
    r->sym = &Y;
    r->dpat = S->ppat[pattern_id].get();
    r->bytes = S->pbytes[pattern_id];
    r->w = w_vals; r->j = j_vals; r->sx = sigma_x; r->ss = sigma_s; r->b = b; r->x = x;
    r->t_submit = now_s();
    if (S->t_first < 0) S->t_first = r->t_submit;
    S->submitted++;
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs.emplace(r->ticket, std::move(r));
    S->cv_work.notify_one();
    return KKT_OK;
}

kkt_status kkt_server_wait(kkt_server* S, int64_t ticket, kkt_solve_info* info, double* latency_s) {
    if (!S) return fail(KKT_ERR_INVALID_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(KKT_ERR_INVALID_ARG, "unknown ticket");
    SrvRequest* r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done; });
    if (info) *info = r->info;
    if (latency_s) *latency_s = r->t_done - r->t_submit;
    const kkt_status st = r->status;
    S->reqs.erase(it);
    return st;
}

static double pct(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * v.size()) - 1);
    return v[std::max<size_t>(k, 0)];
}

kkt_status kkt_server_get_stats(kkt_server* S, kkt_server_stats* out) {
    if (!S || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->waves = S->waves;
    out->mean_wave = S->waves ? (double)S->wave_reqs / S->waves : 0.0;
    out->p50_s = pct(S->lat, 0.50);
    out->p99_s = pct(S->lat, 0.99);
    double sq = 0, ss = 0;
    for (double v : S->qdel) sq += v;
    for (double v : S->svc) ss += v;
    out->mean_queue_s = S->qdel.empty() ? 0.0 : sq / S->qdel.size();
    out->mean_service_s = S->svc.empty() ? 0.0 : ss / S->svc.size();
    out->window_s = S->t_first >= 0 ? S->t_last - S->t_first : 0.0;
    out->throughput = out->window_s > 0 ? S->completed / out->window_s : 0.0;
    return KKT_OK;
}

kkt_status kkt_server_reset_stats(kkt_server* S) {
    if (!S) return fail(KKT_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    S->lat.clear();
    S->qdel.clear();
    S->svc.clear();
    S->submitted = S->completed = S->rejected = S->waves = S->wave_reqs = 0;
    S->t_first = -1.0;
    S->t_last = 0.0;
    return KKT_OK;
}

void kkt_server_destroy(kkt_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& W : S->workers)
        if (W->th.joinable()) W->th.join();
    for (hipEvent_t ev : S->ev_free) (void)hipEventDestroy(ev);
    for (auto& kv : S->reqs)
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete S;
}

}  // extern "C"
