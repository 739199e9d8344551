// Continuous-batching forecast server (wm_serve_*; contracts in wm.h).
//
// One scheduler thread per server drives two HIP streams: a copy stream
// (state in/out and dtype conversion) and a compute stream (processor
// steps).  Each iteration it
//   1. admits queued requests while a state slot is free (slots are carved
//      out of the HBM budget at creation), copying their state in on the
//      copy stream;
//   2. retires finished work by querying events (no blocking waits);
//   3. if fewer than two step batches are queued on the compute stream,
//      forms the next batch: the admitted, idle requests whose next
//      processor (greedy 6 h / 1 h schedule) matches that of the oldest such
//      request, up to max_batch of them, and enqueues one processor step
//      over the batch: with float32 slots the kernels read and write the
//      slots in place through a device array of the batch's slot pointers
//      (written by a small kernel on the compute stream, so no host buffer
//      has to outlive the call); with bfloat16 slots (half the memory) the
//      slots are converted into a float32 batch buffer and back.
// Requests join and leave between steps.  Kernels compute each state's
// tokens the same way whatever the batch, so results match a run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <mutex>
#include <set>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/wm.h"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace wm;

namespace {

enum ReqState { RQ_QUEUED, RQ_LOADING, RQ_IDLE, RQ_RUNNING, RQ_UNLOADING, RQ_DONE };

struct Request {
    uint64_t id = 0;
    int lead = 0;
    std::vector<int> sched;
    int cursor = 0;
    int slot = -1;
    ReqState st = RQ_QUEUED;
    hipEvent_t ev = nullptr;          // completion of the pending copy
    std::vector<float> host_in, host_out;
    wm_req_stats stats{};
};

struct Batch {
    std::vector<Request *> reqs;
    hipEvent_t ev = nullptr;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct wm_server {
    wm_ctx *ctx = nullptr;                // private context (workspace of the compute stream)
    const wm_processor *p6 = nullptr, *p1 = nullptr;
    wm_serve_cfg cfg{};
    int device = 0;
    size_t elems = 0;                     // floats per state
    size_t slot_bytes = 0;
    void *slot_mem = nullptr;
    int nslots = 0;
    std::vector<int> free_slots;
    float *batch = nullptr;               // [max_batch][elems] float32 (bf16 slots)
    float **dptrs = nullptr;              // device array of the batch's slot pointers (f32 slots)
    // cfg.graphs: the step of (processor step size, batch size) as a graph,
    // captured the second time that shape runs (the first, eager, run sets
    // the kernels' one-time attributes outside any capture)
    std::set<std::pair<int, int>> warmed;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::set<std::pair<int, int>> no_graph;   // shapes whose capture failed: they stay eager
    float *stage_in = nullptr, *stage_out = nullptr;   // float32 staging (bf16 slots)
    float *pin_in = nullptr, *pin_out = nullptr;       // pinned host staging of one state
    hipStream_t s_comp = nullptr, s_copy = nullptr;
    std::vector<hipEvent_t> ev_pool;

    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::thread th;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    std::deque<Batch> inflight;
    uint64_t next_id = 1;
    std::chrono::steady_clock::time_point t0;
    int err_code = WM_OK;
    char err_msg[256] = {0};
    bool loading = false;                 // the staging buffer holds an admission in flight
    bool unloading = false;

    void *slot_ptr(int s) { return (char *)slot_mem + (size_t)s * slot_bytes; }

    hipEvent_t get_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void put_event(hipEvent_t e) {
        if (e) ev_pool.push_back(e);
    }
    void set_error(int code, const char *what, hipError_t e) {
        if (err_code == WM_OK) {
            err_code = code;
            snprintf(err_msg, sizeof err_msg, "%s: %s", what, hipGetErrorString(e));
        }
    }
    // Whether the work before event e has finished.  Only hipErrorNotReady
    // means "still running": any other code is an asynchronous failure,
    // recorded so that every later poll reports it.
    bool done(hipEvent_t e) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipSuccess) return true;
        if (q != hipErrorNotReady) set_error(WM_EHIP, "device work", q);
        return false;
    }

    // ---- one scheduler iteration; returns true if it made progress ----
    // Called with `lk` held; host copies of whole states run with it released
    // (only this thread touches a request between admission and RQ_DONE).
    bool step_once(std::unique_lock<std::mutex> &lk) {
        bool progress = false;
        hipError_t e;
        if (err_code != WM_OK) return false;
        // retire state copies
        Request *finished = nullptr;
        for (auto &kv : reqs) {
            Request *r = kv.second;
            if (r->st == RQ_UNLOADING && done(r->ev)) {
                finished = r;
                break;
            }
        }
        if (finished) {
            Request *r = finished;
            put_event(r->ev);
            r->ev = nullptr;
            lk.unlock();
            r->host_out.assign(pin_out, pin_out + elems);
            lk.lock();
            unloading = false;
            free_slots.push_back(r->slot);
            r->slot = -1;
            r->stats.t_done = now_s(t0);
            r->st = RQ_DONE;
            progress = true;
        }
        for (auto &kv : reqs) {
            Request *r = kv.second;
            if (r->st == RQ_LOADING && done(r->ev)) {
                put_event(r->ev);
                r->ev = nullptr;
                loading = false;
                r->host_in.clear();
                r->host_in.shrink_to_fit();
                r->stats.t_admit = now_s(t0);
                r->st = RQ_IDLE;
                progress = true;
            }
        }
        // retire step batches (in order)
        while (!inflight.empty() && done(inflight.front().ev)) {
            Batch &b = inflight.front();
            for (Request *r : b.reqs) {
                r->cursor += 1;
                r->stats.steps += 1;
                r->stats.batches += 1;
                r->stats.max_cobatch = std::max(r->stats.max_cobatch, (int)b.reqs.size());
                r->st = RQ_IDLE;
            }
            put_event(b.ev);
            inflight.pop_front();
            progress = true;
        }
        // start copying out finished states (one at a time through the staging buffer)
        if (!unloading) {
            for (auto &kv : reqs) {
                Request *r = kv.second;
                if (r->st != RQ_IDLE || r->cursor < (int)r->sched.size()) continue;
                const float *src = (const float *)slot_ptr(r->slot);
                if (cfg.state_bf16) {
                    if ((e = launch_convert(slot_ptr(r->slot), true, stage_out, false, elems, s_copy)) != hipSuccess)
                        return set_error(WM_EHIP, "convert out", e), true;
                    src = stage_out;
                }
                if ((e = hipMemcpyAsync(pin_out, src, elems * 4, hipMemcpyDeviceToHost, s_copy)) != hipSuccess)
                    return set_error(WM_EHIP, "copy out", e), true;
                r->ev = get_event();
                if (!r->ev || (e = hipEventRecord(r->ev, s_copy)) != hipSuccess)
                    return set_error(WM_EHIP, "event", e), true;
                r->st = RQ_UNLOADING;
                unloading = true;
                progress = true;
                break;
            }
        }
        // admit the oldest queued request if a slot is free
        if (!loading && !queue.empty() && !free_slots.empty()) {
            Request *r = queue.front();
            queue.pop_front();
            r->slot = free_slots.back();
            free_slots.pop_back();
            r->st = RQ_LOADING;
            loading = true;
            lk.unlock();
            std::memcpy(pin_in, r->host_in.data(), elems * 4);
            lk.lock();
            void *dst = cfg.state_bf16 ? (void *)stage_in : slot_ptr(r->slot);
            if ((e = hipMemcpyAsync(dst, pin_in, elems * 4, hipMemcpyHostToDevice, s_copy)) != hipSuccess)
                return set_error(WM_EHIP, "copy in", e), true;
            if (cfg.state_bf16 &&
                (e = launch_convert(stage_in, false, slot_ptr(r->slot), true, elems, s_copy)) != hipSuccess)
                return set_error(WM_EHIP, "convert in", e), true;
            r->ev = get_event();
            if (!r->ev || (e = hipEventRecord(r->ev, s_copy)) != hipSuccess)
                return set_error(WM_EHIP, "event", e), true;
            progress = true;
        }
        // form the next batch (keep at most two queued on the compute stream)
        if (inflight.size() < 2) {
            std::vector<Request *> idle;
            for (auto &kv : reqs) {
                Request *r = kv.second;
                if (r->st == RQ_IDLE && r->cursor < (int)r->sched.size()) idle.push_back(r);
            }
            if (!idle.empty()) {
                std::sort(idle.begin(), idle.end(), [](Request *a, Request *b) { return a->id < b->id; });
                const int size = idle.front()->sched[idle.front()->cursor];
                Batch b;
                for (Request *r : idle) {
                    if ((int)b.reqs.size() >= cfg.max_batch) break;
                    if (r->sched[r->cursor] == size) b.reqs.push_back(r);
                }
                const int B = (int)b.reqs.size();
                const wm_processor *proc = size == 6 ? p6 : p1;
                int rc;
                // the step itself: eager, or the graph of its shape
                auto step = [&]() -> int {
                    float *x = cfg.state_bf16 ? batch : nullptr;
                    float *const *xs = cfg.state_bf16 ? nullptr : dptrs;
                    const std::pair<int, int> key{size, B};
                    if (!cfg.graphs || !warmed.count(key) || no_graph.count(key)) {
                        warmed.insert(key);
                        return run_step(ctx, proc, B, x, xs, s_comp);
                    }
                    auto it = graphs.find(key);
                    if (it == graphs.end()) {
                        // a shape whose capture fails runs eagerly from then on
                        // (nothing recorded during a capture has executed)
                        auto eager = [&]() {
                            (void)hipGetLastError();
                            no_graph.insert(key);
                            return run_step(ctx, proc, B, x, xs, s_comp);
                        };
                        hipGraph_t gr = nullptr;
                        hipGraphExec_t ex = nullptr;
                        if (hipStreamBeginCapture(s_comp, hipStreamCaptureModeThreadLocal) != hipSuccess) return eager();
                        const int rs = run_step(ctx, proc, B, x, xs, s_comp);
                        const hipError_t ee = hipStreamEndCapture(s_comp, &gr);
                        if (rs != WM_OK) {
                            if (gr) (void)hipGraphDestroy(gr);
                            return rs;
                        }
                        if (ee != hipSuccess) return eager();
                        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                        (void)hipGraphDestroy(gr);
                        if (e != hipSuccess) return eager();
                        it = graphs.emplace(key, ex).first;
                    }
                    e = hipGraphLaunch(it->second, s_comp);
                    return e == hipSuccess ? WM_OK : hip_fail(e, "hipGraphLaunch");
                };
                if (!cfg.state_bf16) {
                    // in place: the step's kernels address the slots through dptrs
                    // (the previous batch's step precedes this write on s_comp)
                    PtrList pl{};
                    for (int i = 0; i < B; ++i) pl.p[i] = (float *)slot_ptr(b.reqs[i]->slot);
                    if ((e = launch_set_ptrs(dptrs, pl, B, s_comp)) != hipSuccess)
                        return set_error(WM_EHIP, "slot pointers", e), true;
                    rc = step();
                } else {
                    for (int i = 0; i < B; ++i) {
                        e = launch_convert(slot_ptr(b.reqs[i]->slot), true, batch + (size_t)i * elems, false, elems,
                                           s_comp);
                        if (e != hipSuccess) return set_error(WM_EHIP, "gather", e), true;
                    }
                    rc = step();
                    for (int i = 0; rc == WM_OK && i < B; ++i) {
                        e = launch_convert(batch + (size_t)i * elems, false, slot_ptr(b.reqs[i]->slot), true, elems,
                                           s_comp);
                        if (e != hipSuccess) return set_error(WM_EHIP, "scatter", e), true;
                    }
                }
                if (rc != WM_OK) {
                    err_code = rc;
                    snprintf(err_msg, sizeof err_msg, "step: %s", wm_last_error());
                    return true;
                }
                b.ev = get_event();
                if (!b.ev || (e = hipEventRecord(b.ev, s_comp)) != hipSuccess)
                    return set_error(WM_EHIP, "event", e), true;
                for (Request *r : b.reqs) r->st = RQ_RUNNING;
                inflight.push_back(std::move(b));
                progress = true;
            }
        }
        return progress;
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            bool prog = false;
            if (err_code == WM_OK) {
                try {
                    prog = step_once(lk);
                } catch (const std::exception &ex) {   // host allocation inside an iteration
                    if (!lk.owns_lock()) lk.lock();
                    err_code = WM_ENOMEM;
                    snprintf(err_msg, sizeof err_msg, "scheduler: %s", ex.what());
                }
            }
            if (!prog) cv.wait_for(lk, std::chrono::microseconds(200));
        }
    }
};

extern "C" {

int wm_serve_create(wm_ctx *ctx, const wm_processor *p6, const wm_processor *p1, const wm_serve_cfg *cfg,
                    wm_server **out) {
    if (!out) return fail(WM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !p6 || !p1 || !cfg) return fail(WM_EINVAL, "NULL argument");
    if (std::memcmp(&p6->g, &p1->g, sizeof(wm_grid)) != 0 || p6->mlp != p1->mlp)
        return fail(WM_EINVAL, "processors have different grids");
    if (cfg->max_batch < 1 || cfg->max_batch > 64) return fail(WM_EINVAL, "max_batch must be 1..64");
    if (cfg->max_slots < 0 || cfg->max_slots > 1024) return fail(WM_EINVAL, "max_slots must be 0..1024");
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    wm_server *s = new (std::nothrow) wm_server();
    if (!s) return fail(WM_ENOMEM, "server allocation");
    s->p6 = p6;
    s->p1 = p1;
    s->cfg = *cfg;
    s->device = ctx->device;
    s->t0 = std::chrono::steady_clock::now();
    const wm_grid &g = p6->g;
    s->elems = (size_t)g.Z * g.Y * g.X * g.C;
    s->slot_bytes = ((s->elems * (cfg->state_bf16 ? 2 : 4)) + 255) & ~(size_t)255;
    auto cleanup = [&](int code) {
        wm_serve_destroy(s);
        return code;
    };
    int rc = wm_ctx_create(ctx->device, &s->ctx);
    if (rc) return cleanup(rc);
    rc = reserve_block_workspace(s->ctx, p6, cfg->max_batch);
    if (rc) return cleanup(rc);
    rc = reserve_block_workspace(s->ctx, p1, cfg->max_batch);
    if (rc) return cleanup(rc);
    if (cfg->state_bf16) {
        if ((e = hipMalloc(&s->batch, (size_t)cfg->max_batch * s->elems * 4)) != hipSuccess) {
            (void)hipGetLastError();
            return cleanup(fail(WM_ENOMEM, "batch buffer: %s", hipGetErrorString(e)));
        }
    } else if ((e = hipMalloc(&s->dptrs, 64 * sizeof(float *))) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(WM_ENOMEM, "slot pointer array: %s", hipGetErrorString(e)));
    }
    if ((e = hipHostMalloc((void **)&s->pin_in, s->elems * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s->pin_out, s->elems * 4, hipHostMallocDefault)) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(WM_ENOMEM, "pinned staging: %s", hipGetErrorString(e)));
    }
    if (cfg->state_bf16) {
        if ((e = hipMalloc(&s->stage_in, s->elems * 4)) != hipSuccess ||
            (e = hipMalloc(&s->stage_out, s->elems * 4)) != hipSuccess) {
            (void)hipGetLastError();
            return cleanup(fail(WM_ENOMEM, "staging buffers: %s", hipGetErrorString(e)));
        }
    }
    size_t free_b = 0, total_b = 0;
    if ((e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) return cleanup(hip_fail(e, "hipMemGetInfo"));
    size_t budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : free_b / 4 * 3;
    if (budget > free_b) budget = free_b;
    int n = (int)std::min<size_t>(budget / s->slot_bytes, 1024);
    if (cfg->max_slots > 0) n = std::min(n, cfg->max_slots);
    if (n < 1) return cleanup(fail(WM_ENOMEM, "HBM budget holds no state slot (%zu bytes per slot)", s->slot_bytes));
    if ((e = hipMalloc(&s->slot_mem, (size_t)n * s->slot_bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(WM_ENOMEM, "%d state slots: %s", n, hipGetErrorString(e)));
    }
    s->nslots = n;
    for (int i = n - 1; i >= 0; --i) s->free_slots.push_back(i);
    if ((e = hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s->s_copy, hipStreamNonBlocking)) != hipSuccess)
        return cleanup(hip_fail(e, "hipStreamCreate"));
    try {
        s->th = std::thread([s] { s->loop(); });
    } catch (...) {
        return cleanup(fail(WM_ENOMEM, "scheduler thread"));
    }
    *out = s;
    return WM_OK;
}

int wm_serve_submit(wm_server *s, const float *x0_host, int lead_hours, uint64_t *id_out) {
    if (!s || !x0_host) return fail(WM_EINVAL, "NULL argument");
    if (lead_hours < 0) return fail(WM_EINVAL, "negative lead time %d", lead_hours);
    const double t_submit = now_s(s->t0);
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(WM_ENOMEM, "request allocation");
    try {
        r->host_in.assign(x0_host, x0_host + s->elems);
        r->sched.resize(greedy_schedule(lead_hours, nullptr, 0));
    } catch (...) {
        delete r;
        return fail(WM_ENOMEM, "request state copy or schedule");
    }
    r->lead = lead_hours;
    greedy_schedule(lead_hours, r->sched.data(), (int)r->sched.size());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        r->stats.id = r->id;
        r->stats.lead_hours = lead_hours;
        r->stats.t_submit = t_submit;
        s->reqs[r->id] = r;
        s->queue.push_back(r);
    }
    s->cv.notify_one();
    if (id_out) *id_out = r->id;
    return WM_OK;
}

int wm_serve_poll(wm_server *s, uint64_t id, float *out_host, wm_req_stats *st) {
    if (!s) return fail(WM_EINVAL, "server is NULL");
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->err_code != WM_OK) return fail(s->err_code, "server failed: %s", s->err_msg);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return fail(WM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
        if (it->second->st != RQ_DONE) return WM_EAGAIN;
        r = it->second;
        s->reqs.erase(it);
    }
    if (out_host) std::memcpy(out_host, r->host_out.data(), s->elems * 4);
    if (st) *st = r->stats;
    delete r;
    return WM_OK;
}

int wm_serve_status(wm_server *s, int *queued, int *running, int *done, int *slots) {
    if (!s) return fail(WM_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    int q = 0, ru = 0, d = 0;
    for (auto &kv : s->reqs) {
        const ReqState st = kv.second->st;
        if (st == RQ_QUEUED) ++q;
        else if (st == RQ_DONE) ++d;
        else ++ru;
    }
    if (queued) *queued = q;
    if (running) *running = ru;
    if (done) *done = d;
    if (slots) *slots = s->nslots;
    return s->err_code;
}

void wm_serve_destroy(wm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->device);
    if (s->s_comp) (void)hipStreamSynchronize(s->s_comp);
    if (s->s_copy) (void)hipStreamSynchronize(s->s_copy);
    for (auto &kv : s->reqs) {
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    for (auto &b : s->inflight)
        if (b.ev) (void)hipEventDestroy(b.ev);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->s_comp) (void)hipStreamDestroy(s->s_comp);
    if (s->s_copy) (void)hipStreamDestroy(s->s_copy);
    if (s->slot_mem) (void)hipFree(s->slot_mem);
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    if (s->batch) (void)hipFree(s->batch);
    if (s->dptrs) (void)hipFree(s->dptrs);
    if (s->stage_in) (void)hipFree(s->stage_in);
    if (s->stage_out) (void)hipFree(s->stage_out);
    if (s->pin_in) (void)hipHostFree(s->pin_in);
    if (s->pin_out) (void)hipHostFree(s->pin_out);
    if (s->ctx) wm_ctx_destroy(s->ctx);
    delete s;
}

}  // extern "C"
