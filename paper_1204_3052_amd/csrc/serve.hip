// Request server: an engine thread that admits matrix-power requests by
// device-memory budget, batches small ones into ragged persistent launches
// while others run (continuous batching), overlaps large ones on several
// streams, and reports per-request timestamps.  The policy (serve_policy.h)
// is shared with mpow_srv_simulate, which runs it against a simulated
// executor on the CPU.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "mpow_internal.h"
#include "serve_policy.h"

using namespace mpow;
using mpow::serve::Launch;
using mpow::serve::Req;
using mpow::serve::Scheduler;

namespace {

constexpr int kStreamDepth = 2;  // requests in flight per stream

double gemm_work(int n, int64_t p) {
    const double nn = (double)n;
    return (double)(mpow_gemm_count(p) + 1) * nn * nn * nn;
}

bool batched_route(int n, int mode, int max_batch) {
    return max_batch > 0 && mode == MPOW_FP32 && n <= kBatchMaxN;
}

}  // namespace

struct mpow_srv {
    int device = 0, max_n = 0, n_streams = 0, max_batch = 0;
    size_t budget = 0;
    char *arena = nullptr;
    char *batch_dev = nullptr;
    std::vector<hipStream_t> streams;
    hipStream_t batch_stream = nullptr;
    BatchContext batch;
    Scheduler *sched = nullptr;

    std::thread thr;
    std::mutex mu;
    std::condition_variable cv, cv_idle;
    std::deque<Req *> inbox;
    std::deque<mpow_completion> done;
    uint64_t next_id = 1, submitted = 0, completed = 0, rejected = 0;
    size_t outstanding = 0;
    bool stop = false;
    int last_error = 0;
    std::chrono::steady_clock::time_point t0;

    // engine-thread state
    struct Flight {
        Req *r;
        hipEvent_t ev;
    };
    std::vector<Flight> plain;
    struct BatchFlight {
        std::vector<Req *> reqs;
        hipEvent_t ev;
    };
    std::deque<BatchFlight> batches;  // at most 2, completing in order
    std::vector<hipEvent_t> ev_pool;
    size_t arena_in_use = 0, arena_peak = 0;  // mirrored under mu for stats
    int queued = 0, in_flight = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    hipEvent_t take_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void complete(Req *r, int status, int route) {
        r->t_end = now();
        mpow_completion c;
        c.id = r->id;
        c.status = status;
        c.route = route;
        c.t_submit = r->t_submit;
        c.t_start = r->t_start;
        c.t_end = r->t_end;
        std::lock_guard<std::mutex> lk(mu);
        done.push_back(c);
        completed += 1;
        outstanding -= 1;
        if (outstanding == 0) cv_idle.notify_all();
        delete r;
    }

    void launch(const Launch &l) {
        const double t = now();
        if (l.batched) {
            const int count = (int)l.reqs.size();
            std::vector<const float *> A(count);
            std::vector<int> n(count);
            std::vector<int64_t> p(count);
            std::vector<float *> out(count);
            std::vector<double *> sc(count);
            for (int i = 0; i < count; ++i) {
                Req *r = l.reqs[i];
                r->t_start = t;
                A[i] = r->A;
                n[i] = r->n;
                p[i] = r->p;
                out[i] = r->out;
                sc[i] = r->scale;
            }
            hipEvent_t ev = nullptr;
            const hipError_t e = batch_enqueue(&batch, count, A.data(), n.data(), p.data(),
                                               out.data(), sc.data(), batch_stream, false, &ev);
            if (e != hipSuccess) {
                last_error = (int)e;
                (void)hipGetLastError();
                for (Req *r : l.reqs) complete(r, MPOW_ERR_DEVICE, 1);
                return;
            }
            batches.push_back({l.reqs, ev});
            return;
        }
        Req *r = l.reqs[0];
        r->t_start = t;
        Workspace ws;
        workspace_carve(arena + r->arena_off, r->n, r->mode, &ws);
        hipStream_t s = streams[r->stream];
        hipEvent_t ev = take_event();
        hipError_t e = ev ? enqueue_power(ws, r->A, r->n, r->p, r->out, r->scale, s, nullptr)
                          : hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipEventRecord(ev, s);
        if (e != hipSuccess) {
            last_error = (int)e;
            (void)hipGetLastError();
            if (ev) ev_pool.push_back(ev);
            sched->finish_plain(r);
            complete(r, MPOW_ERR_DEVICE, 0);
            return;
        }
        plain.push_back({r, ev});
    }

    void engine() {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<Req *> incoming;
            {
                std::lock_guard<std::mutex> lk(mu);
                incoming.assign(inbox.begin(), inbox.end());
                inbox.clear();
                if (stop && outstanding == 0) break;
            }
            bool progress = !incoming.empty();
            for (Req *r : incoming) (void)sched->submit(r);  // fit was checked at submission

            for (size_t i = 0; i < plain.size();) {
                const hipError_t q = hipEventQuery(plain[i].ev);
                if (q == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                Req *r = plain[i].r;
                ev_pool.push_back(plain[i].ev);
                plain[i] = plain.back();
                plain.pop_back();
                sched->finish_plain(r);
                if (q != hipSuccess) {
                    last_error = (int)q;
                    (void)hipGetLastError();
                }
                complete(r, q == hipSuccess ? MPOW_SUCCESS : MPOW_ERR_DEVICE, 0);
                progress = true;
            }
            while (!batches.empty()) {
                const hipError_t q = hipEventQuery(batches.front().ev);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    last_error = (int)q;
                    (void)hipGetLastError();
                }
                for (Req *r : batches.front().reqs)
                    complete(r, q == hipSuccess ? MPOW_SUCCESS : MPOW_ERR_DEVICE, 1);
                batches.pop_front();
                progress = true;
            }
            // a second batch may be queued behind a running one: it is
            // prepared while the first runs and starts as soon as it ends
            const std::vector<Launch> ls = sched->next(batches.size() < 2);
            for (const Launch &l : ls) launch(l);
            progress = progress || !ls.empty();
            {
                std::unique_lock<std::mutex> lk(mu);
                arena_in_use = sched->arena().in_use();
                arena_peak = sched->arena().peak();
                queued = (int)sched->queued();
                in_flight = (int)plain.size();
                for (const BatchFlight &b : batches) in_flight += (int)b.reqs.size();
                if (!progress && inbox.empty() && !stop)
                    cv.wait_for(lk, std::chrono::microseconds(
                                        (plain.empty() && batches.empty()) ? 2000 : 20));
            }
        }
    }
};

extern "C" {

mpow_status mpow_srv_create(mpow_srv_t *out_srv, int device, int max_n, size_t hbm_budget,
                            int n_streams, int max_batch, uint32_t flags) {
    if (!out_srv) return MPOW_ERR_INVALID;
    *out_srv = nullptr;
    if (max_n < 1 || n_streams < 1 || n_streams > 64 || max_batch < 0 || flags != 0 ||
        hbm_budget < serve::Arena::kGranule)
        return MPOW_ERR_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return MPOW_ERR_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return MPOW_ERR_DEVICE;
    mpow_srv *srv = new (std::nothrow) mpow_srv();
    if (!srv) return MPOW_ERR_NOMEM;
    srv->device = device;
    srv->max_n = max_n;
    srv->n_streams = n_streams;
    srv->max_batch = max_batch;
    srv->budget = hbm_budget;
    mpow_status st = MPOW_SUCCESS;
    if (hipMalloc((void **)&srv->arena, hbm_budget) != hipSuccess) st = MPOW_ERR_NOMEM;
    if (st == MPOW_SUCCESS && max_batch > 0) {
        const int bmax = max_n < kBatchMaxN ? max_n : kBatchMaxN;
        int workers[kBatchInstances] = {};
        const bool ok = batch_workers_for(device, workers);
        const int wmax = batch_scratch_workers(workers);
        if (!ok ||
            hipMalloc((void **)&srv->batch_dev, batch_device_bytes(max_batch, bmax, wmax)) != hipSuccess ||
            batch_context_init(&srv->batch, srv->batch_dev, max_batch, bmax, workers) != hipSuccess)
            st = MPOW_ERR_NOMEM;
    }
    for (int i = 0; st == MPOW_SUCCESS && i < n_streams; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) st = MPOW_ERR_DEVICE;
        else srv->streams.push_back(s);
    }
    if (st == MPOW_SUCCESS && hipStreamCreateWithFlags(&srv->batch_stream, hipStreamNonBlocking) != hipSuccess)
        st = MPOW_ERR_DEVICE;
    if (st != MPOW_SUCCESS) {
        (void)hipGetLastError();
        for (auto s : srv->streams) (void)hipStreamDestroy(s);
        if (srv->batch_stream) (void)hipStreamDestroy(srv->batch_stream);
        batch_context_release(&srv->batch);
        if (srv->batch_dev) (void)hipFree(srv->batch_dev);
        if (srv->arena) (void)hipFree(srv->arena);
        delete srv;
        return st;
    }
    srv->sched = new Scheduler(hbm_budget, n_streams, kStreamDepth, max_batch > 0 ? max_batch : 1);
    srv->t0 = std::chrono::steady_clock::now();
    srv->thr = std::thread([srv] { srv->engine(); });
    *out_srv = srv;
    return MPOW_SUCCESS;
}

mpow_status mpow_srv_submit(mpow_srv_t srv, const float *A, int n, int64_t p, int mode, float *out,
                            double *log2_scale, uint64_t *id) {
    if (!srv || !A || !out || n < 1 || n > srv->max_n || p < 0 || mode < 0 || mode > MPOW_BF16X6)
        return MPOW_ERR_INVALID;
    if (((uintptr_t)A & 3) || ((uintptr_t)out & 3) || ((uintptr_t)log2_scale & 7))
        return MPOW_ERR_INVALID;
    const size_t bytes = (size_t)n * n * sizeof(float);
    const uintptr_t a = (uintptr_t)A, o = (uintptr_t)out;
    if (a != o && a < o + bytes && o < a + bytes) return MPOW_ERR_INVALID;
    Req *r = new (std::nothrow) Req();
    if (!r) return MPOW_ERR_NOMEM;
    r->n = n;
    r->p = p;
    r->mode = mode;
    r->A = A;
    r->out = out;
    r->scale = log2_scale;
    r->batched = batched_route(n, mode, srv->max_batch);
    r->ws_bytes = r->batched ? 0 : workspace_bytes(n, mode);
    r->work = gemm_work(n, p);
    if (!r->batched && serve::Arena::granules(r->ws_bytes) > srv->sched->arena().capacity()) {
        delete r;
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->rejected += 1;
        return MPOW_ERR_BUDGET;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            delete r;
            return MPOW_ERR_INVALID;
        }
        r->id = srv->next_id++;
        r->t_submit = srv->now();
        if (id) *id = r->id;
        srv->inbox.push_back(r);
        srv->submitted += 1;
        srv->outstanding += 1;
    }
    srv->cv.notify_one();
    return MPOW_SUCCESS;
}

int mpow_srv_poll(mpow_srv_t srv, mpow_completion *out, int max) {
    if (!srv || (!out && max > 0) || max < 0) return -1;
    std::lock_guard<std::mutex> lk(srv->mu);
    int k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    return k;
}

mpow_status mpow_srv_wait_idle(mpow_srv_t srv, double timeout_s) {
    if (!srv) return MPOW_ERR_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    const bool ok = srv->cv_idle.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                          [srv] { return srv->outstanding == 0; });
    return ok ? MPOW_SUCCESS : MPOW_ERR_TIMEOUT;
}

mpow_status mpow_srv_stats(mpow_srv_t srv, mpow_srv_stats_t *st) {
    if (!srv || !st) return MPOW_ERR_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    st->submitted = srv->submitted;
    st->completed = srv->completed;
    st->rejected = srv->rejected;
    st->queued = srv->queued + (int)srv->inbox.size();
    st->in_flight = srv->in_flight;
    st->arena_capacity = srv->sched->arena().capacity();
    st->arena_in_use = srv->arena_in_use;
    st->arena_peak = srv->arena_peak;
    st->last_device_error = srv->last_error;
    return MPOW_SUCCESS;
}

mpow_status mpow_srv_destroy(mpow_srv_t srv) {
    if (!srv) return MPOW_SUCCESS;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->thr.joinable()) srv->thr.join();
    (void)hipSetDevice(srv->device);
    for (auto s : srv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    if (srv->batch_stream) {
        (void)hipStreamSynchronize(srv->batch_stream);
        (void)hipStreamDestroy(srv->batch_stream);
    }
    for (auto e : srv->ev_pool) (void)hipEventDestroy(e);
    batch_context_release(&srv->batch);
    if (srv->batch_dev) (void)hipFree(srv->batch_dev);
    if (srv->arena) (void)hipFree(srv->arena);
    delete srv->sched;
    delete srv;
    return MPOW_SUCCESS;
}

// ---------------------------------------------------------------- simulation

mpow_status mpow_srv_simulate(const mpow_sim_config *cfg, const mpow_sim_request *reqs, int count,
                              mpow_sim_result *results, size_t *peak_bytes) {
    if (!cfg || count < 0 || (count > 0 && (!reqs || !results)) || cfg->n_streams < 1 ||
        cfg->depth < 1 || cfg->batch_cap < 0 || !(cfg->plain_flops > 0) ||
        !(cfg->batch_flops > 0) || cfg->launch_overhead_s < 0)
        return MPOW_ERR_INVALID;
    for (int i = 0; i < count; ++i)
        if (reqs[i].n < 1 || reqs[i].p < 0 || reqs[i].mode < 0 || reqs[i].mode > MPOW_BF16X6 ||
            (i > 0 && reqs[i].t_arrive < reqs[i - 1].t_arrive))
            return MPOW_ERR_INVALID;

    Scheduler sched(cfg->hbm_budget, cfg->n_streams, cfg->depth,
                    cfg->batch_cap > 0 ? cfg->batch_cap : 1);
    std::vector<Req> rs(count);
    std::vector<double> stream_free(cfg->n_streams, 0.0);
    struct Fl {
        Req *r;
        double end;
    };
    std::vector<Fl> plain;
    struct Bt {
        std::vector<Req *> reqs;
        double end;
    };
    std::deque<Bt> batches;  // at most 2 in flight, run one after another
    int next = 0;
    double t = 0.0;
    int done = 0;
    for (int i = 0; i < count; ++i) {
        Req &r = rs[i];
        r.id = (uint64_t)i;
        r.n = reqs[i].n;
        r.p = reqs[i].p;
        r.mode = reqs[i].mode;
        r.batched = batched_route(r.n, r.mode, cfg->batch_cap);
        r.ws_bytes = r.batched ? 0 : workspace_bytes(r.n, r.mode);
        r.work = gemm_work(r.n, r.p);
        results[i].status = MPOW_SUCCESS;
        results[i].route = r.batched ? 1 : 0;
        results[i].stream = -1;
        results[i].t_admit = results[i].t_start = results[i].t_end = -1.0;
    }
    auto flops = [](const Req &r) { return 2.0 * (double)mpow_gemm_count(r.p) * r.n * (double)r.n * r.n; };
    while (done < count) {
        // next event time
        double te = 1e300;
        if (next < count) te = std::min(te, reqs[next].t_arrive);
        for (const Fl &f : plain) te = std::min(te, f.end);
        if (!batches.empty()) te = std::min(te, batches.front().end);
        if (te == 1e300) return MPOW_ERR_INVALID;  // nothing can progress: policy stuck
        t = std::max(t, te);
        for (size_t i = 0; i < plain.size();) {
            if (plain[i].end <= t) {
                sched.finish_plain(plain[i].r);
                results[plain[i].r->id].t_end = plain[i].end;
                ++done;
                plain[i] = plain.back();
                plain.pop_back();
            } else {
                ++i;
            }
        }
        while (!batches.empty() && batches.front().end <= t) {
            for (Req *r : batches.front().reqs) {
                results[r->id].t_end = batches.front().end;
                ++done;
            }
            batches.pop_front();
        }
        while (next < count && reqs[next].t_arrive <= t) {
            Req *r = &rs[next];
            r->t_submit = reqs[next].t_arrive;
            if (!sched.submit(r)) {
                results[next].status = MPOW_ERR_BUDGET;
                ++done;
            }
            ++next;
        }
        for (const Launch &l : sched.next(batches.size() < 2)) {
            if (l.batched) {
                double f = 0.0;
                for (Req *r : l.reqs) f += flops(*r);
                const double start = batches.empty() ? t : std::max(t, batches.back().end);
                const double end = start + cfg->launch_overhead_s + f / cfg->batch_flops;
                for (Req *r : l.reqs) {
                    results[r->id].t_admit = t;
                    results[r->id].t_start = start;
                }
                batches.push_back({l.reqs, end});
            } else {
                Req *r = l.reqs[0];
                const double start = std::max(t, stream_free[l.stream]);
                const double end = start + cfg->launch_overhead_s + flops(*r) / cfg->plain_flops;
                stream_free[l.stream] = end;
                results[r->id].t_admit = t;
                results[r->id].t_start = start;
                results[r->id].stream = l.stream;
                plain.push_back({r, end});
            }
        }
        if (sched.arena().in_use() > sched.arena().capacity()) return MPOW_ERR_BUDGET;
    }
    if (peak_bytes) *peak_bytes = sched.arena().peak();
    return MPOW_SUCCESS;
}

}  // extern "C"
