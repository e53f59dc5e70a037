// Serving layer: resident systems, admission by device-memory footprint and
// continuous batching of shift requests (shs_server_* in shiftsolve.h).
//
// Worker threads each own a HIP stream.  A free worker takes the oldest
// waiting request; if it is FP64 it also takes every other waiting FP64
// request that still fits in the memory budget (any system, any n and m)
// and runs all their shifts in one launch of the work-item kernel, then
// forms G and the backward error per request.  A mixed-precision request is
// run alone with shs_solve.  Requests submitted meanwhile wait in the queue
// and are admitted by the next free worker, so work from different requests
// overlaps on the device through the workers' streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "handle.hpp"
#include "serve.hpp"

using namespace shs;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t id = 0;
    int32_t sys = 0;
    int64_t s = 0;
    std::vector<double> shifts;   // host copy, 2 s doubles
    int mode = SHS_MODE_FP64, outputs = 0;
    double *X = nullptr, *G = nullptr, *eta = nullptr;
    int64_t ldx = 0, ldg = 0;
    int32_t *status = nullptr;
    size_t footprint = 0;
    bool alone = false;           // runs as its own shs_solve (mixed mode, or blocked FP64)
    Clock::time_point t_submit, t_done;
    int state = 0;                // 0 queued, 1 running, 2 done, 3 failed
    int error = 0;
};

// Device bytes of an FP64 batch entry: reflector store + Y per shift, the
// shifts, per-column maxima, items and a claimed-items counter.
size_t fp64_item_bytes(const shs_handle *h, int64_t s)
{
    SweepGeometry g;
    sweep_geometry(false, (int)h->m, false, &g);
    const size_t refl = sizeof(double) * (size_t)g.refl_stride((int)h->n) * (size_t)s;
    const size_t y = sizeof(double) * 2 * (size_t)(h->m * h->m) * (size_t)s;
    const size_t xw = sizeof(double) * 2 * (size_t)(h->n * h->m) * (size_t)s;   // X when not requested
    const size_t xt = sizeof(double) * (size_t)residual_pack_rows(h->n) * (size_t)residual_pack_ld(h->m * s);
    const size_t misc = 2 * sizeof(double) * (size_t)s + 2 * sizeof(unsigned long long) * (size_t)(h->m * s) +
                        sizeof(ServeItem) * (size_t)s + 5 * 256;
    return refl + y + xw + xt + misc;
}

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct shs_server {
    int device = 0;
    size_t budget = 0;
    int max_batch = 64;
    double blocked_flops = 7.7e8;
    std::vector<shs_handle *> systems;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::unordered_map<int64_t, std::shared_ptr<Request>> reqs;
    int64_t next_id = 1;
    size_t in_use = 0, peak = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, running = 0, solves = 0, batches = 0, max_sys = 0;
    std::vector<double> lat_ms;
    bool any = false;
    Clock::time_point t_first, t_last;

    void worker(int wid);
    int run_fp64_batch(std::vector<std::shared_ptr<Request>> &batch, hipStream_t st);
    int run_alone(Request &r, hipStream_t st);
};

int shs_server::run_fp64_batch(std::vector<std::shared_ptr<Request>> &batch, hipStream_t st)
{
    // workspace layout: per request its scratch, then the item list and counter
    size_t total = 0;
    struct Off { size_t refl, y, xw, shifts, resmax, xmax, xt; };
    std::vector<Off> offs(batch.size());
    int64_t nitems = 0;
    for (size_t b = 0; b < batch.size(); ++b) {
        Request &r = *batch[b];
        shs_handle *h = systems[r.sys];
        SweepGeometry g;
        sweep_geometry(false, (int)h->m, false, &g);
        auto take = [&](size_t bytes) { size_t o = total; total += al256(bytes); return o; };
        offs[b].refl = take(sizeof(double) * (size_t)g.refl_stride((int)h->n) * r.s);
        offs[b].y = take(sizeof(double) * 2 * (size_t)(h->m * h->m) * r.s);
        offs[b].xw = (r.outputs & SHS_OUT_X) ? 0 : take(sizeof(double) * 2 * (size_t)(h->n * h->m) * r.s);
        offs[b].shifts = take(sizeof(double) * 2 * r.s);
        offs[b].resmax = take(sizeof(unsigned long long) * (size_t)(h->m * r.s));
        offs[b].xmax = take(sizeof(unsigned long long) * (size_t)(h->m * r.s));
        offs[b].xt = take(sizeof(double) * (size_t)residual_pack_rows(h->n) * (size_t)residual_pack_ld(h->m * r.s));
        nitems += r.s;
    }
    const size_t items_off = total;
    total += al256(sizeof(ServeItem) * (size_t)nitems);
    const size_t counter_off = total;
    total += 256;
    char *work = nullptr;
    hipError_t e = hipMallocAsync((void **)&work, total, st);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SHS_ERR_NOMEM : SHS_ERR_HIP;

    std::vector<ServeItem> items;
    items.reserve(nitems);
    for (size_t b = 0; b < batch.size(); ++b) {
        Request &r = *batch[b];
        shs_handle *h = systems[r.sys];
        SweepGeometry g;
        sweep_geometry(false, (int)h->m, false, &g);
        const int64_t stride = g.refl_stride((int)h->n);
        double *X = (r.outputs & SHS_OUT_X) ? r.X : (double *)(work + offs[b].xw);
        const int64_t ldx = (r.outputs & SHS_OUT_X) ? r.ldx : h->n;
        for (int64_t j = 0; j < r.s; ++j) {
            ServeItem it;
            it.H = h->H;
            it.ldh = h->ldh;
            it.Rtop = h->Rtop;
            it.refl = (double *)(work + offs[b].refl) + j * stride;
            it.Y = (double *)(work + offs[b].y) + j * 2 * h->m * h->m;
            it.X = X + j * h->m * ldx * 2;
            it.ldx = ldx;
            it.status = r.status + j;
            it.sr = r.shifts[2 * j];
            it.si = r.shifts[2 * j + 1];
            it.n = (int)h->n;
            it.m = (int)h->m;
            items.push_back(it);
        }
    }
    // largest shifts first, so the tail of the launch is short
    std::stable_sort(items.begin(), items.end(), [](const ServeItem &a, const ServeItem &b) {
        return (double)a.n * a.n * (8 * a.m + 2) > (double)b.n * b.n * (8 * b.m + 2);
    });
    if (e == hipSuccess)
        e = hipMemcpyAsync(work + items_off, items.data(), sizeof(ServeItem) * items.size(), hipMemcpyHostToDevice, st);
    for (size_t b = 0; b < batch.size() && e == hipSuccess; ++b)
        e = hipMemcpyAsync(work + offs[b].shifts, batch[b]->shifts.data(), sizeof(double) * 2 * batch[b]->s,
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(work + counter_off, 0, sizeof(unsigned), st);
    if (e == hipSuccess)
        e = launch_serve((const ServeItem *)(work + items_off), (int)nitems, (unsigned *)(work + counter_off), st);
    for (size_t b = 0; b < batch.size() && e == hipSuccess; ++b) {
        Request &r = *batch[b];
        shs_handle *h = systems[r.sys];
        double *X = (r.outputs & SHS_OUT_X) ? r.X : (double *)(work + offs[b].xw);
        const int64_t ldx = (r.outputs & SHS_OUT_X) ? r.ldx : h->n;
        if ((r.outputs & SHS_OUT_G) && h->p > 0) e = g_eval(h, r.s, X, ldx, r.G, r.ldg, st);
        if (e == hipSuccess && (r.outputs & SHS_OUT_ETA))
            e = certify(h, r.s, nullptr, (const double *)(work + offs[b].shifts), X, ldx, nullptr,
                        (unsigned long long *)(work + offs[b].resmax), (unsigned long long *)(work + offs[b].xmax),
                        r.eta, r.status, r.s, (double *)(work + offs[b].xt), st);
    }
    hipError_t e2 = hipFreeAsync(work, st);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? 0 : (e == hipErrorOutOfMemory ? SHS_ERR_NOMEM : SHS_ERR_HIP);
}

int shs_server::run_alone(Request &r, hipStream_t st)
{
    shs_handle *h = systems[r.sys];
    double *dsh = nullptr;
    hipError_t e = hipMallocAsync((void **)&dsh, sizeof(double) * 2 * r.s, st);
    if (e != hipSuccess) return SHS_ERR_NOMEM;
    e = hipMemcpyAsync(dsh, r.shifts.data(), sizeof(double) * 2 * r.s, hipMemcpyHostToDevice, st);
    int rc = e == hipSuccess ? 0 : SHS_ERR_HIP;
    if (rc == 0)
        rc = shs_solve(h, r.s, dsh, r.mode, r.outputs, 1e-13, 5, nullptr, 0, r.X, r.ldx, r.G, r.ldg, r.eta, r.status,
                       st);
    hipFreeAsync(dsh, st);
    e = hipStreamSynchronize(st);
    if (rc == 0 && e != hipSuccess) rc = SHS_ERR_HIP;
    return rc;
}

void shs_server::worker(int wid)
{
    hipSetDevice(device);
    hipStream_t st = streams[wid];
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        size_t fp = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop && pending.empty()) return;
                if (!pending.empty()) {
                    auto head = pending.front();
                    if (in_use + head->footprint <= budget) {
                        pending.pop_front();
                        batch.push_back(head);
                        fp = head->footprint;
                        if (!head->alone) {
                            // every other waiting work-item request that fits joins the launch
                            for (auto it = pending.begin(); it != pending.end() && (int)batch.size() < max_batch;) {
                                if (!(*it)->alone && in_use + fp + (*it)->footprint <= budget) {
                                    fp += (*it)->footprint;
                                    batch.push_back(*it);
                                    it = pending.erase(it);
                                } else {
                                    ++it;
                                }
                            }
                        }
                        break;
                    }
                }
                cv_work.wait(lk);
            }
            in_use += fp;
            peak = std::max(peak, in_use);
            running += (int64_t)batch.size();
            for (auto &r : batch) r->state = 1;
            if (!batch[0]->alone) {
                ++batches;
                std::vector<int32_t> sy;
                for (auto &r : batch) sy.push_back(r->sys);
                std::sort(sy.begin(), sy.end());
                max_sys = std::max<int64_t>(max_sys, std::unique(sy.begin(), sy.end()) - sy.begin());
            }
        }
        const int rc = batch[0]->alone ? run_alone(*batch[0], st) : run_fp64_batch(batch, st);
        const auto now = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= fp;
            running -= (int64_t)batch.size();
            for (auto &r : batch) {
                r->t_done = now;
                r->error = rc;
                r->state = rc == 0 ? 2 : 3;
                if (rc == 0) {
                    ++completed;
                    solves += r->s;
                    lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
                } else {
                    ++failed;
                }
            }
            t_last = now;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

extern "C" {

int shs_server_create(const shs_server_config *cfg, shs_server **out)
{
    if (!cfg) return -1;
    if (!out) return -2;
    if (cfg->abi_version != SHS_ABI_VERSION || cfg->streams < 1 || cfg->streams > 16 || cfg->budget_bytes <= 0 ||
        cfg->max_batch < 1)
        return -1;
    *out = nullptr;
    auto *srv = new (std::nothrow) shs_server();
    if (!srv) return SHS_ERR_NOMEM;
    hipGetDevice(&srv->device);
    srv->budget = (size_t)cfg->budget_bytes;
    srv->max_batch = cfg->max_batch;
    if (cfg->blocked_flops != 0.0) srv->blocked_flops = cfg->blocked_flops;
    for (int i = 0; i < cfg->streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t s2 : srv->streams) hipStreamDestroy(s2);
            delete srv;
            return SHS_ERR_HIP;
        }
        srv->streams.push_back(st);
    }
    for (int i = 0; i < cfg->streams; ++i) srv->workers.emplace_back(&shs_server::worker, srv, i);
    *out = srv;
    return 0;
}

int shs_server_register(shs_server *srv, shs_handle *h, int32_t *sys_id)
{
    if (!srv) return -1;
    if (!h) return -2;
    if (!sys_id) return -3;
    if (h->device != srv->device) return -2;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->systems.push_back(h);
    *sys_id = (int32_t)srv->systems.size() - 1;
    return 0;
}

int shs_server_submit(shs_server *srv, int32_t sys_id, int64_t s, const double *shifts_host, int mode, int outputs,
                      double *X, int64_t ldx, double *G, int64_t ldg, double *eta, int32_t *status, int64_t *req_id)
{
    if (!srv) return -1;
    if (!req_id) return -13;
    shs_handle *h = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (sys_id < 0 || sys_id >= (int32_t)srv->systems.size()) return SHS_ERR_NOTFOUND;
        h = srv->systems[sys_id];
    }
    if (s < 1 || s > INT32_MAX / 64) return -3;
    if (!shifts_host) return -4;
    if (mode != SHS_MODE_FP64 && mode != SHS_MODE_FP32_REFINE) return -5;
    if (!(outputs & (SHS_OUT_X | SHS_OUT_G))) return -6;
    if ((outputs & SHS_OUT_X) && (!X || ldx < h->n)) return -7;
    if ((outputs & SHS_OUT_G) && h->p > 0 && (!G || ldg < h->p)) return -9;
    if (((outputs & SHS_OUT_ETA) || mode == SHS_MODE_FP32_REFINE) && !eta) return -11;
    if (!status) return -12;
    auto r = std::make_shared<Request>();
    r->sys = sys_id;
    r->s = s;
    r->shifts.assign(shifts_host, shifts_host + 2 * s);
    r->mode = mode;
    r->outputs = outputs;
    r->X = X;
    r->ldx = ldx;
    r->G = G;
    r->ldg = ldg;
    r->eta = eta;
    r->status = status;
    // one shift of a big system is too much for one wavefront of the
    // work-item kernel: such FP64 requests take the blocked solve
    const double shift_flops = (8.0 * h->m + 2.0) * (double)h->n * (double)h->n;
    r->alone = mode != SHS_MODE_FP64 || (srv->blocked_flops >= 0.0 && shift_flops > srv->blocked_flops);
    if (!r->alone) {
        r->footprint = fp64_item_bytes(h, s);
    } else {
        size_t b = 0;
        const int rc = shs_solve_workspace(h, s, mode, outputs, &b);
        if (rc != 0) return rc;
        r->footprint = b + sizeof(double) * 2 * s;
    }
    if (r->footprint > srv->budget) return SHS_ERR_NOMEM;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        r->id = srv->next_id++;
        srv->reqs[r->id] = r;
        srv->pending.push_back(r);
        ++srv->submitted;
        if (!srv->any) {
            srv->any = true;
            srv->t_first = r->t_submit;
        }
        *req_id = r->id;
    }
    srv->cv_work.notify_one();
    return 0;
}

int shs_server_poll(shs_server *srv, int64_t req_id, int *state)
{
    if (!srv) return -1;
    if (!state) return -3;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return SHS_ERR_NOTFOUND;
    *state = it->second->state;
    return 0;
}

int shs_server_wait(shs_server *srv, int64_t req_id, double timeout_ms)
{
    if (!srv) return -1;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return SHS_ERR_NOTFOUND;
    auto r = it->second;
    auto done = [&] { return r->state >= 2; };
    if (timeout_ms < 0) {
        srv->cv_done.wait(lk, done);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done)) {
        return SHS_ERR_TIMEOUT;
    }
    return r->state == 2 ? 0 : r->error;
}

int shs_server_latency(shs_server *srv, int64_t req_id, double *ms)
{
    if (!srv) return -1;
    if (!ms) return -3;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return SHS_ERR_NOTFOUND;
    if (it->second->state < 2) return SHS_ERR_BUSY;
    *ms = std::chrono::duration<double, std::milli>(it->second->t_done - it->second->t_submit).count();
    return 0;
}

int shs_server_stats(shs_server *srv, shs_server_stats_t *out)
{
    if (!srv) return -1;
    if (!out) return -2;
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->queued = (int64_t)srv->pending.size();
    out->running = srv->running;
    out->solves = srv->solves;
    out->batches = srv->batches;
    out->max_batch_systems = srv->max_sys;
    out->peak_bytes = (int64_t)srv->peak;
    if (!srv->lat_ms.empty()) {
        std::vector<double> v = srv->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const double pos = q * (double)(v.size() - 1);
            const size_t lo = (size_t)pos;
            const size_t hi = std::min(lo + 1, v.size() - 1);
            return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
    }
    if (srv->any) out->busy_s = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
    return 0;
}

void shs_server_destroy(shs_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    for (hipStream_t st : srv->streams) hipStreamDestroy(st);
    delete srv;
}

}  // extern "C"
