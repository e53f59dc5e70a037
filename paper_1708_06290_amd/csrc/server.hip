// Serving layer: resident systems, admission by device-memory footprint and
// continuous batching of shift requests (shs_server_* in shiftsolve.h).
//
// Worker threads each own a HIP stream.  A free worker takes the oldest
// waiting request.  A request on the work-item route (FP64, one shift small
// enough for one wavefront) takes every other waiting work-item request that
// still fits in the memory budget (any system, any n and m) and runs all
// their shifts in one launch of the work-item kernel, then forms G and the
// backward error per request.  A request on the solve route (mixed
// precision, or FP64 on a system whose shifts need the blocked sweep) takes
// the other waiting requests of the same system, mode and outputs that fit,
// and runs their shifts as one shs_solve.  Requests submitted meanwhile wait
// in the queue and are admitted by the next free worker, so work from
// different requests overlaps on the device through the workers' streams.
// Every kernel of the library computes each shift independently of the
// others in its launch, so a request's results are bitwise the same alone
// and in any batch.
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
    bool alone = false;           // solve route: shs_solve (mixed mode, or blocked FP64)
    Clock::time_point t_arrival, t_done;
    hipEvent_t after = nullptr;   // the caller's stream at submit: the request's work waits for it
    int state = 0;                // SHS_REQ_* (queued, running, done, failed, cancelled)
    bool cancel = false;          // cancelled while running: marked so on completion
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
    bool stop = false, paused = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, running = 0, solves = 0, batches = 0,
            max_sys = 0, max_reqs = 0;
    std::vector<double> lat_ms;
    bool any = false;
    Clock::time_point t_first, t_last;

    void worker(int wid);
    int run_fp64_batch(std::vector<std::shared_ptr<Request>> &batch, hipStream_t st);
    int run_solve_batch(std::vector<std::shared_ptr<Request>> &batch, hipStream_t st);
    size_t solve_batch_bytes(const shs_handle *h, int64_t s, int mode, int outputs) const;
};

namespace {

// The stream waits for the callers' streams of every request in the batch.
hipError_t wait_callers(const std::vector<std::shared_ptr<Request>> &batch, hipStream_t st)
{
    for (auto &r : batch)
        if (r->after) {
            hipError_t e = hipStreamWaitEvent(st, r->after, 0);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace

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
    hipError_t e = wait_callers(batch, st);
    if (e != hipSuccess) return SHS_ERR_HIP;
    char *work = nullptr;
    e = hipMallocAsync((void **)&work, total, st);
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
            e = certify(h, r.s, nullptr, nullptr, (const double *)(work + offs[b].shifts), X, ldx, nullptr,
                        (unsigned long long *)(work + offs[b].resmax), (unsigned long long *)(work + offs[b].xmax),
                        r.eta, r.status, r.s, (double *)(work + offs[b].xt), st);
    }
    hipError_t e2 = hipFreeAsync(work, st);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? 0 : (e == hipErrorOutOfMemory ? SHS_ERR_NOMEM : SHS_ERR_HIP);
}

// Device bytes of one shs_solve over s shifts of h on the solve route: the
// solve's workspace, the shifts and the batch's own X, G, eta and status
// (the requests' outputs are filled from them).
size_t shs_server::solve_batch_bytes(const shs_handle *h, int64_t s, int mode, int outputs) const
{
    size_t ws = 0;
    if (shs_solve_workspace(h, s, mode, outputs, &ws) != 0) return (size_t)-1;
    const size_t x = (outputs & SHS_OUT_X) ? al256(sizeof(double) * 2 * (size_t)(h->n * h->m * s)) : 0;
    const size_t g = (outputs & SHS_OUT_G) && h->p > 0 ? al256(sizeof(double) * 2 * (size_t)(h->p * h->m * s)) : 0;
    return al256(ws) + x + g + 3 * al256(sizeof(double) * 2 * (size_t)s);
}

int shs_server::run_solve_batch(std::vector<std::shared_ptr<Request>> &batch, hipStream_t st)
{
    const Request &r0 = *batch[0];
    shs_handle *h = systems[r0.sys];
    const int64_t n = h->n, m = h->m, p = h->p;
    int64_t S = 0;
    for (auto &r : batch) S += r->s;
    const bool one = batch.size() == 1;
    size_t ws = 0;
    if (shs_solve_workspace(h, S, r0.mode, r0.outputs, &ws) != 0) return SHS_ERR_UNSUPPORTED;
    // a single request writes straight into its own outputs
    const bool wx = (r0.outputs & SHS_OUT_X) && !one, wg = (r0.outputs & SHS_OUT_G) && p > 0 && !one;
    size_t total = 0;
    auto take = [&](size_t bytes) { size_t o = total; total += al256(bytes); return o; };
    const size_t o_ws = take(ws);
    const size_t o_sh = take(sizeof(double) * 2 * S);
    const size_t o_x = wx ? take(sizeof(double) * 2 * n * m * S) : 0;
    const size_t o_g = wg ? take(sizeof(double) * 2 * p * m * S) : 0;
    const size_t o_eta = one ? 0 : take(sizeof(double) * S);
    const size_t o_st = one ? 0 : take(sizeof(int32_t) * S);
    hipError_t e = wait_callers(batch, st);
    if (e != hipSuccess) return SHS_ERR_HIP;
    char *work = nullptr;
    e = hipMallocAsync((void **)&work, total, st);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SHS_ERR_NOMEM : SHS_ERR_HIP;
    int64_t off = 0;
    for (auto &r : batch) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(work + o_sh + sizeof(double) * 2 * off, r->shifts.data(), sizeof(double) * 2 * r->s,
                               hipMemcpyHostToDevice, st);
        off += r->s;
    }
    int rc = e == hipSuccess ? 0 : SHS_ERR_HIP;
    double *X = one ? r0.X : (double *)(work + o_x);
    const int64_t ldx = one ? r0.ldx : n;
    double *G = one ? r0.G : (double *)(work + o_g);
    const int64_t ldg = one ? r0.ldg : std::max<int64_t>(1, p);
    double *eta = one ? r0.eta : (double *)(work + o_eta);
    int32_t *status = one ? r0.status : (int32_t *)(work + o_st);
    if (!one) {
        // a batch certifies every shift (mixed mode needs eta in any case)
        if (!(r0.outputs & SHS_OUT_X)) X = nullptr;
        if (!((r0.outputs & SHS_OUT_G) && p > 0)) G = nullptr;
    }
    if (rc == 0)
        rc = shs_solve(h, S, (const double *)(work + o_sh), r0.mode, r0.outputs | (one ? 0 : SHS_OUT_ETA), 1e-13, 5,
                       work + o_ws, ws, X, ldx, G, ldg, eta, status, st);
    // scatter the batch's outputs to the requests
    off = 0;
    for (auto &r : batch) {
        if (rc != 0 || one) break;
        const int64_t c0 = off * m, nc = r->s * m;
        if (r->outputs & SHS_OUT_X)
            e = hipMemcpy2DAsync(r->X, sizeof(double) * 2 * r->ldx, X + 2 * c0 * n, sizeof(double) * 2 * n,
                                 sizeof(double) * 2 * n, nc, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && (r->outputs & SHS_OUT_G) && p > 0)
            e = hipMemcpy2DAsync(r->G, sizeof(double) * 2 * r->ldg, G + 2 * c0 * ldg, sizeof(double) * 2 * ldg,
                                 sizeof(double) * 2 * p, nc, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && r->eta)
            e = hipMemcpyAsync(r->eta, eta + off, sizeof(double) * r->s, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->status, status + off, sizeof(int32_t) * r->s, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) rc = SHS_ERR_HIP;
        off += r->s;
    }
    hipFreeAsync(work, st);
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
                if (!pending.empty() && !paused) {
                    auto head = pending.front();
                    const shs_handle *hh = systems[head->sys];
                    const size_t head_fp =
                        head->alone ? solve_batch_bytes(hh, head->s, head->mode, head->outputs) : head->footprint;
                    if (in_use + head_fp <= budget) {
                        pending.pop_front();
                        batch.push_back(head);
                        fp = head_fp;
                        int64_t S = head->s;
                        for (auto it = pending.begin(); it != pending.end() && (int)batch.size() < max_batch;) {
                            const Request &r = **it;
                            bool join = false;
                            size_t nfp = 0;
                            if (!head->alone && !r.alone) {
                                // work-item route: any system
                                nfp = fp + r.footprint;
                                join = true;
                            } else if (head->alone && r.alone && r.sys == head->sys && r.mode == head->mode &&
                                       r.outputs == head->outputs) {
                                // solve route: the same system, mode and outputs
                                nfp = solve_batch_bytes(hh, S + r.s, head->mode, head->outputs);
                                join = true;
                            }
                            if (join && in_use + nfp <= budget) {
                                fp = nfp;
                                S += r.s;
                                batch.push_back(*it);
                                it = pending.erase(it);
                            } else {
                                ++it;
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
            for (auto &r : batch) r->state = SHS_REQ_RUNNING;
            ++batches;
            std::vector<int32_t> sy;
            for (auto &r : batch) sy.push_back(r->sys);
            std::sort(sy.begin(), sy.end());
            max_sys = std::max<int64_t>(max_sys, std::unique(sy.begin(), sy.end()) - sy.begin());
            max_reqs = std::max<int64_t>(max_reqs, (int64_t)batch.size());
        }
        const int rc = batch[0]->alone ? run_solve_batch(batch, st) : run_fp64_batch(batch, st);
        const auto now = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= fp;
            running -= (int64_t)batch.size();
            for (auto &r : batch) {
                r->t_done = now;
                r->error = rc;
                if (r->after) {
                    hipEventDestroy(r->after);
                    r->after = nullptr;
                }
                if (r->cancel) {
                    r->state = SHS_REQ_CANCELLED;
                    ++cancelled;
                } else if (rc == 0) {
                    r->state = SHS_REQ_DONE;
                    ++completed;
                    solves += r->s;
                    lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_arrival).count());
                } else {
                    r->state = SHS_REQ_FAILED;
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

double shs_server_clock(void)
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

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

int shs_server_submit_ex(shs_server *srv, int32_t sys_id, int64_t s, const double *shifts_host, int mode,
                         int outputs, double *X, int64_t ldx, double *G, int64_t ldg, double *eta, int32_t *status,
                         const shs_request_opts *opts, int64_t *req_id)
{
    if (!srv) return -1;
    if (!req_id) return -14;
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
    if (opts && opts->abi_version != SHS_ABI_VERSION) return -13;
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
    r->footprint = r->alone ? srv->solve_batch_bytes(h, s, mode, outputs) : fp64_item_bytes(h, s);
    if (r->footprint > srv->budget) return SHS_ERR_NOMEM;
    if (opts && opts->order_after) {
        // the request's work starts after what the caller queued on its stream
        hipSetDevice(srv->device);
        if (hipEventCreateWithFlags(&r->after, hipEventDisableTiming) != hipSuccess) return SHS_ERR_HIP;
        if (hipEventRecord(r->after, (hipStream_t)opts->after_stream) != hipSuccess) {
            hipEventDestroy(r->after);
            return SHS_ERR_HIP;
        }
    }
    const auto now = Clock::now();
    r->t_arrival = now;
    if (opts && opts->arrival_s > 0.0) {
        const auto t = Clock::time_point(std::chrono::duration_cast<Clock::duration>(
            std::chrono::duration<double>(opts->arrival_s)));
        if (t < now) r->t_arrival = t;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        r->id = srv->next_id++;
        srv->reqs[r->id] = r;
        srv->pending.push_back(r);
        ++srv->submitted;
        if (!srv->any || r->t_arrival < srv->t_first) srv->t_first = r->t_arrival;
        srv->any = true;
        *req_id = r->id;
    }
    srv->cv_work.notify_one();
    return 0;
}

int shs_server_submit(shs_server *srv, int32_t sys_id, int64_t s, const double *shifts_host, int mode, int outputs,
                      double *X, int64_t ldx, double *G, int64_t ldg, double *eta, int32_t *status, int64_t *req_id)
{
    return shs_server_submit_ex(srv, sys_id, s, shifts_host, mode, outputs, X, ldx, G, ldg, eta, status, nullptr,
                                req_id);
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
    auto done = [&] { return r->state >= SHS_REQ_DONE; };
    if (timeout_ms < 0) {
        srv->cv_done.wait(lk, done);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done)) {
        return SHS_ERR_TIMEOUT;
    }
    if (r->state == SHS_REQ_DONE) return 0;
    return r->state == SHS_REQ_CANCELLED ? SHS_ERR_CANCELLED : r->error;
}

int shs_server_cancel(shs_server *srv, int64_t req_id)
{
    if (!srv) return -1;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(req_id);
        if (it == srv->reqs.end()) return SHS_ERR_NOTFOUND;
        auto r = it->second;
        if (r->state == SHS_REQ_QUEUED) {
            for (auto q = srv->pending.begin(); q != srv->pending.end(); ++q)
                if (q->get() == r.get()) {
                    srv->pending.erase(q);
                    break;
                }
            if (r->after) {
                hipEventDestroy(r->after);
                r->after = nullptr;
            }
            r->state = SHS_REQ_CANCELLED;
            ++srv->cancelled;
        } else if (r->state == SHS_REQ_RUNNING) {
            r->cancel = true;   // it completes; it is then marked cancelled
        } else {
            return SHS_ERR_STATE;
        }
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
    return 0;
}

int shs_server_pause(shs_server *srv, int paused)
{
    if (!srv) return -1;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->paused = paused != 0;
    }
    srv->cv_work.notify_all();
    return 0;
}

int shs_server_latency(shs_server *srv, int64_t req_id, double *ms)
{
    if (!srv) return -1;
    if (!ms) return -3;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return SHS_ERR_NOTFOUND;
    if (it->second->state != SHS_REQ_DONE) return SHS_ERR_STATE;
    *ms = std::chrono::duration<double, std::milli>(it->second->t_done - it->second->t_arrival).count();
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
    out->cancelled = srv->cancelled;
    out->queued = (int64_t)srv->pending.size();
    out->running = srv->running;
    out->solves = srv->solves;
    out->batches = srv->batches;
    out->max_batch_systems = srv->max_sys;
    out->max_batch_requests = srv->max_reqs;
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
        srv->paused = false;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    for (hipStream_t st : srv->streams) hipStreamDestroy(st);
    for (auto &kv : srv->reqs)
        if (kv.second->after) hipEventDestroy(kv.second->after);
    delete srv;
}

}  // extern "C"
