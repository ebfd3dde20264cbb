// Continuous-batching server for multigrid pressure solves (host side).
//
// One worker thread owns every device object of the server.  Requests wait in
// a FIFO queue; the head is admitted as soon as a slot is free and its
// hierarchy fits the HBM budget (idle resident hierarchies of other
// configurations are evicted, least recently used first, to make room).  Each
// slot has its own non-blocking stream of default priority, so the cycles of
// all running requests overlap on the device.  A hierarchy owns work copies of
// b and x, which keeps the captured one-cycle graph valid from one request to
// the next; a finished hierarchy stays resident and is reused, with a fresh
// coefficient, by the next request of the same configuration.  The stopping
// rule of each request runs on the device; the worker only polls an event per
// batch of cycles.
#include "mg_internal.h"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace nn4mg;

namespace {

bool same_config(const nn4mg_config &a, const nn4mg_config &b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

struct Request {
    unsigned long long tag = 0;
    nn4mg_config cfg{};
    const double *k = nullptr;
    const double *b = nullptr;
    double *x = nullptr;
    double rtol = 1e-8;
    int max_cycles = 100;
    double t_submit = 0.0;
    size_t n = 0;
};

struct Resident {
    nn4mg_config cfg{};
    nn4mg_t H = nullptr;
    double *bw = nullptr;  // work copy of b
    double *xw = nullptr;  // work copy of x
    size_t bytes = 0;
    bool busy = false;
    double last_used = 0.0;
};

struct Slot {
    bool busy = false;
    Request req;
    int res = -1;          // index into residents
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int phase = 0;         // 0 = new, 1 = running
    double t_start = 0.0;
};

}  // namespace

struct nn4mg_server {
    size_t budget = 0;
    int device = 0;
    std::vector<Slot> slots;
    std::vector<Resident> residents;
    std::deque<Request> queue;
    std::vector<nn4mg_result> results;
    std::atomic<size_t> in_use{0}, peak{0};
    int outstanding = 0;  // submitted and not yet finished
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<bool> stop{false};
    std::thread worker;
    std::chrono::steady_clock::time_point t0;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

size_t request_bytes(const nn4mg_config &cfg)
{
    const size_t n = (size_t)cfg.nx * cfg.ny * cfg.nz;
    return nn4mg_bytes_required(&cfg) + 2 * n * sizeof(double);
}

void finish_request(nn4mg_server *S, Slot &sl, const nn4mg_info &info, int status, size_t bytes)
{
    nn4mg_result r;
    std::memset(&r, 0, sizeof(r));
    r.tag = sl.req.tag;
    r.info = info;
    r.info.status = status;
    r.t_submit_ms = sl.req.t_submit;
    r.t_start_ms = sl.t_start;
    r.t_done_ms = S->now_ms();
    r.bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->results.push_back(r);
        S->outstanding--;
    }
    S->cv.notify_all();
    if (sl.res >= 0) {
        S->residents[sl.res].busy = false;
        S->residents[sl.res].last_used = S->now_ms();
    }
    sl.busy = false;
    sl.res = -1;
    sl.phase = 0;
}

void free_resident(nn4mg_server *S, int i)
{
    Resident &R = S->residents[i];
    nn4mg_destroy(R.H);
    if (R.bw) (void)hipFree(R.bw);
    if (R.xw) (void)hipFree(R.xw);
    S->in_use -= R.bytes;
    S->residents.erase(S->residents.begin() + i);
    for (Slot &sl : S->slots)
        if (sl.res > i) sl.res--;
}

// Find or build a resident hierarchy for the request; -1 if memory is short
// right now (nothing changed), -2 on a hard error (status in *err).
int acquire_resident(nn4mg_server *S, Slot &sl, int *err)
{
    const Request &q = sl.req;
    for (size_t i = 0; i < S->residents.size(); ++i) {
        Resident &R = S->residents[i];
        if (!R.busy && same_config(R.cfg, q.cfg)) {
            R.busy = true;
            if ((*err = hier_set_stream(R.H, sl.stream)) ||
                (q.cfg.coef_mode == NN4MG_COEF_NODAL && (*err = nn4mg_update_coef(R.H, q.k)))) {
                R.busy = false;
                return -2;
            }
            return (int)i;
        }
    }
    const size_t need = request_bytes(q.cfg);
    while (S->in_use + need > S->budget) {
        int victim = -1;
        for (size_t i = 0; i < S->residents.size(); ++i)
            if (!S->residents[i].busy && (victim < 0 || S->residents[i].last_used < S->residents[victim].last_used))
                victim = (int)i;
        if (victim < 0) return -1;
        free_resident(S, victim);
    }
    Resident R;
    R.cfg = q.cfg;
    if ((*err = nn4mg_setup(&q.cfg, q.k, (void *)sl.stream, &R.H))) return -2;
    if (hipMalloc((void **)&R.bw, q.n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&R.xw, q.n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        nn4mg_destroy(R.H);
        if (R.bw) (void)hipFree(R.bw);
        *err = NN4MG_ENOMEM;
        return -2;
    }
    R.bytes = nn4mg_bytes_held(R.H) + 2 * q.n * sizeof(double);
    R.busy = true;
    S->in_use += R.bytes;
    if (S->in_use.load() > S->peak.load()) S->peak.store(S->in_use.load());
    S->residents.push_back(R);
    return (int)S->residents.size() - 1;
}

// Advance one slot; returns true if it made progress.
bool step_slot(nn4mg_server *S, Slot &sl)
{
    if (!sl.busy) return false;
    nn4mg_info info;
    std::memset(&info, 0, sizeof(info));
    if (sl.phase == 0) {
        int err = 0;
        const int r = acquire_resident(S, sl, &err);
        if (r == -1) return false;  // waits for memory
        if (r == -2) {
            finish_request(S, sl, info, err, 0);
            return true;
        }
        sl.res = r;
        Resident &R = S->residents[r];
        const size_t bytes = sl.req.n * sizeof(double);
        int rc = NN4MG_OK;
        if (hipMemcpyAsync(R.bw, sl.req.b, bytes, hipMemcpyDeviceToDevice, sl.stream) != hipSuccess ||
            hipMemcpyAsync(R.xw, sl.req.x, bytes, hipMemcpyDeviceToDevice, sl.stream) != hipSuccess)
            rc = NN4MG_EDEVICE;
        if (!rc) rc = solve_begin(R.H, R.bw, R.xw, sl.req.rtol, sl.req.max_cycles, 0);
        if (!rc) rc = solve_enqueue_next(R.H, R.bw, R.xw);
        if (!rc) rc = solve_header_async(R.H, sl.ev);
        if (rc) {
            (void)hipGetLastError();
            finish_request(S, sl, info, rc, R.bytes);
            return true;
        }
        sl.phase = 1;
        return true;
    }
    const hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) return false;
    Resident &R = S->residents[sl.res];
    int rc = (q == hipSuccess) ? NN4MG_OK : NN4MG_EDEVICE;
    if (!rc && !solve_after_header(R.H)) {
        rc = solve_enqueue_next(R.H, R.bw, R.xw);
        if (!rc) rc = solve_header_async(R.H, sl.ev);
        if (!rc) return true;
    }
    int status = rc;
    if (!rc) {
        status = solve_finish(R.H, R.xw, &info);
        if (hipMemcpyAsync(sl.req.x, R.xw, sl.req.n * sizeof(double), hipMemcpyDeviceToDevice, sl.stream) !=
                hipSuccess ||
            hipStreamSynchronize(sl.stream) != hipSuccess)
            status = NN4MG_EDEVICE;
    }
    (void)hipGetLastError();
    finish_request(S, sl, info, status, R.bytes);
    return true;
}

void worker_main(nn4mg_server *S)
{
    (void)hipSetDevice(S->device);
    while (true) {
        bool progress = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop.load() && S->queue.empty()) {
                bool any = false;
                for (Slot &sl : S->slots) any = any || sl.busy;
                if (!any) break;
            }
            for (Slot &sl : S->slots) {
                if (sl.busy || S->queue.empty()) continue;
                sl.req = S->queue.front();
                S->queue.pop_front();
                sl.busy = true;
                sl.phase = 0;
                sl.t_start = S->now_ms();
                progress = true;
            }
        }
        for (Slot &sl : S->slots) progress = step_slot(S, sl) || progress;
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" {

int nn4mg_server_create(size_t budget, int max_slots, nn4mg_srv_t *out)
{
    if (!out || max_slots < 1 || max_slots > 64 || budget == 0)
        return set_error(NN4MG_EINVAL, "server: NULL out, zero budget, or max_slots outside 1..64");
    *out = nullptr;
    nn4mg_server *S = new nn4mg_server();
    S->budget = budget;
    S->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return set_error(NN4MG_EDEVICE, "server: hipGetDevice failed");
    }
    S->slots.resize(max_slots);
    for (Slot &sl : S->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            for (Slot &t : S->slots) {
                if (t.stream) (void)hipStreamDestroy(t.stream);
                if (t.ev) (void)hipEventDestroy(t.ev);
            }
            delete S;
            return set_error(NN4MG_EDEVICE, "server: creating a slot stream or event failed");
        }
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return NN4MG_OK;
}

int nn4mg_server_submit(nn4mg_srv_t S, const nn4mg_config *cfg, const double *k, const double *b, double *x,
                        double rtol, int max_cycles, unsigned long long tag)
{
    if (!S || !cfg || !b || !x || max_cycles < 0 || !(rtol >= 0.0))
        return set_error(NN4MG_EINVAL, "server submit: NULL argument, max_cycles < 0 or rtol < 0");
    if (cfg->coef_mode == NN4MG_COEF_NODAL && !k) return set_error(NN4MG_EINVAL, "server submit: NULL k for NODAL");
    const size_t need = nn4mg_bytes_required(cfg);
    if (need == 0) return set_error(NN4MG_EINVAL, "server submit: invalid configuration");
    if (request_bytes(*cfg) > S->budget) return set_error(NN4MG_EBUSY, "server submit: request exceeds the whole budget");
    Request q;
    q.tag = tag;
    q.cfg = *cfg;
    q.k = k;
    q.b = b;
    q.x = x;
    q.rtol = rtol;
    q.max_cycles = max_cycles;
    q.n = (size_t)cfg->nx * cfg->ny * cfg->nz;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop.load()) return set_error(NN4MG_EINVAL, "server submit: server is stopping");
        q.t_submit = S->now_ms();
        S->queue.push_back(q);
        S->outstanding++;
    }
    return NN4MG_OK;
}

int nn4mg_server_poll(nn4mg_srv_t S, nn4mg_result *out, int cap, int *n_done)
{
    if (!S || (!out && cap > 0)) return set_error(NN4MG_EINVAL, "server poll: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    int n = 0;
    while (n < cap && !S->results.empty()) {
        out[n++] = S->results.front();
        S->results.erase(S->results.begin());
    }
    if (n_done) *n_done = n;
    return NN4MG_OK;
}

int nn4mg_server_drain(nn4mg_srv_t S, double timeout_ms)
{
    if (!S) return set_error(NN4MG_EINVAL, "server: NULL handle");
    std::unique_lock<std::mutex> lk(S->mu);
    auto pred = [&] { return S->outstanding == 0; };
    if (timeout_ms < 0) {
        S->cv.wait(lk, pred);
        return NN4MG_OK;
    }
    if (S->cv.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred)) return NN4MG_OK;
    return set_error(NN4MG_EBUSY, "server drain: timed out with requests outstanding");
}

int nn4mg_server_stats(nn4mg_srv_t S, size_t *in_use, size_t *peak, int *active, int *queued)
{
    if (!S) return set_error(NN4MG_EINVAL, "server: NULL handle");
    std::lock_guard<std::mutex> lk(S->mu);
    if (in_use) *in_use = S->in_use;
    if (peak) *peak = S->peak;
    int a = 0;
    for (const Slot &sl : S->slots) a += sl.busy ? 1 : 0;
    if (active) *active = a;
    if (queued) *queued = (int)S->queue.size();
    return NN4MG_OK;
}

int nn4mg_server_destroy(nn4mg_srv_t S)
{
    if (!S) return NN4MG_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->outstanding -= (int)S->queue.size();
        S->queue.clear();
        S->stop.store(true);
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->device);
    while (!S->residents.empty()) free_resident(S, (int)S->residents.size() - 1);
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    delete S;
    return NN4MG_OK;
}

}  // extern "C"
