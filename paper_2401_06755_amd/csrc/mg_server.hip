// Continuous-batching server for multigrid pressure solves (host side).
//
// One worker thread owns every device object of the server.  Requests wait in
// a FIFO queue and are admitted while fewer than max_slots run.  Requests of
// one configuration are batched: a group is a batched hierarchy of up to 16
// identical copies (one arena, fixed stride), so each kernel of a cycle is one
// launch that advances the tiles of every running copy, and one captured
// graph of that batched cycle serves every batch of cycles.  A request joins a
// free copy of its configuration's group between two batches (its own
// coefficient, right-hand side and iterate are copied in and its solve is
// begun through the copy's view), runs until its own stopping rule fires on
// the device (its workgroups then exit at once in later launches) and leaves
// at the next batch boundary.  Each group has a non-blocking stream of default
// priority, so different configurations overlap on the device.  A group is
// created when its configuration has none with a free copy and the HBM budget
// allows; idle groups (and idle per-request hierarchies) are evicted least
// recently used first.  Configurations with no batched form (flexible CG, no
// one-workgroup coarse end, other than two post-sweeps) run one per slot, each
// with its own stream, hierarchy and one-cycle graph.
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

// One copy of a group: the request it runs, its view and where its request is
// in its life: FREE; ADMIT (coefficient set-up in flight on the admission
// stream, then the host forms the coarsest inverse); RUNNING (in the batches);
// FINISH (projection and state copy-back in flight on the group stream).
enum MemberState { M_FREE = 0, M_ADMIT = 1, M_RUNNING = 2, M_FINISH = 3 };

struct Member {
    int state = M_FREE;
    bool fresh = false;  // started while a batch ran: not in that batch
    Request req;
    double t_start = 0.0;
    nn4mg_hier *V = nullptr;
    hipEvent_t ev = nullptr;  // completion of the member's ADMIT or FINISH work
    double *hk = nullptr;     // pinned: the coarsest level's k, the inverse, the check flag
    double *inv = nullptr;
    int *bad = nullptr;
};

struct Group {
    nn4mg_config cfg{};
    nn4mg_hier *G = nullptr;
    std::vector<Member> m;
    hipStream_t stream = nullptr;
    hipStream_t admit = nullptr;  // copies and coefficient set-up of joining requests
    hipEvent_t ev = nullptr;
    bool in_flight = false;  // a batch of cycles and the members' headers are enqueued
    size_t bytes = 0;
    double last_used = 0.0;
    void *pinned = nullptr;
    int busy() const
    {
        int n = 0;
        for (const Member &mb : m) n += mb.state != M_FREE ? 1 : 0;
        return n;
    }
};

constexpr int kGroupCap = 16;
constexpr int kMaxBatchCycles = 16;

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
    std::vector<Group *> groups;
    std::vector<nn4mg_config> unbatchable;  // configurations with no batched form
    int max_active = 0;
    std::atomic<int> active_now{0};         // running requests, as the worker last counted them
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

void push_result(nn4mg_server *S, const Request &q, double t_start, const nn4mg_info &info, int status,
                 size_t bytes)
{
    nn4mg_result r;
    std::memset(&r, 0, sizeof(r));
    r.tag = q.tag;
    r.info = info;
    r.info.status = status;
    r.t_submit_ms = q.t_submit;
    r.t_start_ms = t_start;
    r.t_done_ms = S->now_ms();
    r.bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->results.push_back(r);
        S->outstanding--;
    }
    S->cv.notify_all();
}

void finish_request(nn4mg_server *S, Slot &sl, const nn4mg_info &info, int status, size_t bytes)
{
    push_result(S, sl.req, sl.t_start, info, status, bytes);
    if (sl.res >= 0) {
        S->residents[sl.res].busy = false;
        S->residents[sl.res].last_used = S->now_ms();
    }
    sl.busy = false;
    sl.res = -1;
    sl.phase = 0;
}

void free_group(nn4mg_server *S, int i);

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

// Evict idle per-request hierarchies and idle groups, least recently used
// first, until `need` more bytes fit the budget; false if they cannot.
bool make_room(nn4mg_server *S, size_t need)
{
    if (need > S->budget) return false;
    while (S->in_use + need > S->budget) {
        int vr = -1, vg = -1;
        double tr = 0.0, tg = 0.0;
        for (size_t i = 0; i < S->residents.size(); ++i)
            if (!S->residents[i].busy && (vr < 0 || S->residents[i].last_used < tr)) {
                vr = (int)i;
                tr = S->residents[i].last_used;
            }
        for (size_t i = 0; i < S->groups.size(); ++i) {
            const Group *g = S->groups[i];
            if (!g->in_flight && g->busy() == 0 && (vg < 0 || g->last_used < tg)) {
                vg = (int)i;
                tg = g->last_used;
            }
        }
        if (vr < 0 && vg < 0) return false;
        if (vg < 0 || (vr >= 0 && tr <= tg))
            free_resident(S, vr);
        else
            free_group(S, vg);
    }
    return true;
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
    if (!make_room(S, request_bytes(q.cfg))) return -1;
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

// ---- groups ----

bool batchable(const nn4mg_server *S, const nn4mg_config &cfg)
{
    for (const nn4mg_config &c : S->unbatchable)
        if (same_config(c, cfg)) return false;
    return true;
}

size_t group_bytes(const nn4mg_config &cfg, int cap)
{
    return (size_t)cap * request_bytes(cfg);
}

void destroy_group_objects(Group *g)
{
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->admit) (void)hipStreamSynchronize(g->admit);
    for (Member &mb : g->m) {
        view_destroy(mb.V);
        if (mb.ev) (void)hipEventDestroy(mb.ev);
    }
    if (g->G) nn4mg_destroy(g->G);
    if (g->pinned) (void)hipHostFree(g->pinned);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    if (g->admit) (void)hipStreamDestroy(g->admit);
    if (g->ev) (void)hipEventDestroy(g->ev);
    delete g;
}

void free_group(nn4mg_server *S, int i)
{
    Group *g = S->groups[i];
    S->in_use -= g->bytes;
    destroy_group_objects(g);
    S->groups.erase(S->groups.begin() + i);
}

void finish_member(nn4mg_server *S, Group *g, Member &mb, const nn4mg_info &info, int status)
{
    push_result(S, mb.req, mb.t_start, info, status, g->bytes / g->m.size());
    mb.state = M_FREE;
    mb.fresh = false;
    g->last_used = S->now_ms();
    // a solve that ended on an error may have left its stopping flag clear:
    // set it (after the group's work so far), so later batches skip the copy
    if (status != NN4MG_OK && status != NN4MG_ENOTCONV && status != NN4MG_EBREAKDOWN) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipStreamSynchronize(g->admit);
        (void)hipGetLastError();
        hier_use_stream(mb.V, g->stream);
        (void)hier_mark_idle(mb.V);
        (void)hipGetLastError();
    }
}

void fail_member(nn4mg_server *S, Group *g, Member &mb, int status)
{
    (void)hipGetLastError();
    nn4mg_info info;
    std::memset(&info, 0, sizeof(info));
    finish_member(S, g, mb, info, status);
}

// A new group for cfg (its copies idle); nullptr if memory is short or the
// configuration has no batched form (then recorded as unbatchable).
Group *create_group(nn4mg_server *S, const nn4mg_config &cfg)
{
    // as many copies as fit the budget, up to the running-request limit and
    // kGroupCap; fewer (halving) while busy work holds the memory
    int cap = S->max_active < kGroupCap ? S->max_active : kGroupCap;
    const size_t per = request_bytes(cfg);
    if ((size_t)cap * per > S->budget) cap = (int)(S->budget / per);
    while (cap >= 1 && !make_room(S, group_bytes(cfg, cap))) cap /= 2;
    if (cap < 1) return nullptr;
    Group *g = new Group();
    g->cfg = cfg;
    if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&g->admit, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        destroy_group_objects(g);
        return nullptr;
    }
    const int rc = setup_hier(&cfg, nullptr, g->stream, cap, &g->G, true);
    if (rc) {
        (void)hipGetLastError();
        g->G = nullptr;
        destroy_group_objects(g);
        if (rc == NN4MG_EINVAL) S->unbatchable.push_back(cfg);
        return nullptr;
    }
    const size_t nc = (size_t)hier_coarse_cells(g->G);
    const size_t per_member = nc + nc * nc + 1;  // doubles: hk, inv, flag
    bool ok = hipHostMalloc(&g->pinned, per_member * sizeof(double) * cap, hipHostMallocDefault) == hipSuccess;
    g->m.resize(cap);
    const bool nodal = cfg.coef_mode == NN4MG_COEF_NODAL;
    for (int c = 0; ok && c < cap; ++c) {
        Member &mb = g->m[c];
        double *base = (double *)g->pinned + per_member * c;
        mb.hk = base;
        mb.inv = base + nc;
        mb.bad = (int *)(base + nc + nc * nc);
        ok = view_create(g->G, c, &mb.V) == NN4MG_OK &&
             hipEventCreateWithFlags(&mb.ev, hipEventDisableTiming) == hipSuccess && hier_mark_idle(mb.V) == NN4MG_OK &&
             // a constant coefficient is the same for every request: set up once
             (nodal || hier_load_coef(mb.V, nullptr) == NN4MG_OK);
    }
    if (!ok) {
        (void)hipGetLastError();
        destroy_group_objects(g);
        return nullptr;
    }
    g->bytes = nn4mg_bytes_held(g->G);
    g->last_used = S->now_ms();
    S->in_use += g->bytes;
    if (S->in_use.load() > S->peak.load()) S->peak.store(S->in_use.load());
    S->groups.push_back(g);
    return g;
}

// Start request q on idle copy i.  The copy's stopping flag is set, so a
// batch in flight on the group stream does not touch it: its right-hand
// side, iterate and coefficient go in on the admission stream; the host
// finishes the coefficient set-up when that work has arrived (advance_member).
void admit_member(nn4mg_server *S, Group *g, int i, const Request &q, double t_start)
{
    Member &mb = g->m[i];
    mb.req = q;
    mb.t_start = t_start;
    mb.state = M_ADMIT;
    mb.fresh = false;
    nn4mg_hier *V = mb.V;
    const size_t bytes = q.n * sizeof(double);
    hier_use_stream(V, g->admit);
    int rc = NN4MG_OK;
    if (hipMemcpyAsync(hier_bw(V), q.b, bytes, hipMemcpyDeviceToDevice, g->admit) != hipSuccess ||
        hipMemcpyAsync(hier_xw(V), q.x, bytes, hipMemcpyDeviceToDevice, g->admit) != hipSuccess)
        rc = NN4MG_EDEVICE;
    if (!rc && q.cfg.coef_mode == NN4MG_COEF_NODAL) rc = coef_begin(V, q.k, mb.hk, mb.bad);
    if (!rc && hipEventRecord(mb.ev, g->admit) != hipSuccess) rc = NN4MG_EDEVICE;
    hier_use_stream(V, g->stream);
    if (rc) fail_member(S, g, mb, rc);
}

// Move a member on when its enqueued work has arrived.  ADMIT: the coarsest
// inverse and its upload, then (ordered after the admission work and after
// any batch in flight) the solve's start on the group stream.  FINISH: the
// result.
bool advance_member(nn4mg_server *S, Group *g, Member &mb)
{
    if (mb.state != M_ADMIT && mb.state != M_FINISH) return false;
    const hipError_t e = hipEventQuery(mb.ev);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) {
        fail_member(S, g, mb, NN4MG_EDEVICE);
        return true;
    }
    nn4mg_hier *V = mb.V;
    if (mb.state == M_FINISH) {
        nn4mg_info info;
        std::memset(&info, 0, sizeof(info));
        const int status = solve_finish_complete(V, &info);
        finish_member(S, g, mb, info, status);
        return true;
    }
    int rc = NN4MG_OK;
    if (mb.req.cfg.coef_mode == NN4MG_COEF_NODAL) {
        hier_use_stream(V, g->admit);
        rc = coef_end(V, mb.hk, mb.bad, mb.inv);
        if (!rc && hipEventRecord(mb.ev, g->admit) != hipSuccess) rc = NN4MG_EDEVICE;
        hier_use_stream(V, g->stream);
    }
    if (!rc && hipStreamWaitEvent(g->stream, mb.ev, 0) != hipSuccess) rc = NN4MG_EDEVICE;
    if (!rc) rc = solve_begin(V, hier_bw(V), hier_xw(V), mb.req.rtol, mb.req.max_cycles, 0);
    if (rc) {
        fail_member(S, g, mb, rc);
        return true;
    }
    mb.state = M_RUNNING;
    mb.fresh = g->in_flight;
    return true;
}

// Place request q: a free copy of a group of its configuration (or of a new
// group when every group of it is full), or a free slot for a configuration
// with no batched form.  False: it has to wait.
bool place_request(nn4mg_server *S, const Request &q, double t_start)
{
    if (batchable(S, q.cfg)) {
        for (Group *g : S->groups) {
            if (!same_config(g->cfg, q.cfg)) continue;
            for (size_t i = 0; i < g->m.size(); ++i)
                if (g->m[i].state == M_FREE) {
                    admit_member(S, g, (int)i, q, t_start);
                    return true;
                }
        }
        if (Group *g = create_group(S, q.cfg)) {
            admit_member(S, g, 0, q, t_start);
            return true;
        }
        if (batchable(S, q.cfg)) return false;  // memory is short right now
    }
    for (Slot &sl : S->slots)
        if (!sl.busy) {
            sl.req = q;
            sl.busy = true;
            sl.phase = 0;
            sl.t_start = t_start;
            return true;
        }
    return false;
}

// A group whose batch completed: members whose solve ended get their
// projection and state copy-back enqueued (FINISH); the others have their
// next batch planned.
bool poll_group(nn4mg_server *S, Group *g)
{
    if (!g->in_flight) return false;
    const hipError_t e = hipEventQuery(g->ev);
    if (e == hipErrorNotReady) return false;
    g->in_flight = false;
    for (Member &mb : g->m) {
        if (mb.state != M_RUNNING) continue;
        if (mb.fresh) {  // started during the batch: its first batch is the next one
            mb.fresh = false;
            continue;
        }
        if (e != hipSuccess) {
            fail_member(S, g, mb, NN4MG_EDEVICE);
            continue;
        }
        if (!solve_after_header(mb.V)) continue;
        int rc = solve_finish_enqueue(mb.V, hier_xw(mb.V));
        if (!rc && hipMemcpyAsync(mb.req.x, hier_xw(mb.V), mb.req.n * sizeof(double), hipMemcpyDeviceToDevice,
                                  g->stream) != hipSuccess)
            rc = NN4MG_EDEVICE;
        if (!rc && hipEventRecord(mb.ev, g->stream) != hipSuccess) rc = NN4MG_EDEVICE;
        if (rc) {
            fail_member(S, g, mb, rc);
            continue;
        }
        mb.state = M_FINISH;
    }
    return true;
}

// Enqueue the next batch of an idle group with running members: as many
// cycles as the member closest to its end has planned (members that have not
// run a batch yet have no estimate and do not shorten it), over the copies up
// to the last running one, then every running member's state header, then the
// group's event.
bool launch_group(nn4mg_server *S, Group *g)
{
    if (g->in_flight) return false;
    int n = kMaxBatchCycles, k = 0;
    for (size_t i = 0; i < g->m.size(); ++i) {
        const Member &mb = g->m[i];
        if (mb.state != M_RUNNING) continue;
        k = (int)i + 1;
        if (hier_started(mb.V) && hier_planned(mb.V) < n) n = hier_planned(mb.V);
    }
    if (k == 0) return false;
    if (n < 1) n = 1;
    int rc = batch_enqueue_cycles(g->G, n, k);
    for (Member &mb : g->m) {
        if (mb.state != M_RUNNING || rc) continue;
        hier_note_enqueued(mb.V, n);
        rc = solve_header_copy(mb.V);
    }
    if (!rc && hipEventRecord(g->ev, g->stream) != hipSuccess) rc = NN4MG_EDEVICE;
    if (rc) {
        for (Member &mb : g->m)
            if (mb.state == M_RUNNING) fail_member(S, g, mb, rc);
        return true;
    }
    g->in_flight = true;
    return true;
}

int active_count(const nn4mg_server *S)
{
    int a = 0;
    for (const Slot &sl : S->slots) a += sl.busy ? 1 : 0;
    for (const Group *g : S->groups) a += g->busy();
    return a;
}

void worker_main(nn4mg_server *S)
{
    (void)hipSetDevice(S->device);
    while (true) {
        bool progress = false;
        for (Group *g : S->groups) {
            progress = poll_group(S, g) || progress;
            for (Member &mb : g->m) progress = advance_member(S, g, mb) || progress;
        }
        std::vector<Request> incoming;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            const int active = active_count(S);
            if (S->stop.load() && S->queue.empty() && active == 0) break;
            for (int free = S->max_active - active; free > 0 && !S->queue.empty(); --free) {
                incoming.push_back(S->queue.front());
                S->queue.pop_front();
            }
        }
        std::vector<Request> wait;
        for (const Request &q : incoming) {
            if (place_request(S, q, S->now_ms()))
                progress = true;
            else
                wait.push_back(q);
        }
        if (!wait.empty()) {
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto it = wait.rbegin(); it != wait.rend(); ++it) S->queue.push_front(*it);
        }
        for (Group *g : S->groups) progress = launch_group(S, g) || progress;
        for (Slot &sl : S->slots) progress = step_slot(S, sl) || progress;
        S->active_now.store(active_count(S));
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
    S->max_active = max_slots;
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
    if (active) *active = S->active_now.load();
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
    while (!S->groups.empty()) free_group(S, (int)S->groups.size() - 1);
    while (!S->residents.empty()) free_resident(S, (int)S->residents.size() - 1);
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    delete S;
    return NN4MG_OK;
}

}  // extern "C"
