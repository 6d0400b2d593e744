// dpd_server.cpp -- continuous-batching request server over the box and batch
// API of include/dpd.h, plus the few non-synchronising runtime calls of
// dpd_runtime.hpp.
//
// Requests are admitted in arrival order by HBM footprint: each needs
// dpd_workspace_bytes of its geometry, carved first-fit out of one
// caller-owned device pool, plus a slot.  Admitted requests keep their state
// resident; every pump runs one quantum of steps for all active requests as
// one batch per density class (one launch per kernel for all requests of
// a class, each class at its own launch shape) on the server stream.
// The host does not wait for that quantum: requests that finish with it have
// their results copied to pinned host memory behind it on the same stream,
// and a later pump, once those copies are done, completes them and frees
// their memory; meanwhile new requests are set up on a second stream.  At
// most two quanta are in flight.  A request's result is the same bits whether
// it ran alone or in a mix: the batch computes every box exactly as it would
// alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "dpd.h"
#include "dpd_internal.hpp"
#include "dpd_runtime.hpp"
#include "pool_alloc.hpp"

namespace {

int sfail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return dpd::set_error(code, buf);
}

// Re-raise a box/batch error with its message.
int pass(int rc, const char* where)
{
    char msg[512];
    std::snprintf(msg, sizeof msg, "%s", dpd_last_error());
    return sfail(rc, "%s: %s", where, msg);
}

using dpd::align256;
using dpd::PoolAlloc;

// Pinned host blocks for results, reused by size (best fit).
struct PinnedPool {
    std::multimap<size_t, char*> free;
    std::vector<std::pair<char*, size_t>> all;

    char* take(size_t bytes)
    {
        auto it = free.lower_bound(bytes);
        if (it != free.end() && it->first <= 2 * bytes + (1u << 20)) {
            char* p = it->second;
            free.erase(it);
            return p;
        }
        char* p = nullptr;
        if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        all.emplace_back(p, bytes);
        return p;
    }
    void give(char* p)
    {
        for (const auto& a : all)
            if (a.first == p) {
                free.emplace(a.second, p);
                return;
            }
    }
    void release()
    {
        for (const auto& a : all) (void)hipHostFree(a.first);
        all.clear();
        free.clear();
    }
};

struct Req {
    uint64_t ticket = 0;
    dpd_geom geom{};
    dpd_params params{};
    uint64_t seed = 0;
    int64_t nsteps = 0;
    double init_kT = 0.0;
    uint64_t init_seed = 0;
    std::vector<float> pos, vel;          // initial state (empty: generated on the device)
    size_t bytes = 0, off = 0;
    bool has_block = false;
    dpd_box box = nullptr;
    int64_t done_steps = 0;
    int32_t status = DPD_EAGAIN;
    dpd_stats stats{};
    // final state (id order) and device statistics, copied to pinned host
    // memory behind the request's last quantum
    char* out = nullptr;
    float* out_pos = nullptr;
    float* out_vel = nullptr;
    dpd::DevStats* out_stats = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

// Requests whose last quantum has been enqueued, with the event that passes
// when their result copies are done.
struct Retiring {
    hipEvent_t done = nullptr;
    std::vector<Req*> reqs;
};

}  // namespace

struct dpd_server_s {
    char* pool = nullptr;
    size_t pool_bytes = 0;
    int max_slots = 0;
    static constexpr int kClasses = 2;  // dilute (rho <= 4.5) and dense fluids: each its own batch
    hipStream_t stream = nullptr;       // the caller's: quanta and result copies
    hipStream_t admin = nullptr;        // setting up admitted requests
    PoolAlloc alloc;
    size_t batch_off[kClasses] = {0, 0}, batch_bytes = 0;   // batch tables, reserved at the pool start
    std::deque<Req*> queue;
    std::vector<Req*> active;
    std::deque<Retiring> retiring;
    int n_retiring = 0;
    std::vector<hipEvent_t> spare_events;
    hipEvent_t quantum_done[2] = {nullptr, nullptr};
    bool quantum_used[2] = {false, false};
    int quantum_next = 0;
    PinnedPool pinned;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    dpd_batch batch[kClasses] = {nullptr, nullptr};
    bool members_changed = true;
    std::chrono::steady_clock::time_point t0;
    int64_t steps_run = 0;                        // particle-steps completed
    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

hipEvent_t take_event(dpd_server_s* s)
{
    if (!s->spare_events.empty()) {
        hipEvent_t e = s->spare_events.back();
        s->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void free_block(dpd_server_s* s, Req* r)
{
    if (r->has_block) {
        s->alloc.release(r->off, r->bytes);
        r->has_block = false;
    }
    r->pos.clear();
    r->pos.shrink_to_fit();
    r->vel.clear();
    r->vel.shrink_to_fit();
}

// Retire a request that never ran or failed (no copies in flight): destroy
// its box and free its memory at once.
int retire_now(dpd_server_s* s, Req* r, int status)
{
    r->status = status;
    r->t_done = s->now();
    if (r->box) {
        dpd_destroy(r->box);
        r->box = nullptr;
    }
    free_block(s, r);
    return DPD_OK;
}

// Queue the result copies of a request whose last quantum was just enqueued.
int retire_enqueue(dpd_server_s* s, Req* r, Retiring& grp)
{
    const size_t n3 = (size_t)r->geom.n * 3;
    const size_t state_bytes = (n3 * sizeof(float) + 255) & ~(size_t)255;
    r->out = s->pinned.take(2 * state_bytes + sizeof(dpd::DevStats));
    if (!r->out) return sfail(DPD_ENOMEM, "dpd_server: pinned host allocation failed");
    r->out_pos = (float*)r->out;
    r->out_vel = (float*)(r->out + state_bytes);
    r->out_stats = (dpd::DevStats*)(r->out + 2 * state_bytes);
    const int rc = dpd::box_enqueue_results(r->box, r->out_pos, r->out_vel, r->out_stats);
    if (rc) return pass(rc, "dpd_server: results");
    grp.reqs.push_back(r);
    return DPD_OK;
}

// Complete the retiring groups whose copies are done (all of them when
// `wait`): statistics, status, completion time; the box and its memory are
// released.  Groups complete in order.
int reap(dpd_server_s* s, bool wait)
{
    while (!s->retiring.empty()) {
        Retiring& g = s->retiring.front();
        const hipError_t e = wait ? hipEventSynchronize(g.done) : hipEventQuery(g.done);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return sfail(DPD_EDEVICE, "dpd_server: %s", hipGetErrorString(e));
        const double t = s->now();
        for (Req* r : g.reqs) {
            dpd::stats_from_device(*r->out_stats, &r->stats);
            r->status = r->stats.nonfinite ? DPD_ENONFINITE : DPD_OK;
            r->t_done = t;
            dpd::box_release(r->box);      // its last work is behind the event
            r->box = nullptr;
            free_block(s, r);
        }
        s->n_retiring -= (int)g.reqs.size();
        s->spare_events.push_back(g.done);
        s->retiring.pop_front();
    }
    return DPD_OK;
}

// Density class of a request: the default launch shapes differ at rho 4.5
// (one launch has one shape, so the two classes are batched apart).
int density_class(const Req* r)
{
    const double nc = (double)r->geom.cells[0] * r->geom.cells[1] * r->geom.cells[2];
    return (double)r->geom.n / nc <= 4.5 ? 0 : 1;
}

// Create the request's box in its pool block and load its state, on the
// setup stream; then later work of the box goes to the server stream.
int materialise(dpd_server_s* s, Req* r)
{
    dpd_box b = nullptr;
    int rc = dpd_create(&r->geom, s->pool + r->off, r->bytes, (void*)s->admin, &b);
    if (rc) return pass(rc, "dpd_server: create");
    r->box = b;
    if ((rc = dpd_set_params(b, &r->params)) || (rc = dpd_set_seed(b, r->seed))) return pass(rc, "dpd_server: setup");
    // every box of a class batch at one launch shape, the fastest of a sweep
    // over batches of the served mix's boxes (MI355X): 6x6x4 cells for the
    // dilute class, 4x4x2 for the dense one, 1024 threads each (a fluid too
    // dense for that shape's LDS keeps the box's own default)
    static const int32_t kTile[dpd_server_s::kClasses][3] = {{6, 6, 4}, {4, 4, 2}};
    if (dpd_set_force_threads(b, 1024) != DPD_OK || dpd_set_tile(b, kTile[density_class(r)]) != DPD_OK) {
        static const int32_t kDefault[3] = {0, 0, 0};
        if ((rc = dpd_set_force_threads(b, 0)) || (rc = dpd_set_tile(b, kDefault))) return pass(rc, "dpd_server: tile");
    }
    if (!r->pos.empty() || r->geom.n == 0)
        rc = dpd_set_state(b, r->pos.empty() ? nullptr : r->pos.data(), r->vel.empty() ? nullptr : r->vel.data(),
                           DPD_HOST);
    else
        rc = dpd_init_random(b, r->init_kT, r->init_seed);
    if (rc) return pass(rc, "dpd_server: state");
    // the setup calls above have synchronised the setup stream
    return dpd::box_set_stream(b, s->stream);
}

void admit(dpd_server_s* s)
{
    while (!s->queue.empty() && (int)s->active.size() + s->n_retiring < s->max_slots) {
        Req* r = s->queue.front();
        size_t off = 0;
        if (!s->alloc.alloc(r->bytes, &off)) break;          // arrival order: wait for memory
        s->queue.pop_front();
        r->off = off;
        r->has_block = true;
        r->t_admit = s->now();
        const int rc = materialise(s, r);
        if (rc != DPD_OK) {
            retire_now(s, r, rc);
            continue;
        }
        if (r->nsteps == 0) {
            retire_now(s, r, DPD_OK);
            continue;
        }
        s->active.push_back(r);
        s->members_changed = true;
    }
}

}  // namespace

extern "C" {

int dpd_server_create(void* dev_pool, size_t pool_bytes, int32_t max_slots, void* hip_stream, dpd_server* out)
{
    if (!out) return sfail(DPD_EINVAL, "dpd_server_create: null output");
    *out = nullptr;
    if (!dev_pool || ((uintptr_t)dev_pool & 255)) return sfail(DPD_EINVAL, "dpd_server_create: pool null or misaligned");
    if (max_slots < 1 || max_slots > 4096) return sfail(DPD_EINVAL, "dpd_server_create: max_slots must be in 1..4096");
    size_t tb = 0;
    if (dpd_batch_workspace_bytes(max_slots, &tb)) return pass(DPD_EINVAL, "dpd_server_create");
    tb = align256(tb);
    if (pool_bytes <= dpd_server_s::kClasses * tb)
        return sfail(DPD_ENOMEM, "dpd_server_create: pool smaller than the batch tables");
    dpd_server_s* s = new (std::nothrow) dpd_server_s();
    if (!s) return sfail(DPD_ENOMEM, "dpd_server_create: host allocation failed");
    hipError_t e = hipStreamCreateWithFlags(&s->admin, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->quantum_done[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipEvent_t q : s->quantum_done)
            if (q) (void)hipEventDestroy(q);
        if (s->admin) (void)hipStreamDestroy(s->admin);
        delete s;
        return sfail(DPD_EDEVICE, "dpd_server_create: %s", hipGetErrorString(e));
    }
    s->pool = (char*)dev_pool;
    s->pool_bytes = pool_bytes;
    s->max_slots = max_slots;
    s->stream = (hipStream_t)hip_stream;
    s->alloc.reset(pool_bytes);
    for (int c = 0; c < dpd_server_s::kClasses; ++c) s->alloc.alloc(tb, &s->batch_off[c]);
    s->batch_bytes = tb;
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return DPD_OK;
}

int dpd_server_submit(dpd_server s, const dpd_request* q, uint64_t* ticket)
{
    if (!s || !q || !ticket) return sfail(DPD_EINVAL, "dpd_server_submit: null argument");
    size_t bytes = 0;
    if (dpd_workspace_bytes(&q->geom, &bytes)) return pass(DPD_EINVAL, "dpd_server_submit: geometry");
    if (q->nsteps < 0) return sfail(DPD_EINVAL, "dpd_server_submit: nsteps < 0");
    if (align256(bytes) > s->pool_bytes - dpd_server_s::kClasses * s->batch_bytes)
        return sfail(DPD_ENOMEM, "dpd_server_submit: request needs %zu bytes, more than the whole pool", bytes);
    if ((q->pos_n3 == nullptr) != (q->vel_n3 == nullptr))
        return sfail(DPD_EINVAL, "dpd_server_submit: give both pos and vel, or neither");
    auto r = std::unique_ptr<Req>(new (std::nothrow) Req());
    if (!r) return sfail(DPD_ENOMEM, "dpd_server_submit: host allocation failed");
    r->ticket = s->next_ticket++;
    r->geom = q->geom;
    r->params = q->params;
    r->seed = q->seed;
    r->nsteps = q->nsteps;
    r->init_kT = q->init_kT;
    r->init_seed = q->init_seed;
    r->bytes = bytes;
    if (q->pos_n3) {
        r->pos.assign(q->pos_n3, q->pos_n3 + (size_t)q->geom.n * 3);
        r->vel.assign(q->vel_n3, q->vel_n3 + (size_t)q->geom.n * 3);
    }
    r->t_submit = s->now();
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
    return DPD_OK;
}

int dpd_server_pump(dpd_server s, int32_t quantum_steps, int32_t* ran_steps)
{
    if (!s) return sfail(DPD_EINVAL, "dpd_server_pump: null server");
    if (quantum_steps < 1) return sfail(DPD_EINVAL, "dpd_server_pump: quantum_steps < 1");
    if (ran_steps) *ran_steps = 0;
    int rc = reap(s, false);
    if (rc) return rc;
    admit(s);
    if (s->active.empty()) return reap(s, s->queue.empty());   // nothing to run: let the last copies finish
    // a quantum never runs a request past its end
    int64_t q = quantum_steps;
    for (Req* r : s->active) q = std::min(q, r->nsteps - r->done_steps);
    std::vector<dpd_box> boxes[dpd_server_s::kClasses];
    for (Req* r : s->active) boxes[density_class(r)].push_back(r->box);
    for (int c = 0; c < dpd_server_s::kClasses; ++c) {
        if (boxes[c].empty()) continue;
        if (s->members_changed || !s->batch[c]) {
            if (!s->batch[c])
                rc = dpd_batch_create(boxes[c].data(), (int32_t)boxes[c].size(), s->pool + s->batch_off[c],
                                      s->batch_bytes, (void*)s->stream, &s->batch[c]);
            else
                rc = dpd::batch_set_boxes(s->batch[c], boxes[c].data(), (int32_t)boxes[c].size());
            if (rc) return pass(rc, "dpd_server_pump: batch");
        }
        rc = dpd_batch_step(s->batch[c], q);
        if (rc) return pass(rc, "dpd_server_pump: step");
    }
    s->members_changed = false;
    if (ran_steps) *ran_steps = (int32_t)q;
    // requests that end with this quantum: their results are copied out
    // behind it, and a later pump completes them
    Retiring grp;
    std::vector<Req*> still;
    for (Req* r : s->active) {
        r->done_steps += q;
        s->steps_run += q * r->geom.n;
        if (r->done_steps < r->nsteps) {
            still.push_back(r);
            continue;
        }
        rc = retire_enqueue(s, r, grp);
        if (rc) return rc;
    }
    s->active.swap(still);
    if (!grp.reqs.empty()) {
        grp.done = take_event(s);
        if (!grp.done) return sfail(DPD_EDEVICE, "dpd_server_pump: event creation failed");
        if (hipEventRecord(grp.done, s->stream) != hipSuccess) return sfail(DPD_EDEVICE, "dpd_server_pump: event record");
        s->n_retiring += (int)grp.reqs.size();
        s->retiring.push_back(std::move(grp));
        s->members_changed = true;
    }
    // at most two quanta in flight: wait for the one before this
    const int k = s->quantum_next;
    s->quantum_next ^= 1;
    if (hipEventRecord(s->quantum_done[k], s->stream) != hipSuccess)
        return sfail(DPD_EDEVICE, "dpd_server_pump: event record");
    s->quantum_used[k] = true;
    if (s->quantum_used[k ^ 1] && hipEventSynchronize(s->quantum_done[k ^ 1]) != hipSuccess)
        return sfail(DPD_EDEVICE, "dpd_server_pump: quantum failed");
    return reap(s, false);
}

int dpd_server_poll(dpd_server s, uint64_t ticket, dpd_result* res, float* pos_n3, float* vel_n3)
{
    if (!s || !res) return sfail(DPD_EINVAL, "dpd_server_poll: null argument");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(DPD_ENOTFOUND, "dpd_server_poll: unknown ticket %llu", (unsigned long long)ticket);
    Req* r = it->second.get();
    if (r->status == DPD_EAGAIN) {
        const int rc = reap(s, false);
        if (rc) return rc;
        if (r->status == DPD_EAGAIN) return DPD_EAGAIN;
    }
    std::memset(res, 0, sizeof *res);
    res->stats = r->stats;
    res->status = r->status;
    res->t_submit = r->t_submit;
    res->t_admit = r->t_admit;
    res->t_done = r->t_done;
    const size_t bytes = (size_t)r->geom.n * 3 * sizeof(float);
    if (r->out) {
        if (pos_n3 && bytes) std::memcpy(pos_n3, r->out_pos, bytes);
        if (vel_n3 && bytes) std::memcpy(vel_n3, r->out_vel, bytes);
        s->pinned.give(r->out);
        r->out = nullptr;
    }
    s->reqs.erase(it);
    return DPD_OK;
}

int dpd_server_counts(dpd_server s, int32_t* queued, int32_t* active, int64_t* particle_steps)
{
    if (!s) return sfail(DPD_EINVAL, "dpd_server_counts: null server");
    if (queued) *queued = (int32_t)s->queue.size();
    if (active) *active = (int32_t)s->active.size() + s->n_retiring;
    if (particle_steps) *particle_steps = s->steps_run;
    return DPD_OK;
}

double dpd_server_clock(dpd_server s) { return s ? s->now() : 0.0; }

int dpd_server_destroy(dpd_server s)
{
    if (!s) return DPD_OK;
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->admin);
    (void)reap(s, true);
    for (dpd_batch b : s->batch)
        if (b) dpd_batch_destroy(b);
    for (Req* r : s->active)
        if (r->box) dpd::box_release(r->box);
    for (Retiring& g : s->retiring) {
        for (Req* r : g.reqs)
            if (r->box) dpd::box_release(r->box);
        (void)hipEventDestroy(g.done);
    }
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->quantum_done)
        if (e) (void)hipEventDestroy(e);
    s->pinned.release();
    (void)hipStreamDestroy(s->admin);
    delete s;
    return DPD_OK;
}

}  // extern "C"
