// dpd_server.cpp -- continuous-batching request server over the box and batch
// API of include/dpd.h (it uses nothing below that API).
//
// Requests are admitted in arrival order by HBM footprint: each needs
// dpd_workspace_bytes of its geometry, carved first-fit out of one
// caller-owned device pool, plus a slot.  Admitted requests keep their state
// resident; every pump runs one quantum of steps for all active requests as
// one batch (one launch per kernel for all of them), retires the ones that
// finished (results copied to host memory, pool block freed) and admits
// queued requests into the freed memory and slots.  A request's result is
// the same bits whether it ran alone or in a mix: the batch computes every
// box exactly as it would alone.
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
    std::vector<float> out_pos, out_vel;  // final state, id order
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct dpd_server_s {
    char* pool = nullptr;
    size_t pool_bytes = 0;
    int max_slots = 0;
    hipStream_t stream = nullptr;
    PoolAlloc alloc;
    size_t batch_off = 0, batch_bytes = 0;       // batch tables, reserved at the pool start
    std::deque<Req*> queue;
    std::vector<Req*> active;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    dpd_batch batch = nullptr;
    bool members_changed = true;
    std::chrono::steady_clock::time_point t0;
    int64_t steps_run = 0;                        // particle-steps completed
    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

int retire(dpd_server_s* s, Req* r, int status)
{
    r->status = status;
    r->t_done = s->now();
    if (r->box) {
        const int64_t n = r->geom.n;
        if (status == DPD_OK || status == DPD_ENONFINITE) {
            r->out_pos.resize((size_t)n * 3);
            r->out_vel.resize((size_t)n * 3);
            int rc = dpd_get_stats(r->box, &r->stats);
            if (rc != DPD_OK && rc != DPD_ENONFINITE) r->status = rc;
            if (rc == DPD_ENONFINITE) r->status = rc;
            if (n > 0) {
                if (dpd_read(r->box, DPD_POS, r->out_pos.data(), DPD_HOST) != DPD_OK ||
                    dpd_read(r->box, DPD_VEL, r->out_vel.data(), DPD_HOST) != DPD_OK)
                    r->status = DPD_EDEVICE;
            }
        }
        dpd_destroy(r->box);
        r->box = nullptr;
    }
    if (r->has_block) {
        s->alloc.release(r->off, r->bytes);
        r->has_block = false;
    }
    r->pos.clear();
    r->pos.shrink_to_fit();
    r->vel.clear();
    r->vel.shrink_to_fit();
    return DPD_OK;
}

// Create the request's box in its pool block and load its state.
int materialise(dpd_server_s* s, Req* r)
{
    dpd_box b = nullptr;
    int rc = dpd_create(&r->geom, s->pool + r->off, r->bytes, (void*)s->stream, &b);
    if (rc) return pass(rc, "dpd_server: create");
    r->box = b;
    if ((rc = dpd_set_params(b, &r->params)) || (rc = dpd_set_seed(b, r->seed))) return pass(rc, "dpd_server: setup");
    if (!r->pos.empty() || r->geom.n == 0)
        rc = dpd_set_state(b, r->pos.empty() ? nullptr : r->pos.data(), r->vel.empty() ? nullptr : r->vel.data(),
                           DPD_HOST);
    else
        rc = dpd_init_random(b, r->init_kT, r->init_seed);
    if (rc) return pass(rc, "dpd_server: state");
    return DPD_OK;
}

void admit(dpd_server_s* s)
{
    while (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
        Req* r = s->queue.front();
        size_t off = 0;
        if (!s->alloc.alloc(r->bytes, &off)) break;          // arrival order: wait for memory
        s->queue.pop_front();
        r->off = off;
        r->has_block = true;
        r->t_admit = s->now();
        const int rc = materialise(s, r);
        if (rc != DPD_OK) {
            retire(s, r, rc);
            continue;
        }
        if (r->nsteps == 0) {
            retire(s, r, DPD_OK);
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
    if (pool_bytes <= tb) return sfail(DPD_ENOMEM, "dpd_server_create: pool smaller than the batch tables");
    dpd_server_s* s = new (std::nothrow) dpd_server_s();
    if (!s) return sfail(DPD_ENOMEM, "dpd_server_create: host allocation failed");
    s->pool = (char*)dev_pool;
    s->pool_bytes = pool_bytes;
    s->max_slots = max_slots;
    s->stream = (hipStream_t)hip_stream;
    s->alloc.reset(pool_bytes);
    s->alloc.alloc(tb, &s->batch_off);
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
    if (align256(bytes) > s->pool_bytes - s->batch_bytes)
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
    admit(s);
    if (s->active.empty()) return DPD_OK;
    // a quantum never runs a request past its end
    int64_t q = quantum_steps;
    for (Req* r : s->active) q = std::min(q, r->nsteps - r->done_steps);
    if (s->members_changed || !s->batch) {
        if (s->batch) dpd_batch_destroy(s->batch);
        s->batch = nullptr;
        std::vector<dpd_box> boxes;
        for (Req* r : s->active) boxes.push_back(r->box);
        int rc = dpd_batch_create(boxes.data(), (int32_t)boxes.size(), s->pool + s->batch_off, s->batch_bytes,
                                  (void*)s->stream, &s->batch);
        if (rc) return pass(rc, "dpd_server_pump: batch");
        s->members_changed = false;
    }
    int rc = dpd_batch_step(s->batch, q);
    if (rc) return pass(rc, "dpd_server_pump: step");
    if (ran_steps) *ran_steps = (int32_t)q;
    std::vector<Req*> still;
    for (Req* r : s->active) {
        r->done_steps += q;
        s->steps_run += q * r->geom.n;
        if (r->done_steps >= r->nsteps) {
            retire(s, r, DPD_OK);
            s->members_changed = true;
        } else {
            still.push_back(r);
        }
    }
    s->active.swap(still);
    if (s->members_changed) admit(s);
    return DPD_OK;
}

int dpd_server_poll(dpd_server s, uint64_t ticket, dpd_result* res, float* pos_n3, float* vel_n3)
{
    if (!s || !res) return sfail(DPD_EINVAL, "dpd_server_poll: null argument");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(DPD_ENOTFOUND, "dpd_server_poll: unknown ticket %llu", (unsigned long long)ticket);
    Req* r = it->second.get();
    if (r->status == DPD_EAGAIN) return DPD_EAGAIN;
    std::memset(res, 0, sizeof *res);
    res->stats = r->stats;
    res->status = r->status;
    res->t_submit = r->t_submit;
    res->t_admit = r->t_admit;
    res->t_done = r->t_done;
    if (pos_n3 && !r->out_pos.empty()) std::memcpy(pos_n3, r->out_pos.data(), r->out_pos.size() * sizeof(float));
    if (vel_n3 && !r->out_vel.empty()) std::memcpy(vel_n3, r->out_vel.data(), r->out_vel.size() * sizeof(float));
    s->reqs.erase(it);
    return DPD_OK;
}

int dpd_server_counts(dpd_server s, int32_t* queued, int32_t* active, int64_t* particle_steps)
{
    if (!s) return sfail(DPD_EINVAL, "dpd_server_counts: null server");
    if (queued) *queued = (int32_t)s->queue.size();
    if (active) *active = (int32_t)s->active.size();
    if (particle_steps) *particle_steps = s->steps_run;
    return DPD_OK;
}

double dpd_server_clock(dpd_server s) { return s ? s->now() : 0.0; }

int dpd_server_destroy(dpd_server s)
{
    if (!s) return DPD_OK;
    if (s->batch) dpd_batch_destroy(s->batch);
    for (Req* r : s->active)
        if (r->box) dpd_destroy(r->box);
    (void)hipStreamSynchronize(s->stream);
    delete s;
    return DPD_OK;
}

}  // extern "C"
