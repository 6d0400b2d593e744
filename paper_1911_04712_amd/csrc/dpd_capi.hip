// dpd_capi.hip -- host runtime behind include/dpd.h: box state, workspace
// layout, validation, the step pipeline and its HIP-graph capture.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "dpd.h"
#include "dpd_internal.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(DPD_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool geom_ok(const dpd_geom* g)
{
    if (!g || g->reserved != 0) return false;
    for (int k = 0; k < 3; ++k)
        if (g->cells[k] < 3 || g->cells[k] > 4096) return false;
    const int64_t nc = (int64_t)g->cells[0] * g->cells[1] * g->cells[2];
    return g->n >= 0 && g->n <= (int64_t(1) << 30) && nc < (int64_t(1) << 31) - 1;
}

// Spacing of FP32 numbers at L_max: 2^(floor(log2 L_max) - 23).
double grid_of(const dpd_geom* g)
{
    int lmax = g->cells[0];
    for (int k = 1; k < 3; ++k) lmax = g->cells[k] > lmax ? g->cells[k] : lmax;
    int e = 0;
    while ((2 << e) <= lmax) ++e;   // 2^e <= lmax < 2^(e+1)
    return std::ldexp(1.0, e - 23);
}

}  // namespace

namespace dpd {

Layout make_layout(int64_t n, int64_t nc)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes > 0 ? bytes : 1); return o; };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    L.pos_a = take(nn * sizeof(float4));
    L.vel_a = take(nn * sizeof(float4));
    L.pos_b = take(nn * sizeof(float4));
    L.vel_b = take(nn * sizeof(float4));
    L.force = take(nn * sizeof(float4));
    L.keyslot = take(nn * sizeof(int2));
    L.perm = take(nn * sizeof(int));
    L.out = take(nn * 3 * sizeof(float));
    L.count = take((size_t)nc * sizeof(int));
    L.cell_start = take((size_t)(nc + 1) * sizeof(int));
    L.bsum = take((size_t)((nc + kScanChunk - 1) / kScanChunk) * sizeof(int));
    L.partials = take((size_t)kIntegrateMaxBlocks * kPartials * sizeof(double));
    L.profile = take((size_t)kProfileMaxBins * 2 * sizeof(long long));
    L.stats = take(sizeof(DevStats));
    L.flags = take(4 * sizeof(int));
    L.total = off;
    return L;
}

}  // namespace dpd

struct dpd_box_s {
    dpd_geom geom{};
    int n = 0;
    int nc = 0;
    int cells[3] = {0, 0, 0};
    float L[3] = {0, 0, 0};
    double q = 0.0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    dpd::Layout lay{};
    float4 *pos_a = nullptr, *vel_a = nullptr, *pos_b = nullptr, *vel_b = nullptr, *force = nullptr;
    int2* keyslot = nullptr;
    int* perm = nullptr;
    float* out = nullptr;
    int *count = nullptr, *cell_start = nullptr, *bsum = nullptr, *flags = nullptr;
    double* partials = nullptr;
    long long* profile = nullptr;
    dpd::DevStats* st = nullptr;

    dpd_params params{};
    bool have_params = false;
    uint64_t seed = 0;
    bool have_seed = false;
    bool have_state = false;
    bool keys_valid = false;   // keyslot/count describe pos_a
    bool binned = false;       // pos_b/vel_b/cell_start describe the current state
    bool have_force = false;   // force/pos_b hold the last step's forces

    // pair-force tiling
    int tile_req[3] = {0, 0, 0};
    dpd::TileConst tc{};

    // captured multi-step graph
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;
    bool graph_dirty = true;
};

namespace {

constexpr int kGraphSteps = 8;

dpd::ForceConst force_const(const dpd_box_s* b)
{
    dpd::ForceConst fc{};
    const dpd_params& p = b->params;
    fc.pc.a = (float)p.a;
    fc.pc.gamma = (float)p.gamma;
    fc.pc.sig_rdt = (float)(std::sqrt(2.0 * p.gamma * p.kT) / std::sqrt(p.dt));
    fc.pc.k0 = (uint32_t)b->seed;
    fc.pc.k1 = (uint32_t)(b->seed >> 32);
    for (int k = 0; k < 3; ++k) {
        fc.L[k] = b->L[k];
        fc.cells[k] = b->cells[k];
    }
    fc.body_f = (float)p.body_f;
    fc.flow_axis = p.flow_axis;
    fc.grad_axis = p.grad_axis;
    fc.half_grad = 0.5f * b->L[p.grad_axis];
    return fc;
}

dpd::StepConst step_const(const dpd_box_s* b)
{
    dpd::StepConst sc{};
    const dpd_params& p = b->params;
    sc.dt = (float)p.dt;
    sc.dtm = (float)(p.dt / p.mass);
    sc.half_dtm = (float)(0.5 * p.dt / p.mass);
    sc.q = (float)b->q;
    sc.inv_q = (float)(1.0 / b->q);
    for (int k = 0; k < 3; ++k) {
        sc.L[k] = b->L[k];
        sc.cells[k] = b->cells[k];
    }
    sc.flow_axis = p.flow_axis;
    sc.grad_axis = p.grad_axis;
    sc.nbins = p.profile_bins;
    sc.grad_scale = (float)((double)p.profile_bins / (double)b->cells[p.grad_axis]);
    sc.mass = p.mass;
    sc.inv_dof = b->n >= 2 ? 1.0 / (3.0 * (double)(b->n - 1)) : 0.0;
    const double vol = (double)b->cells[0] * b->cells[1] * b->cells[2];
    sc.inv_vol = 1.0 / vol;
    sc.rho = (double)b->n / vol;
    return sc;
}

// Binning of pos_a into pos_b/vel_b + cell_start (keys must be valid).
hipError_t enqueue_bin(dpd_box_s* b, hipStream_t s)
{
    return dpd::launch_bin(b->keyslot, b->pos_a, b->vel_a, b->n, b->nc, b->count, b->bsum, b->cell_start, b->perm,
                           b->pos_b, b->vel_b, s);
}

// Default cell tile of the LDS force kernel (measured on MI355X): 8x4x4
// cells at solvent densities up to 4.5, 3x3x3 above; both keep two
// workgroups' LDS per CU.
void choose_tile(dpd_box_s* b)
{
    int t[3] = {b->tile_req[0], b->tile_req[1], b->tile_req[2]};
    if (t[0] <= 0) {
        const double rho = b->nc > 0 ? (double)b->n / (double)b->nc : 0.0;
        const bool dilute = rho <= 4.5;
        t[0] = dilute ? 8 : 3;
        t[1] = dilute ? 4 : 3;
        t[2] = dilute ? 4 : 3;
    }
    b->tc = dpd::make_tile_const(b->cells, b->n, t, 0, 0);
}

hipError_t enqueue_force(dpd_box_s* b, const dpd::ForceConst& fc, hipStream_t s)
{
    if (b->params.flags & DPD_FLAG_REFERENCE_FORCE)
        return dpd::launch_force_gather(b->pos_b, b->vel_b, b->cell_start, b->n, fc, &b->st->step, b->force,
                                        &b->st->nonfinite, s);
    return dpd::launch_force_tiled(b->pos_b, b->vel_b, b->cell_start, b->n, fc, b->tc, &b->st->step, b->force,
                                   &b->st->nonfinite, s);
}

// Forces on the binned state and the integrate step back into pos_a/vel_a.
hipError_t enqueue_force_integrate(dpd_box_s* b, hipStream_t s)
{
    const dpd::ForceConst fc = force_const(b);
    hipError_t e = enqueue_force(b, fc, s);
    if (e != hipSuccess) return e;
    if (b->params.flags & DPD_FLAG_VIRIAL) {
        e = dpd::launch_virial(b->pos_b, b->cell_start, b->n, fc, b->st, s);
        if (e != hipSuccess) return e;
    }
    const dpd::StepConst sc = step_const(b);
    return dpd::launch_integrate(b->pos_b, b->vel_b, b->force, b->n, sc, b->pos_a, b->vel_a, b->count, b->keyslot,
                                 b->partials, b->profile, b->st, s);
}

int rebuild_graph(dpd_box_s* b)
{
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < kGraphSteps && e == hipSuccess; ++k) {
        e = enqueue_bin(b, b->cap_stream);
        if (e == hipSuccess) e = enqueue_force_integrate(b, b->cap_stream);
    }
    hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(DPD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(DPD_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    b->graph_steps = kGraphSteps;
    b->graph_dirty = false;
    return DPD_OK;
}

int sync_box(dpd_box_s* b)
{
    HIPCHK(hipStreamSynchronize(b->stream));
    return DPD_OK;
}

hipMemcpyKind kind_to(int where) { return where == DPD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

}  // namespace

extern "C" {

const char* dpd_last_error(void) { return g_err; }

int dpd_position_grid(const dpd_geom* geom, double* q)
{
    if (!geom_ok(geom) || !q) return fail(DPD_EINVAL, "dpd_position_grid: invalid geometry or null output");
    *q = grid_of(geom);
    return DPD_OK;
}

int dpd_workspace_bytes(const dpd_geom* geom, size_t* bytes)
{
    if (!geom_ok(geom) || !bytes) return fail(DPD_EINVAL, "dpd_workspace_bytes: invalid geometry or null output");
    const int64_t nc = (int64_t)geom->cells[0] * geom->cells[1] * geom->cells[2];
    *bytes = dpd::make_layout(geom->n, nc).total;
    return DPD_OK;
}

int dpd_create(const dpd_geom* geom, void* dev_ws, size_t ws_bytes, void* hip_stream, dpd_box* out)
{
    if (!out) return fail(DPD_EINVAL, "dpd_create: null output");
    *out = nullptr;
    if (!geom_ok(geom)) return fail(DPD_EINVAL, "dpd_create: invalid geometry (cells >= 3, 0 <= n <= 2^30)");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(DPD_EINVAL, "dpd_create: workspace null or not 256-byte aligned");
    const int64_t nc = (int64_t)geom->cells[0] * geom->cells[1] * geom->cells[2];
    const dpd::Layout lay = dpd::make_layout(geom->n, nc);
    if (ws_bytes < lay.total)
        return fail(DPD_ENOMEM, "dpd_create: workspace of %zu bytes, %zu needed", ws_bytes, lay.total);
    dpd_box_s* b = new (std::nothrow) dpd_box_s();
    if (!b) return fail(DPD_ENOMEM, "dpd_create: host allocation failed");
    b->geom = *geom;
    b->n = (int)geom->n;
    b->nc = (int)nc;
    for (int k = 0; k < 3; ++k) {
        b->cells[k] = geom->cells[k];
        b->L[k] = (float)geom->cells[k];
    }
    b->q = grid_of(geom);
    b->stream = (hipStream_t)hip_stream;
    b->ws = (char*)dev_ws;
    b->lay = lay;
    b->pos_a = (float4*)(b->ws + lay.pos_a);
    b->vel_a = (float4*)(b->ws + lay.vel_a);
    b->pos_b = (float4*)(b->ws + lay.pos_b);
    b->vel_b = (float4*)(b->ws + lay.vel_b);
    b->force = (float4*)(b->ws + lay.force);
    b->keyslot = (int2*)(b->ws + lay.keyslot);
    b->perm = (int*)(b->ws + lay.perm);
    b->out = (float*)(b->ws + lay.out);
    b->count = (int*)(b->ws + lay.count);
    b->cell_start = (int*)(b->ws + lay.cell_start);
    b->bsum = (int*)(b->ws + lay.bsum);
    b->partials = (double*)(b->ws + lay.partials);
    b->profile = (long long*)(b->ws + lay.profile);
    b->st = (dpd::DevStats*)(b->ws + lay.stats);
    b->flags = (int*)(b->ws + lay.flags);
    choose_tile(b);
    hipError_t e = dpd::force_tiled_prepare(b->tc);
    if (e == hipSuccess) e = dpd::launch_fill_i32(b->count, 0, nc, b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32((int*)b->st, 0, (int64_t)(sizeof(dpd::DevStats) / 4), b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32((int*)b->profile, 0, (int64_t)dpd::kProfileMaxBins * 4, b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32(b->flags, 0, 4, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return fail(DPD_EDEVICE, "dpd_create: %s", hipGetErrorString(e));
    }
    *out = b;
    return DPD_OK;
}

int dpd_set_params(dpd_box b, const dpd_params* p)
{
    if (!b || !p) return fail(DPD_EINVAL, "dpd_set_params: null argument");
    const double vals[6] = {p->a, p->gamma, p->kT, p->dt, p->mass, p->body_f};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(DPD_EINVAL, "dpd_set_params: non-finite parameter");
    if (!(p->dt > 0.0) || !(p->mass > 0.0) || p->gamma < 0.0 || p->kT < 0.0)
        return fail(DPD_EINVAL, "dpd_set_params: need dt > 0, mass > 0, gamma >= 0, kT >= 0");
    if (p->flow_axis < 0 || p->flow_axis > 2 || p->grad_axis < 0 || p->grad_axis > 2 || p->flow_axis == p->grad_axis)
        return fail(DPD_EINVAL, "dpd_set_params: flow_axis and grad_axis must be distinct axes in 0..2");
    if (p->profile_bins < 0 || p->profile_bins > dpd::kProfileMaxBins)
        return fail(DPD_EINVAL, "dpd_set_params: profile_bins must be in [0, %d]", dpd::kProfileMaxBins);
    if (p->flags & ~(DPD_FLAG_VIRIAL | DPD_FLAG_REFERENCE_FORCE)) return fail(DPD_EINVAL, "dpd_set_params: unknown flags");
    const double sig = std::sqrt(2.0 * p->gamma * p->kT) / std::sqrt(p->dt);
    if (!std::isfinite(sig) || sig > 1e8 || std::fabs(p->a) > 1e8 || p->gamma > 1e8)
        return fail(DPD_EINVAL, "dpd_set_params: parameters out of the FP32 force range");
    b->params = *p;
    b->have_params = true;
    b->graph_dirty = true;
    return DPD_OK;
}

int dpd_set_tile(dpd_box b, const int32_t tile[3])
{
    if (!b || !tile) return fail(DPD_EINVAL, "dpd_set_tile: null argument");
    const bool dflt = tile[0] == 0 && tile[1] == 0 && tile[2] == 0;
    if (!dflt)
        for (int k = 0; k < 3; ++k)
            if (tile[k] < 1 || tile[k] > 16) return fail(DPD_EINVAL, "dpd_set_tile: edges must be in 1..16");
    for (int k = 0; k < 3; ++k) b->tile_req[k] = tile[k];
    choose_tile(b);
    if (b->tc.lds_bytes > 160 * 1024) {
        for (int k = 0; k < 3; ++k) b->tile_req[k] = 0;
        choose_tile(b);
        return fail(DPD_EINVAL, "dpd_set_tile: tile needs more LDS than a CU has");
    }
    HIPCHK(dpd::force_tiled_prepare(b->tc));
    b->graph_dirty = true;
    return DPD_OK;
}

int dpd_set_seed(dpd_box b, uint64_t seed)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_seed: null box");
    b->seed = seed;
    b->have_seed = true;
    b->graph_dirty = true;
    return DPD_OK;
}

int dpd_set_state(dpd_box b, const float* pos_n3, const float* vel_n3, int where)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_state: null box");
    if (where != DPD_HOST && where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_set_state: bad `where`");
    if (b->n > 0 && (!pos_n3 || !vel_n3)) return fail(DPD_EINVAL, "dpd_set_state: null array");
    b->have_state = b->keys_valid = b->binned = b->have_force = false;
    const float *pp = pos_n3, *vp = vel_n3;
    const size_t bytes = (size_t)b->n * 3 * sizeof(float);
    if (where == DPD_HOST && b->n > 0) {
        HIPCHK(hipMemcpyAsync(b->pos_b, pos_n3, bytes, hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->vel_b, vel_n3, bytes, hipMemcpyHostToDevice, b->stream));
        pp = (const float*)b->pos_b;
        vp = (const float*)b->vel_b;
    }
    HIPCHK(dpd::launch_fill_i32(b->flags, 0, 4, b->stream));
    HIPCHK(dpd::launch_fill_i32(b->count, 0, b->nc, b->stream));
    HIPCHK(dpd::launch_fill_i32((int*)b->st, 0, (int64_t)(sizeof(dpd::DevStats) / 4), b->stream));
    HIPCHK(dpd::launch_fill_i32((int*)b->profile, 0, (int64_t)dpd::kProfileMaxBins * 4, b->stream));
    HIPCHK(dpd::launch_load_state(pp, vp, b->n, b->pos_a, b->vel_a, (float)b->q, (float)(1.0 / b->q), b->L, b->flags,
                                  b->stream));
    HIPCHK(dpd::launch_keys(b->pos_a, b->n, b->cells, b->count, b->keyslot, b->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, b->flags, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (bad) return fail(DPD_EINVAL, "dpd_set_state: a position is outside [0, L) or a value is non-finite");
    b->have_state = true;
    b->keys_valid = true;
    return DPD_OK;
}

int dpd_build_cells(dpd_box b)
{
    if (!b) return fail(DPD_EINVAL, "dpd_build_cells: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_build_cells: no state loaded");
    if (b->binned) return DPD_OK;
    HIPCHK(enqueue_bin(b, b->stream));
    b->binned = true;
    b->keys_valid = false;
    b->have_force = false;
    return DPD_OK;
}

int dpd_step(dpd_box b, int64_t nsteps)
{
    if (!b) return fail(DPD_EINVAL, "dpd_step: null box");
    if (nsteps < 0) return fail(DPD_EINVAL, "dpd_step: nsteps < 0");
    if (!b->have_params || !b->have_seed || !b->have_state)
        return fail(DPD_ESTATE, "dpd_step: set params, seed and state first");
    if (nsteps == 0) return DPD_OK;
    int64_t left = nsteps;
    if (b->binned) {                      // first step reuses the existing cell list
        HIPCHK(enqueue_force_integrate(b, b->stream));
        b->binned = false;
        --left;
    }
    if (left >= kGraphSteps) {
        if (b->graph_dirty || !b->graph) {
            const int rc = rebuild_graph(b);
            if (rc) return rc;
        }
        while (left >= b->graph_steps) {
            HIPCHK(hipGraphLaunch(b->graph, b->stream));
            left -= b->graph_steps;
        }
    }
    for (; left > 0; --left) {
        HIPCHK(enqueue_bin(b, b->stream));
        HIPCHK(enqueue_force_integrate(b, b->stream));
    }
    b->keys_valid = true;
    b->have_force = true;
    return DPD_OK;
}

int dpd_profile_steps(dpd_box b, int64_t nsteps, double* ms_out)
{
    if (!b || !ms_out) return fail(DPD_EINVAL, "dpd_profile_steps: null argument");
    if (nsteps < 1) return fail(DPD_EINVAL, "dpd_profile_steps: nsteps < 1");
    if (!b->have_params || !b->have_seed || !b->have_state)
        return fail(DPD_ESTATE, "dpd_profile_steps: set params, seed and state first");
    hipEvent_t ev[5] = {};
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    double acc[4] = {0, 0, 0, 0};
    int rc = DPD_OK;
    for (int64_t k = 0; k < nsteps && rc == DPD_OK; ++k) {
        const dpd::ForceConst fc = force_const(b);
        const dpd::StepConst sc = step_const(b);
        hipError_t e = hipEventRecord(ev[0], b->stream);
        if (e == hipSuccess && !b->binned) e = enqueue_bin(b, b->stream);
        b->binned = false;
        if (e == hipSuccess) e = hipEventRecord(ev[1], b->stream);
        if (e == hipSuccess) e = enqueue_force(b, fc, b->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[2], b->stream);
        if (e == hipSuccess && (b->params.flags & DPD_FLAG_VIRIAL))
            e = dpd::launch_virial(b->pos_b, b->cell_start, b->n, fc, b->st, b->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[3], b->stream);
        if (e == hipSuccess)
            e = dpd::launch_integrate(b->pos_b, b->vel_b, b->force, b->n, sc, b->pos_a, b->vel_a, b->count,
                                      b->keyslot, b->partials, b->profile, b->st, b->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[4], b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
        for (int s = 0; s < 4 && e == hipSuccess; ++s) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, ev[s], ev[s + 1]);
            acc[s] += ms;
        }
        if (e != hipSuccess) rc = fail(DPD_EDEVICE, "dpd_profile_steps: %s", hipGetErrorString(e));
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    b->keys_valid = true;
    b->have_force = true;
    for (int s = 0; s < 4; ++s) ms_out[s] = acc[s] / (double)nsteps;
    return DPD_OK;
}

int dpd_read(dpd_box b, int what, float* out_n3, int where)
{
    if (!b) return fail(DPD_EINVAL, "dpd_read: null box");
    if (where != DPD_HOST && where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_read: bad `where`");
    if (b->n > 0 && !out_n3) return fail(DPD_EINVAL, "dpd_read: null output");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_read: no state loaded");
    float* dst = where == DPD_DEVICE ? out_n3 : b->out;
    switch (what) {
    case DPD_POS:
        HIPCHK(dpd::launch_to_rows(b->pos_a, nullptr, 0.0f, b->pos_a, b->n, dst, b->stream));
        break;
    case DPD_VEL:
        HIPCHK(dpd::launch_to_rows(b->vel_a, nullptr, 0.0f, b->pos_a, b->n, dst, b->stream));
        break;
    case DPD_FORCE:
        if (!b->have_force) return fail(DPD_ESTATE, "dpd_read: no forces (step first)");
        HIPCHK(dpd::launch_to_rows(b->force, nullptr, 0.0f, b->pos_b, b->n, dst, b->stream));
        break;
    case DPD_VEL_CENTRED:
        if (!b->have_force) return fail(DPD_ESTATE, "dpd_read: no forces (step first)");
        HIPCHK(dpd::launch_to_rows(b->vel_a, b->force, (float)(-0.5 * b->params.dt / b->params.mass), b->pos_b, b->n,
                                   dst, b->stream));
        break;
    default:
        return fail(DPD_EINVAL, "dpd_read: unknown quantity %d", what);
    }
    if (where == DPD_HOST && b->n > 0)
        HIPCHK(hipMemcpyAsync(out_n3, b->out, (size_t)b->n * 3 * sizeof(float), hipMemcpyDeviceToHost, b->stream));
    return sync_box(b);
}

int dpd_read_raw(dpd_box b, float* pos4, float* vel4, int32_t* cell_start, int where)
{
    if (!b) return fail(DPD_EINVAL, "dpd_read_raw: null box");
    if (where != DPD_HOST && where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_read_raw: bad `where`");
    if (!(b->binned || b->have_force)) return fail(DPD_ESTATE, "dpd_read_raw: no cell list (build_cells or step first)");
    const size_t pb = (size_t)b->n * sizeof(float4);
    if (pos4 && b->n > 0) HIPCHK(hipMemcpyAsync(pos4, b->pos_b, pb, kind_to(where), b->stream));
    if (vel4 && b->n > 0) HIPCHK(hipMemcpyAsync(vel4, b->vel_b, pb, kind_to(where), b->stream));
    if (cell_start)
        HIPCHK(hipMemcpyAsync(cell_start, b->cell_start, (size_t)(b->nc + 1) * sizeof(int), kind_to(where), b->stream));
    return sync_box(b);
}

int dpd_get_stats(dpd_box b, dpd_stats* out)
{
    if (!b || !out) return fail(DPD_EINVAL, "dpd_get_stats: null argument");
    dpd::DevStats s;
    HIPCHK(hipMemcpyAsync(&s, b->st, sizeof s, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    std::memset(out, 0, sizeof *out);
    for (int k = 0; k < 3; ++k) {
        out->momentum[k] = s.last[k];
        out->sum_momentum[k] = s.sum_momentum[k];
    }
    out->ke_half = s.last[3];
    out->ke_centred = s.last[4];
    out->kT_centred = s.last_kT_centred;
    out->virial = s.last_virial;
    out->pressure = s.last_pressure;
    out->sum_kT_centred = s.sum_kT_centred;
    out->sum_pressure = s.sum_pressure;
    out->nsamples = s.nsamples;
    out->step = s.step;
    out->nonfinite = s.nonfinite;
    out->escaped = s.escaped;
    if (s.nonfinite) return fail(DPD_ENONFINITE, "dpd_get_stats: non-finite value seen");
    return DPD_OK;
}

int dpd_get_profile(dpd_box b, double* sum_v, double* count, int32_t nbins)
{
    if (!b || !sum_v || !count) return fail(DPD_EINVAL, "dpd_get_profile: null argument");
    if (!b->have_params || nbins != b->params.profile_bins || nbins <= 0)
        return fail(DPD_EINVAL, "dpd_get_profile: nbins must equal params.profile_bins (> 0)");
    static thread_local long long buf[2 * dpd::kProfileMaxBins];
    HIPCHK(hipMemcpyAsync(buf, b->profile, (size_t)nbins * 2 * sizeof(long long), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int k = 0; k < nbins; ++k) {
        sum_v[k] = (double)buf[2 * k] / dpd::kProfScale;
        count[k] = (double)buf[2 * k + 1];
    }
    return DPD_OK;
}

int dpd_reset_accumulators(dpd_box b)
{
    if (!b) return fail(DPD_EINVAL, "dpd_reset_accumulators: null box");
    char* base = (char*)b->st;
    const size_t off = offsetof(dpd::DevStats, sum_kT_centred);
    const size_t len = offsetof(dpd::DevStats, nsamples) + sizeof(unsigned long long) - off;
    HIPCHK(hipMemsetAsync(base + off, 0, len, b->stream));
    HIPCHK(hipMemsetAsync(b->profile, 0, (size_t)dpd::kProfileMaxBins * 2 * sizeof(long long), b->stream));
    return DPD_OK;
}

int dpd_destroy(dpd_box b)
{
    if (!b) return DPD_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    if (e != hipSuccess) return fail(DPD_EDEVICE, "dpd_destroy: %s", hipGetErrorString(e));
    return DPD_OK;
}

int dpd_philox(const uint32_t* ctr4, const uint32_t* key2, int64_t n, uint32_t* out4, int where, void* hip_stream)
{
    if (where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_philox: device pointers only");
    if (n < 0 || (n > 0 && (!ctr4 || !key2 || !out4))) return fail(DPD_EINVAL, "dpd_philox: bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(dpd::launch_philox(ctr4, key2, n, out4, s));
    HIPCHK(hipStreamSynchronize(s));
    return DPD_OK;
}

int dpd_box_muller(const uint32_t* w0, const uint32_t* w1, int64_t n, float* xi, int where, void* hip_stream)
{
    if (where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_box_muller: device pointers only");
    if (n < 0 || (n > 0 && (!w0 || !w1 || !xi))) return fail(DPD_EINVAL, "dpd_box_muller: bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(dpd::launch_box_muller(w0, w1, n, xi, s));
    HIPCHK(hipStreamSynchronize(s));
    return DPD_OK;
}

}  // extern "C"
