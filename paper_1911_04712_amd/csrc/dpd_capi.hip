// dpd_capi.hip -- host runtime behind include/dpd.h: box state, workspace
// layout, validation, the step pipeline and its HIP-graph capture, batches
// of boxes and the tile autotuner.
//
// Every step kernel reads a per-box descriptor (BoxDesc) from device memory
// and maps its workgroups to boxes through prefix tables (LaunchPlan), so a
// box alone is a batch of one and runs the very same kernels, with the same
// per-box work partition, as inside a batch.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <array>
#include <mutex>
#include <string>
#include <vector>

#include "dpd.h"
#include "dpd_internal.hpp"
#include "dpd_runtime.hpp"

static_assert(DPD_FLAG_VIRIAL == dpd::kFlagVirial, "flag mismatch");
static_assert(DPD_FLAG_REFERENCE_FORCE == dpd::kFlagReference, "flag mismatch");

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
    // 3 n < 2^31: the n x 3 row arrays are indexed with 32-bit offsets
    return g->n >= 0 && g->n <= ((int64_t(1) << 31) - 1) / 3 && nc < (int64_t(1) << 31) - 1;
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

constexpr int kGraphMax = 64;           // steps per captured graph of a single box (longer runs replay it)
constexpr int kBatchGraphMax = 1024;    // a batch run of up to this many steps is one graph launch
constexpr int kBatchGraphMin = 64;      // shorter batch runs are launched directly (no capture)
constexpr size_t kLdsLimit = 160 * 1024 - 1280;  // LDS per CU less the kernels' static LDS

// Tile shapes the autotuners try (cells per edge).
constexpr int kTuneCand[][3] = {{4, 4, 4}, {8, 4, 4}, {8, 4, 2}, {6, 3, 3}, {4, 4, 2}, {4, 2, 2}, {2, 2, 4},
                                {4, 2, 4}, {2, 4, 4}, {3, 3, 3}, {6, 4, 4}, {2, 2, 2}, {8, 2, 2}, {6, 6, 4},
                                {8, 8, 4}, {3, 3, 2}, {8, 3, 3}, {6, 4, 2}, {6, 2, 2}, {6, 6, 3}, {6, 6, 6},
                                {8, 6, 4}, {12, 4, 4}, {12, 6, 4}, {8, 8, 2}, {6, 6, 2}, {12, 3, 3}};

}  // namespace

namespace dpd {

int set_error(int code, const char* msg)
{
    std::snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

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
    L.cellof = take(nn * sizeof(int));
    L.out = take(nn * 3 * sizeof(float));
    L.count = take((size_t)nc * sizeof(int));
    L.cell_start = take((size_t)(nc + 1) * sizeof(int));
    L.bsum = take((size_t)((nc + kSubChunk - 1) / kSubChunk) * sizeof(int));
    // one partial per integrate block, or per force tile when the kick-drift
    // is fused into the force kernel (a tile holds at least one cell)
    L.partials = take((size_t)std::max<int64_t>(kIntegrateMaxBlocks, nc) * kPartials * sizeof(double));
    L.profile = take((size_t)kProfileMaxBins * 2 * sizeof(long long));
    L.stats = take(sizeof(DevStats));
    L.flags = take(4 * sizeof(int));
    L.desc = take(sizeof(BoxDesc));
    L.pre = take((size_t)kNumWork * 2 * sizeof(int));
    L.total = off;
    return L;
}

}  // namespace dpd

namespace {

// Captured multi-step graphs of one launch group, kept by run length (a few
// lengths, least recently used first out).  Each graph holds its steps and
// the final fold of the reductions, so a run is complete when it returns.
struct GraphCache {
    static constexpr int kSlots = 4;
    struct Slot {
        int64_t steps = 0;
        hipGraphExec_t exec = nullptr;
        uint64_t used = 0;
    } slot[kSlots];
    hipStream_t cap = nullptr;
    uint64_t tick = 0;

    void clear()
    {
        for (Slot& s : slot) {
            if (s.exec) (void)hipGraphExecDestroy(s.exec);
            s = Slot{};
        }
    }
    void release()
    {
        clear();
        if (cap) (void)hipStreamDestroy(cap);
        cap = nullptr;
    }
    Slot* find(int64_t steps)
    {
        for (Slot& s : slot)
            if (s.exec && s.steps == steps) return &s;
        return nullptr;
    }
    Slot* victim()
    {
        Slot* v = &slot[0];
        for (Slot& s : slot) {
            if (!s.exec) return &s;
            if (s.used < v->used) v = &s;
        }
        return v;
    }
};

}  // namespace

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

    dpd::BoxDesc hd{};          // host copy of the device descriptor
    dpd::BoxDesc* d_desc = nullptr;
    int* d_pre = nullptr;
    dpd::LaunchPlan lp{};
    int* flags = nullptr;
    float* out = nullptr;

    dpd_params params{};
    bool have_params = false;
    uint64_t seed = 0;
    bool have_seed = false;
    bool have_state = false;
    bool keys_valid = false;   // keyslot/count describe pos_a
    bool binned = false;       // pos_b/vel_b/cell_start describe the current state
    bool have_force = false;   // force/pos_b hold the last step's forces

    int tile_req[3] = {0, 0, 0};
    int threads_req = 0;       // workgroup size of the tile kernel (0: kForceBlock)

    // species: ntypes = 0 uses params.a / params.gamma for every pair
    int ntypes = 0;
    double a_tab[dpd::kMaxTypes * dpd::kMaxTypes] = {};
    double g_tab[dpd::kMaxTypes * dpd::kMaxTypes] = {};
    double rc_tab[dpd::kMaxTypes * dpd::kMaxTypes] = {};
    int max_type = 0;          // largest species assigned since the state was loaded
    int n_frozen = 0;          // frozen wall particles of the current state
    double rho_occ = 0.0;      // particles per occupied cell of the loaded state (0: use n / nc)

    // captured multi-step graphs (dropped when the launch shape changes)
    GraphCache graphs;
    bool graph_dirty = true;
};

struct dpd_batch_s {
    std::vector<dpd_box_s*> boxes;
    int capacity = 0;          // most boxes the device tables hold
    hipStream_t stream = nullptr;
    dpd::BoxDesc* d_desc = nullptr;
    int* d_pre = nullptr;
    std::vector<int> pre;      // host copy [kNumWork][nbox + 1]
    dpd::LaunchPlan lp{};
    GraphCache graphs;
    bool graph_dirty = true;
    hipEvent_t done = nullptr;     // the last run's end (boxes on other streams wait for it)
    hipEvent_t pending = nullptr;  // work queued on a box's own stream (the run waits for it)
    // pinned staging of the tables, two buffers used in turn: the copy from
    // one may still be queued behind a running step while the other is filled
    char* stage[2] = {nullptr, nullptr};
    size_t stage_bytes[2] = {0, 0};
    hipEvent_t stage_done[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_next = 0;
};

namespace {

dpd::ForceConst force_const(const dpd_box_s* b)
{
    dpd::ForceConst fc{};
    const dpd_params& p = b->params;
    auto sig_rdt = [&](double g) { return (float)(std::sqrt(2.0 * g * p.kT) / std::sqrt(p.dt)); };
    fc.pc.k0 = (uint32_t)b->seed;
    fc.pc.k1 = (uint32_t)(b->seed >> 32);
    // ntypes > 1 switches the kernels to the pair table: several species, or
    // one species with a cutoff of its own below the cell edge
    fc.ntypes = (b->ntypes == 1 && b->rc_tab[0] != 1.0) ? 2 : b->ntypes;
    if (b->ntypes >= 1) {
        constexpr int M = dpd::kMaxTypes;
        for (int u = 0; u < b->ntypes; ++u)
            for (int v = 0; v < b->ntypes; ++v) {
                const double a = b->a_tab[u * M + v], g = b->g_tab[u * M + v], rc = b->rc_tab[u * M + v];
                fc.tab[u * M + v] = make_float4((float)a, (float)g, sig_rdt(g), (float)(1.0 / rc));
            }
        fc.pc.a = fc.tab[0].x;         // one species: the table's only entry, on the plain path
        fc.pc.gamma = fc.tab[0].y;
        fc.pc.sig_rdt = fc.tab[0].z;
    } else {
        fc.pc.a = (float)p.a;
        fc.pc.gamma = (float)p.gamma;
        fc.pc.sig_rdt = sig_rdt(p.gamma);
    }
    if (b->ntypes <= 1) {              // every entry is the one species (a batch may run this box on
        const float4 e0 = b->ntypes == 1 ? fc.tab[0] : make_float4(fc.pc.a, fc.pc.gamma, fc.pc.sig_rdt, 1.0f);
        for (auto& e : fc.tab) e = e0; // the table path, whatever its particles' .w hold)
    }
    fc.pc.kgen = (p.kexp != 0.0 && p.kexp != 1.0) ? 1 : 0;
    fc.pc.kexp = fc.pc.kgen ? (float)p.kexp : 1.0f;
    for (int k = 0; k < 3; ++k) {
        fc.L[k] = b->L[k];
        fc.cells[k] = b->cells[k];
    }
    fc.body_f = (float)p.body_f;
    fc.flow_axis = p.flow_axis;
    fc.grad_axis = p.grad_axis;
    fc.half_grad = 0.5f * b->L[p.grad_axis];
    fc.body_uniform = (p.flags & DPD_FLAG_BODY_UNIFORM) ? 1 : 0;
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
    const int nfree = b->n - b->n_frozen;
    sc.inv_dof = nfree >= 2 ? 1.0 / (3.0 * (double)(nfree - 1)) : 0.0;
    sc.wall_kind = p.wall_kind;
    sc.wall_h = (float)p.wall_h;
    for (int k = 0; k < 3; ++k) sc.centre[k] = 0.5f * b->L[k];
    sc.wall_r_in = (float)p.wall_r_in;
    const double om[2] = {p.omega_in, p.omega_out};
    for (int c = 0; c < 2; ++c) {
        sc.omega[c] = (float)om[c];
        sc.rot[c][0] = (float)std::cos(om[c] * p.dt);
        sc.rot[c][1] = (float)std::sin(om[c] * p.dt);
    }
    const double vol = (double)b->cells[0] * b->cells[1] * b->cells[2];
    sc.inv_vol = 1.0 / vol;
    sc.rho = (double)b->n / vol;
    return sc;
}

// Default cell tile and workgroup size of the LDS force kernel, from
// sweeps on MI355X.  A box large enough to give at least kBigTiles tiles of
// the large shape takes it: 6x6x4 cells with 1024 threads at densities up
// to 4.5 (the 48^3 box at rho = 3 steps in 82.6 us, against 93 us with 4x4x4
// and 512), 8x4x4 with 1024 above (the 192x96x96 box at rho = 8: 4.99 ms
// against 5.67 ms with 4x4x4).  Smaller boxes keep more, smaller tiles for
// parallelism: 4x4x4 (dilute) or 4x2x2 (dense) with 512 threads.  Where a
// shape's LDS does not fit a CU (denser fluids) the next one of the list that
// does.
struct Shape {
    int t[3];
    int threads;
};
constexpr int kBigTiles = 512;
constexpr Shape kDiluteShapes[] = {{{6, 6, 4}, 1024}, {{4, 4, 4}, 512}, {{4, 2, 2}, 512}, {{2, 2, 2}, 256}};
constexpr Shape kDenseShapes[] = {{{8, 4, 4}, 1024}, {{4, 2, 2}, 512}, {{3, 2, 2}, 512}, {{2, 2, 2}, 256}};
static_assert(sizeof kDiluteShapes == sizeof kDenseShapes, "both lists have four shapes");

dpd::TileConst tile_for(const dpd_box_s* b, const int* req, int threads = 0)
{
    if (threads <= 0) threads = b->threads_req;     // 0: the default of the shape
    // the tile capacities follow the density of the occupied cells: a box
    // with walls leaves the cells beyond the frozen layers empty
    // (unless that would not fit a CU's LDS, as for a clump of particles:
    // overfull tiles then take the gather path)
    const double rho_mean = b->nc > 0 ? (double)b->n / (double)b->nc : 0.0;
    dpd::TileConst tc{};
    for (const double rho : {b->rho_occ > 1.1 * rho_mean ? b->rho_occ : rho_mean, rho_mean}) {
        if (req[0] > 0) {
            tc = dpd::make_tile_const(b->cells, rho, req, threads > 0 ? threads : dpd::kForceBlock, 0, 0);
            if ((size_t)tc.lds_bytes <= kLdsLimit) return tc;
            continue;
        }
        const Shape* shapes = rho <= 4.5 ? kDiluteShapes : kDenseShapes;
        for (int k = 0; k < 4; ++k) {
            tc = dpd::make_tile_const(b->cells, rho, shapes[k].t, threads > 0 ? threads : shapes[k].threads, 0, 0);
            if (k == 0 && tc.ntiles < kBigTiles) continue;     // a small box: more, smaller tiles
            if ((size_t)tc.lds_bytes <= kLdsLimit) return tc;
        }
    }
    return tc;   // nothing fits at any capacity: the callers report it
}

// Rebuild the host descriptor and single-box plan from the box's current
// settings and copy both to the device (stream-ordered, then synchronised so
// the host buffers can change again).
int push_desc(dpd_box_s* b)
{
    dpd::BoxDesc& d = b->hd;
    char* w = b->ws;
    const dpd::Layout& L = b->lay;
    d.pos_a = (float4*)(w + L.pos_a);
    d.vel_a = (float4*)(w + L.vel_a);
    d.pos_b = (float4*)(w + L.pos_b);
    d.vel_b = (float4*)(w + L.vel_b);
    d.force = (float4*)(w + L.force);
    d.keyslot = (int2*)(w + L.keyslot);
    d.perm = (int*)(w + L.perm);
    d.cellof = (int*)(w + L.cellof);
    d.count = (int*)(w + L.count);
    d.cell_start = (int*)(w + L.cell_start);
    d.bsum = (int*)(w + L.bsum);
    d.partials = (double*)(w + L.partials);
    d.profile = (long long*)(w + L.profile);
    d.st = (dpd::DevStats*)(w + L.stats);
    d.n = b->n;
    d.nc = b->nc;
    d.nchunks = (b->nc + dpd::kScanChunk - 1) / dpd::kScanChunk;
    d.nsub = (b->nc + dpd::kSubChunk - 1) / dpd::kSubChunk;
    d.nblk_int = dpd::integrate_blocks(b->n);
    d.flags = b->have_params ? b->params.flags : 0;
    if (b->have_params) {
        d.fc = force_const(b);
        d.sc = step_const(b);
    }
    d.tc = tile_for(b, b->tile_req);
    int pre[dpd::kNumWork * 2];
    const dpd::LaunchPlan old = b->lp;
    for (int k = 0; k < dpd::kNumWork; ++k) {
        pre[2 * k] = 0;
        pre[2 * k + 1] = dpd::box_work(d, k);
        b->lp.total[k] = pre[2 * k + 1];
    }
    b->lp.desc = b->d_desc;
    b->lp.pre = b->d_pre;
    b->lp.nbox = 1;
    b->lp.lds_force = d.tc.lds_bytes;
    b->lp.force_threads = d.tc.threads;
    b->lp.any_virial = (d.flags & DPD_FLAG_VIRIAL) != 0;
    b->lp.reference_force = (d.flags & DPD_FLAG_REFERENCE_FORCE) != 0;
    // the species instantiation also carries the species of particles that
    // have one while the box is back to one species from the params (same
    // forces: every table entry is then that one pair)
    b->lp.species = d.fc.ntypes > 1 || b->max_type > 0;
    b->lp.walls = d.sc.wall_kind != 0 || b->n_frozen > 0;
    b->lp.fuse = !b->lp.reference_force;      // the reference force path has no tile kernel to fuse into
    // a captured graph holds the kernel choice and the launch shapes
    if (old.lds_force != b->lp.lds_force || old.any_virial != b->lp.any_virial ||
        old.reference_force != b->lp.reference_force || old.species != b->lp.species || old.walls != b->lp.walls ||
        old.fuse != b->lp.fuse ||
        old.force_threads != b->lp.force_threads)
        b->graph_dirty = true;
    for (int k = 0; k < dpd::kNumWork; ++k) b->graph_dirty |= old.total[k] != b->lp.total[k];
    HIPCHK(dpd::force_tiled_prepare(d.tc.lds_bytes));
    HIPCHK(hipMemcpyAsync(b->d_desc, &d, sizeof d, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_pre, pre, sizeof pre, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DPD_OK;
}

hipError_t enqueue_step_tail(const dpd::LaunchPlan& lp, hipStream_t s)
{
    hipError_t e = dpd::launch_force(lp, s, true);
    if (e == hipSuccess) e = dpd::launch_virial(lp, s);
    if (e == hipSuccess && !lp.fuse) e = dpd::launch_integrate(lp, s);
    return e;
}

hipError_t enqueue_steps(const dpd::LaunchPlan& lp, int64_t nsteps, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        e = dpd::launch_bin(lp, s);
        if (e == hipSuccess) e = enqueue_step_tail(lp, s);
    }
    return e;
}

// Capture nsteps steps and the final fold of the reductions as one graph.
int capture(const dpd::LaunchPlan& lp, int64_t nsteps, hipStream_t* cap, hipGraphExec_t* exec)
{
    *exec = nullptr;
    if (!*cap) HIPCHK(hipStreamCreateWithFlags(cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(*cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_steps(lp, nsteps, *cap);
    if (e == hipSuccess) e = dpd::launch_fold(lp, *cap);
    hipError_t e2 = hipStreamEndCapture(*cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(DPD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *exec = nullptr;
        return fail(DPD_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return DPD_OK;
}

// The graph of a run of `steps` steps: from the cache, else captured (the
// least recently used length makes room).  `dirty` drops every cached graph
// first (the launch shape changed).
int graph_for(GraphCache& gc, bool& dirty, const dpd::LaunchPlan& lp, int64_t steps, hipGraphExec_t* out)
{
    if (dirty) {
        gc.clear();
        dirty = false;
    }
    GraphCache::Slot* s = gc.find(steps);
    if (!s) {
        s = gc.victim();
        if (s->exec) (void)hipGraphExecDestroy(s->exec);
        *s = GraphCache::Slot{};
        hipGraphExec_t ex = nullptr;
        const int rc = capture(lp, steps, &gc.cap, &ex);
        if (rc) return rc;
        s->steps = steps;
        s->exec = ex;
    }
    s->used = ++gc.tick;
    *out = s->exec;
    return DPD_OK;
}

// How dpd_step runs n steps after its optional first step: `full` graphs of
// `g` steps, then one graph of `tail` steps.
struct RunPlan {
    int64_t g = 0, full = 0, tail = 0;
};

RunPlan plan_run(int64_t n, int64_t gmax)
{
    RunPlan p;
    if (n <= 0) return p;
    p.g = n < gmax ? n : gmax;
    p.full = n / p.g;
    p.tail = n - p.full * p.g;
    return p;
}

int sync_box(dpd_box_s* b)
{
    HIPCHK(hipStreamSynchronize(b->stream));
    return DPD_OK;
}

hipMemcpyKind kind_to(int where) { return where == DPD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

bool ready(const dpd_box_s* b) { return b->have_params && b->have_seed && b->have_state; }

// ---- autotuner cache ----------------------------------------------------------
// A JSON file of tuned (tile, workgroup size) per key: the GPU architecture,
// the revision of the force kernel's sources (fixed at build time), and the
// box geometry, density and kernel variant, or a batch's list of those.
// One entry per line, written and read by the two functions below.
#ifndef DPD_KERNEL_REV
#define DPD_KERNEL_REV "dev"
#endif

struct TuneEntry {
    std::string key;
    int tile[3] = {0, 0, 0};
    int threads = 0;
    double ms = 0.0;
};

struct TuneCacheFile {
    std::mutex mu;
    std::string path;                 // empty: no cache
    std::vector<TuneEntry> entries;
};

TuneCacheFile& tune_file()
{
    static TuneCacheFile f;
    return f;
}

void tune_read(TuneCacheFile& f)
{
    f.entries.clear();
    FILE* fp = std::fopen(f.path.c_str(), "r");
    if (!fp) return;
    char line[8192];
    while (std::fgets(line, sizeof line, fp)) {
        const char* k = std::strstr(line, "\"key\": \"");
        const char* t = std::strstr(line, "\"tile\": [");
        const char* h = std::strstr(line, "\"threads\": ");
        const char* m = std::strstr(line, "\"ms\": ");
        if (!k || !t || !h || !m) continue;
        k += 8;
        const char* ke = std::strchr(k, '"');
        if (!ke) continue;
        TuneEntry e;
        e.key.assign(k, ke);
        if (std::sscanf(t + 9, "%d, %d, %d", &e.tile[0], &e.tile[1], &e.tile[2]) != 3) continue;
        if (std::sscanf(h + 11, "%d", &e.threads) != 1 || std::sscanf(m + 6, "%lf", &e.ms) != 1) continue;
        f.entries.push_back(e);
    }
    std::fclose(fp);
}

void tune_write(const TuneCacheFile& f)
{
    const std::string tmp = f.path + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;                  // a read-only place: the cache stays in memory
    std::fprintf(fp, "{\"dpd_tune_cache\": 1, \"entries\": [\n");
    for (size_t i = 0; i < f.entries.size(); ++i) {
        const TuneEntry& e = f.entries[i];
        std::fprintf(fp, "  {\"key\": \"%s\", \"tile\": [%d, %d, %d], \"threads\": %d, \"ms\": %.6g}%s\n",
                     e.key.c_str(), e.tile[0], e.tile[1], e.tile[2], e.threads, e.ms,
                     i + 1 < f.entries.size() ? "," : "");
    }
    std::fprintf(fp, "]}\n");
    const bool ok = std::fclose(fp) == 0;
    if (ok) (void)std::rename(tmp.c_str(), f.path.c_str());
}

bool tune_lookup(const std::string& key, TuneEntry* out)
{
    TuneCacheFile& f = tune_file();
    std::lock_guard<std::mutex> lk(f.mu);
    if (f.path.empty()) return false;
    for (const TuneEntry& e : f.entries)
        if (e.key == key) {
            *out = e;
            return true;
        }
    return false;
}

void tune_store(const std::string& key, const int tile[3], int threads, double ms)
{
    TuneCacheFile& f = tune_file();
    std::lock_guard<std::mutex> lk(f.mu);
    if (f.path.empty()) return;
    tune_read(f);                     // another process may have added entries
    TuneEntry e;
    e.key = key;
    for (int k = 0; k < 3; ++k) e.tile[k] = tile[k];
    e.threads = threads;
    e.ms = ms;
    bool found = false;
    for (TuneEntry& x : f.entries)
        if (x.key == key) {
            x = e;
            found = true;
        }
    if (!found) f.entries.push_back(e);
    tune_write(f);
}

bool tune_cache_on()
{
    TuneCacheFile& f = tune_file();
    std::lock_guard<std::mutex> lk(f.mu);
    return !f.path.empty();
}

std::string arch_name(hipStream_t)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// The part of a key that describes one box: what the kernel's speed depends on.
std::string box_tune_part(const dpd_box_s* b)
{
    char buf[160];
    const double rho = b->nc > 0 ? (double)b->n / (double)b->nc : 0.0;
    const double rho_t = b->rho_occ > 1.1 * rho ? b->rho_occ : rho;
    std::snprintf(buf, sizeof buf, "%dx%dx%d/rho%.2f/sp%d/kg%d", b->cells[0], b->cells[1], b->cells[2], rho_t,
                  b->hd.fc.ntypes > 1 ? 1 : 0, b->hd.fc.pc.kgen);
    return buf;
}

std::string tune_key_prefix(hipStream_t s) { return arch_name(s) + "|" DPD_KERNEL_REV "|"; }

// Lay a validated geometry out in `dev_ws` (large enough, 256-byte aligned)
// and clear the counters, accumulators and flags that the step kernels
// expect at zero.  The body of dpd_create, shared with dpd_run_static.
int box_init(dpd_box_s* b, const dpd_geom* geom, void* dev_ws, void* hip_stream)
{
    const int64_t nc = (int64_t)geom->cells[0] * geom->cells[1] * geom->cells[2];
    const dpd::Layout lay = dpd::make_layout(geom->n, nc);
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
    b->d_desc = (dpd::BoxDesc*)(b->ws + lay.desc);
    b->d_pre = (int*)(b->ws + lay.pre);
    b->flags = (int*)(b->ws + lay.flags);
    b->out = (float*)(b->ws + lay.out);
    const int rc = push_desc(b);
    if (rc != DPD_OK) return rc;
    hipError_t e = dpd::launch_fill_i32(b->hd.count, 0, nc, b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32(b->hd.bsum, 0, b->hd.nsub, b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32((int*)b->hd.st, 0, (int64_t)(sizeof(dpd::DevStats) / 4), b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32((int*)b->hd.profile, 0, (int64_t)dpd::kProfileMaxBins * 4, b->stream);
    if (e == hipSuccess) e = dpd::launch_fill_i32(b->flags, 0, 4, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(DPD_EDEVICE, "dpd_create: %s", hipGetErrorString(e));
    return DPD_OK;
}


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
    if (!geom_ok(geom)) return fail(DPD_EINVAL, "dpd_create: invalid geometry (cells in 3..4096, 0 <= n <= (2^31 - 1) / 3)");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(DPD_EINVAL, "dpd_create: workspace null or not 256-byte aligned");
    const int64_t nc = (int64_t)geom->cells[0] * geom->cells[1] * geom->cells[2];
    const dpd::Layout lay = dpd::make_layout(geom->n, nc);
    if (ws_bytes < lay.total)
        return fail(DPD_ENOMEM, "dpd_create: workspace of %zu bytes, %zu needed", ws_bytes, lay.total);
    dpd_box_s* b = new (std::nothrow) dpd_box_s();
    if (!b) return fail(DPD_ENOMEM, "dpd_create: host allocation failed");
    const int rc = box_init(b, geom, dev_ws, hip_stream);
    if (rc != DPD_OK) {
        delete b;
        return rc;
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
    if (p->flags & ~(DPD_FLAG_VIRIAL | DPD_FLAG_REFERENCE_FORCE | DPD_FLAG_BODY_UNIFORM))
        return fail(DPD_EINVAL, "dpd_set_params: unknown flags");
    if (p->wall_kind < DPD_WALL_NONE || p->wall_kind > DPD_WALL_CYLINDERS || p->reserved2 != 0)
        return fail(DPD_EINVAL, "dpd_set_params: wall_kind must be a DPD_WALL_* value and reserved2 0");
    if (!std::isfinite(p->wall_r_in) || !std::isfinite(p->omega_in) || !std::isfinite(p->omega_out))
        return fail(DPD_EINVAL, "dpd_set_params: non-finite cylinder parameter");
    if (p->wall_kind == DPD_WALL_CYLINDERS && !(p->wall_r_in > 0.0 && p->wall_r_in < p->wall_h))
        return fail(DPD_EINVAL, "dpd_set_params: cylinders need 0 < wall_r_in < wall_h");
    if (p->wall_kind != DPD_WALL_NONE) {
        if (!std::isfinite(p->wall_h) || !(p->wall_h > 0.0))
            return fail(DPD_EINVAL, "dpd_set_params: wall_h must be finite and > 0");
        for (int k = 0; k < 3; ++k) {
            const bool used = p->wall_kind == DPD_WALL_PLATES ? k == p->grad_axis : k != p->flow_axis;
            if (used && !(p->wall_h + 1.0 < 0.5 * b->cells[k]))
                return fail(DPD_EINVAL, "dpd_set_params: the wall and its frozen layer must fit: wall_h + 1 < L/2 "
                            "on axis %d", k);
        }
    }
    if (!(p->kexp >= 0.0 && p->kexp <= 1.0)) return fail(DPD_EINVAL, "dpd_set_params: kexp must be in [0, 1]");
    const double sig = std::sqrt(2.0 * p->gamma * p->kT) / std::sqrt(p->dt);
    if (!std::isfinite(sig) || sig > 1e8 || std::fabs(p->a) > 1e8 || p->gamma > 1e8)
        return fail(DPD_EINVAL, "dpd_set_params: parameters out of the FP32 force range");
    const int old_flags = b->have_params ? b->params.flags : -1;
    b->params = *p;
    b->have_params = true;
    if (old_flags != p->flags) b->graph_dirty = true;   // the launch sequence depends on the flags only
    return push_desc(b);
}

int dpd_set_species(dpd_box b, int32_t ntypes, const double* a_tab, const double* gamma_tab, const double* rc_tab)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_species: null box");
    if (ntypes < 0 || ntypes > dpd::kMaxTypes) return fail(DPD_EINVAL, "dpd_set_species: ntypes must be in 0..%d", dpd::kMaxTypes);
    if (ntypes > 0 && (!a_tab || !gamma_tab)) return fail(DPD_EINVAL, "dpd_set_species: null table");
    if (ntypes > 0 && b->max_type >= ntypes)
        return fail(DPD_EINVAL, "dpd_set_species: particles of species %d exist; need ntypes > %d", b->max_type, b->max_type);
    for (int u = 0; u < ntypes; ++u)
        for (int v = 0; v < ntypes; ++v) {
            const double a = a_tab[u * ntypes + v], g = gamma_tab[u * ntypes + v];
            if (!std::isfinite(a) || !std::isfinite(g) || g < 0.0 || std::fabs(a) > 1e8 || g > 1e8)
                return fail(DPD_EINVAL, "dpd_set_species: entry (%d, %d) not finite, gamma < 0 or out of range", u, v);
            if (a != a_tab[v * ntypes + u] || g != gamma_tab[v * ntypes + u])
                return fail(DPD_EINVAL, "dpd_set_species: tables must be symmetric (entry (%d, %d))", u, v);
            if (rc_tab) {
                const double c = rc_tab[u * ntypes + v];
                if (!(c >= 1.0 / 16.0 && c <= 1.0) || c != rc_tab[v * ntypes + u])
                    return fail(DPD_EINVAL, "dpd_set_species: cutoff (%d, %d) must be symmetric and in [1/16, 1]", u, v);
            }
        }
    constexpr int M = dpd::kMaxTypes;
    for (int k = 0; k < M * M; ++k) {
        b->a_tab[k] = b->g_tab[k] = 0.0;
        b->rc_tab[k] = 1.0;
    }
    for (int u = 0; u < ntypes; ++u)
        for (int v = 0; v < ntypes; ++v) {
            b->a_tab[u * M + v] = a_tab[u * ntypes + v];
            b->g_tab[u * M + v] = gamma_tab[u * ntypes + v];
            if (rc_tab) b->rc_tab[u * M + v] = rc_tab[u * ntypes + v];
        }
    b->ntypes = ntypes;
    return push_desc(b);
}

int dpd_get_species(dpd_box b, int32_t* ntypes)
{
    if (!b || !ntypes) return fail(DPD_EINVAL, "dpd_get_species: null argument");
    *ntypes = b->ntypes;
    return DPD_OK;
}

int dpd_set_types(dpd_box b, const int32_t* type_host)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_types: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_set_types: no state loaded");
    if (b->ntypes < 1) return fail(DPD_ESTATE, "dpd_set_types: set the species tables first");
    if (b->n > 0 && !type_host) return fail(DPD_EINVAL, "dpd_set_types: null array");
    int mx = 0;
    for (int i = 0; i < b->n; ++i) {
        if (type_host[i] < 0 || type_host[i] >= b->ntypes)
            return fail(DPD_EINVAL, "dpd_set_types: particle %d has species %d outside 0..%d", i, type_host[i], b->ntypes - 1);
        mx = std::max(mx, (int)type_host[i]);
    }
    if (b->n == 0) return DPD_OK;
    const dpd::BoxDesc& d = b->hd;
    int* staged = (int*)b->out;
    HIPCHK(hipMemcpyAsync(staged, type_host, (size_t)b->n * sizeof(int), hipMemcpyHostToDevice, b->stream));
    HIPCHK(dpd::launch_set_types(d.pos_a, d.vel_a, b->n, staged, b->stream));
    if (b->binned || b->have_force)     // pos_b / vel_b hold a copy of the state in cell order
        HIPCHK(dpd::launch_set_types(d.pos_b, d.vel_b, b->n, staged, b->stream));
    b->max_type = mx;
    HIPCHK(hipStreamSynchronize(b->stream));
    return push_desc(b);                // the kernel instantiation follows the species present
}

int dpd_get_types(dpd_box b, int32_t* type_host)
{
    if (!b) return fail(DPD_EINVAL, "dpd_get_types: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_get_types: no state loaded");
    if (b->n > 0 && !type_host) return fail(DPD_EINVAL, "dpd_get_types: null array");
    if (b->n == 0) return DPD_OK;
    const dpd::BoxDesc& d = b->hd;
    int* staged = (int*)b->out;
    HIPCHK(dpd::launch_get_types(d.pos_a, d.vel_a, b->n, staged, b->stream));
    HIPCHK(hipMemcpyAsync(type_host, staged, (size_t)b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    return sync_box(b);
}

int dpd_set_frozen(dpd_box b, const uint8_t* frozen_host)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_frozen: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_set_frozen: no state loaded");
    if (b->n > 0 && !frozen_host) return fail(DPD_EINVAL, "dpd_set_frozen: null array");
    int nf = 0;
    for (int i = 0; i < b->n; ++i) nf += frozen_host[i] ? 1 : 0;
    if (b->n - nf < 2) return fail(DPD_EINVAL, "dpd_set_frozen: at least 2 particles must stay free");
    const dpd::BoxDesc& d = b->hd;
    unsigned char* staged = (unsigned char*)b->out;
    HIPCHK(hipMemcpyAsync(staged, frozen_host, (size_t)b->n, hipMemcpyHostToDevice, b->stream));
    HIPCHK(dpd::launch_set_frozen(d.pos_a, d.vel_a, b->n, staged, d.sc, b->stream));
    if (b->binned || b->have_force)     // pos_b / vel_b hold a copy of the state in cell order
        HIPCHK(dpd::launch_set_frozen(d.pos_b, d.vel_b, b->n, staged, d.sc, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->n_frozen = nf;
    return push_desc(b);                // degrees of freedom of kT
}

int dpd_get_frozen(dpd_box b, uint8_t* frozen_host)
{
    if (!b) return fail(DPD_EINVAL, "dpd_get_frozen: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_get_frozen: no state loaded");
    if (b->n > 0 && !frozen_host) return fail(DPD_EINVAL, "dpd_get_frozen: null array");
    if (b->n == 0) return DPD_OK;
    const dpd::BoxDesc& d = b->hd;
    unsigned char* staged = (unsigned char*)b->out;
    HIPCHK(dpd::launch_get_frozen(d.pos_a, d.vel_a, b->n, staged, b->stream));
    HIPCHK(hipMemcpyAsync(frozen_host, staged, (size_t)b->n, hipMemcpyDeviceToHost, b->stream));
    return sync_box(b);
}

int dpd_wall_sdf(dpd_box b, float* sdf_host)
{
    if (!b) return fail(DPD_EINVAL, "dpd_wall_sdf: null box");
    if (!b->have_state || !b->have_params) return fail(DPD_ESTATE, "dpd_wall_sdf: needs params and a state");
    if (b->params.wall_kind == DPD_WALL_NONE) return fail(DPD_ESTATE, "dpd_wall_sdf: the params name no wall");
    if (b->n > 0 && !sdf_host) return fail(DPD_EINVAL, "dpd_wall_sdf: null array");
    if (b->n == 0) return DPD_OK;
    const dpd::BoxDesc& d = b->hd;
    HIPCHK(dpd::launch_wall_sdf(d.pos_a, b->n, d.sc, b->out, b->stream));
    HIPCHK(hipMemcpyAsync(sdf_host, b->out, (size_t)b->n * sizeof(float), hipMemcpyDeviceToHost, b->stream));
    return sync_box(b);
}

int dpd_set_tile(dpd_box b, const int32_t tile[3])
{
    if (!b || !tile) return fail(DPD_EINVAL, "dpd_set_tile: null argument");
    const bool dflt = tile[0] == 0 && tile[1] == 0 && tile[2] == 0;
    if (!dflt)
        for (int k = 0; k < 3; ++k)
            if (tile[k] < 1 || tile[k] > 16) return fail(DPD_EINVAL, "dpd_set_tile: edges must be in 1..16");
    if ((size_t)tile_for(b, tile).lds_bytes > kLdsLimit)
        return fail(DPD_EINVAL, "dpd_set_tile: tile needs more LDS than a CU has");
    for (int k = 0; k < 3; ++k) b->tile_req[k] = tile[k];
    b->graph_dirty = true;
    return push_desc(b);
}

int dpd_set_force_threads(dpd_box b, int32_t threads)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_force_threads: null box");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(DPD_EINVAL, "dpd_set_force_threads: threads must be 0, 256, 512 or 1024");
    const int saved = b->threads_req;
    b->threads_req = threads;
    if ((size_t)tile_for(b, b->tile_req).lds_bytes > kLdsLimit) {
        b->threads_req = saved;
        return fail(DPD_EINVAL, "dpd_set_force_threads: the tile would need more LDS than a CU has");
    }
    return push_desc(b);
}

int dpd_get_force_threads(dpd_box b, int32_t* threads)
{
    if (!b || !threads) return fail(DPD_EINVAL, "dpd_get_force_threads: null argument");
    *threads = b->hd.tc.threads;
    return DPD_OK;
}

int dpd_get_tile(dpd_box b, int32_t tile[3])
{
    if (!b || !tile) return fail(DPD_EINVAL, "dpd_get_tile: null argument");
    for (int k = 0; k < 3; ++k) tile[k] = b->hd.tc.T[k];
    return DPD_OK;
}

int dpd_set_seed(dpd_box b, uint64_t seed)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_seed: null box");
    b->seed = seed;
    b->have_seed = true;
    return push_desc(b);
}

int dpd_set_step(dpd_box b, uint64_t step)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_step: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_set_step: no state loaded");
    HIPCHK(hipStreamSynchronize(b->stream));           // no step may be in flight
    const unsigned long long s = step;
    HIPCHK(hipMemcpyAsync(&b->hd.st->step, &s, sizeof s, hipMemcpyHostToDevice, b->stream));
    return sync_box(b);
}

int dpd_set_state(dpd_box b, const float* pos_n3, const float* vel_n3, int where)
{
    if (!b) return fail(DPD_EINVAL, "dpd_set_state: null box");
    if (where != DPD_HOST && where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_set_state: bad `where`");
    if (b->n > 0 && (!pos_n3 || !vel_n3)) return fail(DPD_EINVAL, "dpd_set_state: null array");
    b->have_state = b->keys_valid = b->binned = b->have_force = false;
    b->max_type = 0;                                   // every particle starts as species 0, free
    b->n_frozen = 0;
    const dpd::BoxDesc& d = b->hd;
    const float *pp = pos_n3, *vp = vel_n3;
    const size_t bytes = (size_t)b->n * 3 * sizeof(float);
    if (where == DPD_HOST && b->n > 0) {
        HIPCHK(hipMemcpyAsync(d.pos_b, pos_n3, bytes, hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(d.vel_b, vel_n3, bytes, hipMemcpyHostToDevice, b->stream));
        pp = (const float*)d.pos_b;
        vp = (const float*)d.vel_b;
    }
    HIPCHK(dpd::launch_fill_i32(b->flags, 0, 4, b->stream));
    HIPCHK(dpd::launch_fill_i32(d.count, 0, b->nc, b->stream));
    HIPCHK(dpd::launch_fill_i32(d.bsum, 0, d.nsub, b->stream));
    HIPCHK(dpd::launch_fill_i32((int*)d.st, 0, (int64_t)(sizeof(dpd::DevStats) / 4), b->stream));
    HIPCHK(dpd::launch_fill_i32((int*)d.profile, 0, (int64_t)dpd::kProfileMaxBins * 4, b->stream));
    HIPCHK(dpd::launch_load_state(pp, vp, b->n, d.pos_a, d.vel_a, (float)b->q, (float)(1.0 / b->q), b->L, b->flags,
                                  b->stream));
    HIPCHK(dpd::launch_keys(d.pos_a, b->n, b->cells, d.count, d.bsum, d.keyslot, b->stream));
    HIPCHK(dpd::launch_count_nonempty(d.count, b->nc, b->flags + 1, b->stream));
    int bad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bad, b->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (bad[0]) return fail(DPD_EINVAL, "dpd_set_state: a position is outside [0, L) or a value is non-finite");
    b->rho_occ = bad[1] > 0 ? (double)b->n / (double)bad[1] : 0.0;
    const int rc = push_desc(b);        // capacities, no frozen particles
    if (rc) return rc;
    b->have_state = true;
    b->keys_valid = true;
    return DPD_OK;
}

int dpd_init_random(dpd_box b, double kT, uint64_t seed)
{
    if (!b) return fail(DPD_EINVAL, "dpd_init_random: null box");
    if (!b->have_params) return fail(DPD_ESTATE, "dpd_init_random: set params first (the mass scales velocities)");
    if (!std::isfinite(kT) || kT < 0.0) return fail(DPD_EINVAL, "dpd_init_random: kT must be finite and >= 0");
    b->have_state = b->keys_valid = b->binned = b->have_force = false;
    b->max_type = 0;                                   // every particle starts as species 0, free
    b->n_frozen = 0;
    const dpd::BoxDesc& d = b->hd;
    HIPCHK(dpd::launch_fill_i32(b->flags, 0, 4, b->stream));
    HIPCHK(dpd::launch_fill_i32(d.count, 0, b->nc, b->stream));
    HIPCHK(dpd::launch_fill_i32(d.bsum, 0, d.nsub, b->stream));
    HIPCHK(dpd::launch_fill_i32((int*)d.st, 0, (int64_t)(sizeof(dpd::DevStats) / 4), b->stream));
    HIPCHK(dpd::launch_fill_i32((int*)d.profile, 0, (int64_t)dpd::kProfileMaxBins * 4, b->stream));
    // the id-order staging buffer (12 B per particle) holds the per-block sums
    const int scratch = (int)std::min<int64_t>((int64_t)b->n * 3 / 2, (int64_t)1 << 30);
    HIPCHK(dpd::launch_init_random(b->n, b->L, (float)b->q, std::sqrt(kT / b->params.mass), seed, d.pos_a, d.vel_a,
                                   (double*)b->out, scratch, b->stream));
    HIPCHK(dpd::launch_keys(d.pos_a, b->n, b->cells, d.count, d.bsum, d.keyslot, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->rho_occ = 0.0;                   // uniform positions
    const int rc = push_desc(b);        // no frozen particles
    if (rc) return rc;
    b->have_state = true;
    b->keys_valid = true;
    return DPD_OK;
}

int dpd_build_cells(dpd_box b)
{
    if (!b) return fail(DPD_EINVAL, "dpd_build_cells: null box");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_build_cells: no state loaded");
    if (b->binned) return DPD_OK;
    HIPCHK(dpd::launch_bin(b->lp, b->stream));
    b->binned = true;
    b->keys_valid = false;
    b->have_force = false;
    return DPD_OK;
}

int dpd_step(dpd_box b, int64_t nsteps)
{
    if (!b) return fail(DPD_EINVAL, "dpd_step: null box");
    if (nsteps < 0) return fail(DPD_EINVAL, "dpd_step: nsteps < 0");
    if (!ready(b)) return fail(DPD_ESTATE, "dpd_step: set params, seed and state first");
    if (nsteps == 0) return DPD_OK;
    // the graphs first: a failed capture leaves the box as it was
    const int64_t left = nsteps - (b->binned ? 1 : 0);
    const RunPlan rp = plan_run(left, kGraphMax);
    hipGraphExec_t gfull = nullptr, gtail = nullptr;
    if (rp.full) {
        const int rc = graph_for(b->graphs, b->graph_dirty, b->lp, rp.g, &gfull);
        if (rc) return rc;
    }
    if (rp.tail) {
        const int rc = graph_for(b->graphs, b->graph_dirty, b->lp, rp.tail, &gtail);
        if (rc) return rc;
    }
    if (b->binned) {                      // first step reuses the existing cell list
        HIPCHK(enqueue_step_tail(b->lp, b->stream));
        b->binned = false;
        if (left == 0) HIPCHK(dpd::launch_fold(b->lp, b->stream));   // its reductions
    }
    for (int64_t k = 0; k < rp.full; ++k) HIPCHK(hipGraphLaunch(gfull, b->stream));
    if (rp.tail) HIPCHK(hipGraphLaunch(gtail, b->stream));
    b->keys_valid = true;
    b->have_force = true;
    return DPD_OK;
}

int dpd_prepare_steps(dpd_box b, int64_t nsteps)
{
    if (!b) return fail(DPD_EINVAL, "dpd_prepare_steps: null box");
    if (nsteps < 0) return fail(DPD_EINVAL, "dpd_prepare_steps: nsteps < 0");
    if (!ready(b)) return fail(DPD_ESTATE, "dpd_prepare_steps: set params, seed and state first");
    const int64_t left = nsteps - (b->binned && nsteps > 0 ? 1 : 0);
    const RunPlan rp = plan_run(left, kGraphMax);
    hipGraphExec_t g = nullptr;
    if (rp.full) {
        const int rc = graph_for(b->graphs, b->graph_dirty, b->lp, rp.g, &g);
        if (rc) return rc;
    }
    if (rp.tail) {
        const int rc = graph_for(b->graphs, b->graph_dirty, b->lp, rp.tail, &g);
        if (rc) return rc;
    }
    return DPD_OK;
}

int dpd_profile_steps(dpd_box b, int64_t nsteps, double* ms_out)
{
    if (!b || !ms_out) return fail(DPD_EINVAL, "dpd_profile_steps: null argument");
    if (nsteps < 1) return fail(DPD_EINVAL, "dpd_profile_steps: nsteps < 1");
    if (!ready(b)) return fail(DPD_ESTATE, "dpd_profile_steps: set params, seed and state first");
    // one event pair per stage, recorded by the stage's first kernel as it
    // starts and its last as it ends: the times are the kernels' own
    hipEvent_t ev[8] = {};
    int rc = DPD_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(DPD_EDEVICE, "dpd_profile_steps: hipEventCreate failed");
    double acc[4] = {0, 0, 0, 0};
    for (int64_t k = 0; k < nsteps && rc == DPD_OK; ++k) {
        const bool bin = !b->binned;
        hipError_t e = hipSuccess;
        if (bin) e = dpd::launch_bin(b->lp, b->stream, ev[0], ev[1]);
        b->binned = false;
        if (e == hipSuccess) e = dpd::launch_force(b->lp, b->stream, true, ev[2], ev[3]);
        const bool vir = b->lp.any_virial && b->lp.total[dpd::kWPart] > 0, integ = !b->lp.fuse;
        if (e == hipSuccess && vir) e = dpd::launch_virial(b->lp, b->stream, ev[4], ev[5]);
        if (e == hipSuccess && integ) e = dpd::launch_integrate(b->lp, b->stream, ev[6], ev[7]);
        // the reductions' fold normally rides in the next step's gather: here
        // it runs after the timed stages
        if (e == hipSuccess) e = dpd::launch_fold(b->lp, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        const bool timed[4] = {bin, true, vir, integ};
        for (int st = 0; st < 4 && e == hipSuccess; ++st) {
            if (!timed[st]) continue;
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, ev[2 * st], ev[2 * st + 1]);
            acc[st] += ms;
        }
        if (e != hipSuccess) rc = fail(DPD_EDEVICE, "dpd_profile_steps: %s", hipGetErrorString(e));
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    b->keys_valid = true;
    b->have_force = true;
    for (int st = 0; st < 4; ++st) ms_out[st] = acc[st] / (double)nsteps;
    return DPD_OK;
}

int dpd_time_force(dpd_box b, int32_t reps, double* ms_out)
{
    if (!b || !ms_out) return fail(DPD_EINVAL, "dpd_time_force: null argument");
    if (reps < 1 || reps > 10000) return fail(DPD_EINVAL, "dpd_time_force: reps must be in 1..10000");
    if (!ready(b)) return fail(DPD_ESTATE, "dpd_time_force: set params, seed and state first");
    // forces of the current positions; the state does not advance
    if (!b->binned) {
        HIPCHK(dpd::launch_bin(b->lp, b->stream));
        b->binned = true;
        b->keys_valid = false;
    }
    b->have_force = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = dpd::launch_force(b->lp, b->stream, false);          // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = dpd::launch_force(b->lp, b->stream, false);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(DPD_EDEVICE, "dpd_time_force: %s", hipGetErrorString(e));
    *ms_out = (double)ms / reps;
    return DPD_OK;
}

namespace {

// Timing the force kernel with the kick-drift fused (the kernel every box
// steps with, the reference force path aside) writes the next state and adds to the cell
// counters, the reductions and the flow profile.  The tuners keep the
// diagnostics and profile bins on the host before such launches and put
// everything back after them: the cell-ordered copy (pos_b, vel_b) becomes
// the state again (a reordering the stable binning undoes), and the counters
// start from zero as after a binning.
struct FusedKeep {
    dpd::DevStats st{};
    std::vector<long long> prof;
};

int fused_keep(const dpd_box_s* b, FusedKeep& k)
{
    const dpd::BoxDesc& d = b->hd;
    k.prof.assign((size_t)b->params.profile_bins * 2, 0);
    HIPCHK(hipMemcpyAsync(&k.st, d.st, sizeof k.st, hipMemcpyDeviceToHost, b->stream));
    if (!k.prof.empty())
        HIPCHK(hipMemcpyAsync(k.prof.data(), d.profile, k.prof.size() * sizeof(long long), hipMemcpyDeviceToHost,
                              b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DPD_OK;
}

int fused_restore(const dpd_box_s* b, const FusedKeep& k)
{
    const dpd::BoxDesc& d = b->hd;
    const size_t rows = (size_t)b->n * sizeof(float4);
    HIPCHK(hipMemcpyAsync(d.pos_a, d.pos_b, rows, hipMemcpyDeviceToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(d.vel_a, d.vel_b, rows, hipMemcpyDeviceToDevice, b->stream));
    HIPCHK(dpd::launch_fill_i32(d.count, 0, b->nc, b->stream));
    HIPCHK(dpd::launch_fill_i32(d.bsum, 0, d.nsub, b->stream));
    HIPCHK(hipMemcpyAsync(d.st, &k.st, sizeof k.st, hipMemcpyHostToDevice, b->stream));
    if (!k.prof.empty())
        HIPCHK(hipMemcpyAsync(d.profile, k.prof.data(), k.prof.size() * sizeof(long long), hipMemcpyHostToDevice,
                              b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DPD_OK;
}

}  // namespace

int dpd_tune_tile(dpd_box b, int32_t reps, int32_t tile_out[3], double* ms_out)
{
    if (!b || !tile_out) return fail(DPD_EINVAL, "dpd_tune_tile: null argument");
    if (reps < 1 || reps > 1000) return fail(DPD_EINVAL, "dpd_tune_tile: reps must be in 1..1000");
    if (!ready(b)) return fail(DPD_ESTATE, "dpd_tune_tile: set params, seed and state first");
    if (b->params.flags & DPD_FLAG_REFERENCE_FORCE)
        return fail(DPD_EINVAL, "dpd_tune_tile: the reference force path has no tiles");
    // The force kernel is timed on the current positions (binned once); the
    // state does not advance and the results do not depend on the tile.
    if (!b->binned) {
        HIPCHK(dpd::launch_bin(b->lp, b->stream));
        b->binned = true;
        b->keys_valid = false;
    }
    std::string key;
    if (tune_cache_on()) {
        key = tune_key_prefix(b->stream) + "box|" + box_tune_part(b);
        TuneEntry e;
        if (tune_lookup(key, &e) && (e.threads == 256 || e.threads == 512 || e.threads == 1024) &&
            e.tile[0] >= 1 && e.tile[1] >= 1 && e.tile[2] >= 1 && e.tile[0] <= 16 && e.tile[1] <= 16 &&
            e.tile[2] <= 16 && (size_t)tile_for(b, e.tile, e.threads).lds_bytes <= kLdsLimit) {
            for (int k = 0; k < 3; ++k) b->tile_req[k] = e.tile[k];
            b->threads_req = e.threads;
            b->have_force = false;
            b->graph_dirty = true;
            const int rc = push_desc(b);
            if (rc) return rc;
            for (int k = 0; k < 3; ++k) tile_out[k] = b->hd.tc.T[k];
            if (ms_out) *ms_out = e.ms;
            return DPD_OK;
        }
    }
    const auto& cand = kTuneCand;
    const int saved[3] = {b->tile_req[0], b->tile_req[1], b->tile_req[2]};
    const int saved_threads = b->threads_req;
    // A box whose steps fuse the kick-drift into the force kernel is timed
    // with that kernel: its per-tile write-out costs more on small tiles than
    // the forces alone show.
    const bool fused = b->lp.fuse;
    FusedKeep keep;
    if (fused) {
        const int rk = fused_keep(b, keep);
        if (rk) return rk;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    int bt[3] = {0, 0, 0}, bthreads = 0;
    int rc = DPD_OK;
    for (const int threads : dpd::kForceBlocks)
    for (const auto& c : cand) {
        if (rc) break;
        if ((size_t)tile_for(b, c, threads).lds_bytes > kLdsLimit) continue;
        for (int k = 0; k < 3; ++k) b->tile_req[k] = c[k];
        b->threads_req = threads;
        rc = push_desc(b);
        if (rc) break;
        float ms = 0.0f;
        hipError_t e = dpd::launch_force(b->lp, b->stream, fused);          // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = dpd::launch_force(b->lp, b->stream, fused);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = fail(DPD_EDEVICE, "dpd_tune_tile: %s", hipGetErrorString(e));
            break;
        }
        const double per = ms / reps;
        if (per < best) {
            best = per;
            for (int k = 0; k < 3; ++k) bt[k] = b->hd.tc.T[k];
            bthreads = threads;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (fused) {
        const int rr = fused_restore(b, keep);
        if (rr) return rr;
    }
    const bool won = rc == DPD_OK && bt[0] > 0;
    for (int k = 0; k < 3; ++k) b->tile_req[k] = won ? bt[k] : saved[k];
    b->threads_req = won ? bthreads : saved_threads;
    b->have_force = false;
    b->graph_dirty = true;
    const int rc2 = push_desc(b);
    if (rc) return rc;
    if (rc2) return rc2;
    if (won && !key.empty()) tune_store(key, bt, bthreads, best);
    for (int k = 0; k < 3; ++k) tile_out[k] = bt[k];
    if (ms_out) *ms_out = best;
    return DPD_OK;
}

int dpd_read(dpd_box b, int what, float* out_n3, int where)
{
    if (!b) return fail(DPD_EINVAL, "dpd_read: null box");
    if (where != DPD_HOST && where != DPD_DEVICE) return fail(DPD_EINVAL, "dpd_read: bad `where`");
    if (b->n > 0 && !out_n3) return fail(DPD_EINVAL, "dpd_read: null output");
    if (!b->have_state) return fail(DPD_ESTATE, "dpd_read: no state loaded");
    const dpd::BoxDesc& d = b->hd;
    float* dst = where == DPD_DEVICE ? out_n3 : b->out;
    switch (what) {
    case DPD_POS:
        HIPCHK(dpd::launch_to_rows(d.pos_a, nullptr, 0.0f, d.pos_a, b->n, dst, b->stream));
        break;
    case DPD_VEL:
        HIPCHK(dpd::launch_to_rows(d.vel_a, nullptr, 0.0f, d.pos_a, b->n, dst, b->stream));
        break;
    case DPD_FORCE:
        if (!b->have_force) return fail(DPD_ESTATE, "dpd_read: no forces (step first)");
        HIPCHK(dpd::launch_to_rows(d.force, nullptr, 0.0f, d.pos_b, b->n, dst, b->stream));
        break;
    case DPD_VEL_CENTRED:
        if (!b->have_force) return fail(DPD_ESTATE, "dpd_read: no forces (step first)");
        HIPCHK(dpd::launch_to_rows(d.vel_a, d.force, (float)(-0.5 * b->params.dt / b->params.mass), d.pos_b, b->n,
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
    const dpd::BoxDesc& d = b->hd;
    const size_t pb = (size_t)b->n * sizeof(float4);
    if (pos4 && b->n > 0) HIPCHK(hipMemcpyAsync(pos4, d.pos_b, pb, kind_to(where), b->stream));
    if (vel4 && b->n > 0) HIPCHK(hipMemcpyAsync(vel4, d.vel_b, pb, kind_to(where), b->stream));
    if (cell_start)
        HIPCHK(hipMemcpyAsync(cell_start, d.cell_start, (size_t)(b->nc + 1) * sizeof(int), kind_to(where), b->stream));
    return sync_box(b);
}

int dpd_get_stats(dpd_box b, dpd_stats* out)
{
    if (!b || !out) return fail(DPD_EINVAL, "dpd_get_stats: null argument");
    dpd::DevStats s;
    HIPCHK(hipMemcpyAsync(&s, b->hd.st, sizeof s, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    dpd::stats_from_device(s, out);
    if (s.nonfinite) return fail(DPD_ENONFINITE, "dpd_get_stats: non-finite value seen");
    return DPD_OK;
}

int dpd_get_profile(dpd_box b, double* sum_v, double* count, int32_t nbins)
{
    if (!b || !sum_v || !count) return fail(DPD_EINVAL, "dpd_get_profile: null argument");
    if (!b->have_params || nbins != b->params.profile_bins || nbins <= 0)
        return fail(DPD_EINVAL, "dpd_get_profile: nbins must equal params.profile_bins (> 0)");
    std::vector<long long> buf((size_t)nbins * 2);
    HIPCHK(hipMemcpyAsync(buf.data(), b->hd.profile, (size_t)nbins * 2 * sizeof(long long), hipMemcpyDeviceToHost,
                          b->stream));
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
    char* base = (char*)b->hd.st;
    const size_t off = offsetof(dpd::DevStats, sum_kT_centred);
    const size_t len = offsetof(dpd::DevStats, nsamples) + sizeof(unsigned long long) - off;
    HIPCHK(hipMemsetAsync(base + off, 0, len, b->stream));
    HIPCHK(hipMemsetAsync(b->hd.profile, 0, (size_t)dpd::kProfileMaxBins * 2 * sizeof(long long), b->stream));
    return DPD_OK;
}

int dpd_destroy(dpd_box b)
{
    if (!b) return DPD_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    b->graphs.release();
    delete b;
    if (e != hipSuccess) return fail(DPD_EDEVICE, "dpd_destroy: %s", hipGetErrorString(e));
    return DPD_OK;
}

}  // extern "C"

// ---- a box in the library's own device memory (dpd_run_static) -------------
//
// Each GPU the library runs on holds one copy of this array until the process
// ends.  In host code its name is only a host-side stand-in: the device
// address of the current GPU's copy comes from hipGetSymbolAddress, once per
// device, and only that address is ever handed to a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[DPD_STATIC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`.
int scratch_ptr(void** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DPD_EDEVICE, "dpd_run_static: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DPD_EDEVICE, "dpd_run_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DPD_OK;
}

// The run of dpd_run_static on box b laid out in the static array.
int run_static_on(dpd_box_s* b, const dpd_params* params, uint64_t seed, uint64_t step0, const float* pos_n3,
                  const float* vel_n3, int64_t nsteps, float* pos_out_n3, float* vel_out_n3, dpd_stats* stats)
{
    int rc = dpd_set_params(b, params);
    if (rc == DPD_OK) rc = dpd_set_seed(b, seed);
    if (rc == DPD_OK) rc = dpd_set_state(b, pos_n3, vel_n3, DPD_DEVICE);
    if (rc == DPD_OK && step0 != 0) rc = dpd_set_step(b, step0);
    if (rc != DPD_OK) return rc;
    if (nsteps > 0) {
        // the steps of dpd_step, launched directly (instantiating a graph
        // would allocate), then the fold of the last step's reductions
        HIPCHK(enqueue_steps(b->lp, nsteps, b->stream));
        HIPCHK(dpd::launch_fold(b->lp, b->stream));
        b->keys_valid = true;
        b->have_force = true;
    }
    if ((rc = dpd_read(b, DPD_POS, pos_out_n3, DPD_DEVICE)) || (rc = dpd_read(b, DPD_VEL, vel_out_n3, DPD_DEVICE)))
        return rc;
    if (stats) return dpd_get_stats(b, stats);
    return sync_box(b);
}

}  // namespace

extern "C" {

int dpd_run_static(const dpd_geom* geom, const dpd_params* params, uint64_t seed, uint64_t step0,
                   const float* pos_n3, const float* vel_n3, int64_t nsteps, float* pos_out_n3, float* vel_out_n3,
                   dpd_stats* stats, void* hip_stream)
{
    if (!geom || !params) return fail(DPD_EINVAL, "dpd_run_static: null geometry or params");
    if (!geom_ok(geom)) return fail(DPD_EINVAL, "dpd_run_static: invalid geometry (cells in 3..4096, 0 <= n <= (2^31 - 1) / 3)");
    if (nsteps < 0) return fail(DPD_EINVAL, "dpd_run_static: nsteps < 0");
    const int64_t nc = (int64_t)geom->cells[0] * geom->cells[1] * geom->cells[2];
    const size_t need = dpd::make_layout(geom->n, nc).total;
    if (need > (size_t)DPD_STATIC_WS_BYTES)
        return fail(DPD_ENOMEM, "dpd_run_static: the box needs %zu bytes of workspace, more than the %zu bytes of "
                    "the library's static array (DPD_STATIC_WS_BYTES); use dpd_create with a workspace",
                    need, (size_t)DPD_STATIC_WS_BYTES);
    if (geom->n > 0 && (!pos_n3 || !vel_n3 || !pos_out_n3 || !vel_out_n3))
        return fail(DPD_EINVAL, "dpd_run_static: null particle array");
    void* ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc) return rc;
    dpd_box_s b;                        // host object only: nothing of it outlives the call
    rc = box_init(&b, geom, ws, hip_stream);
    if (rc == DPD_OK)
        rc = run_static_on(&b, params, seed, step0, pos_n3, vel_n3, nsteps, pos_out_n3, vel_out_n3, stats);
    const hipError_t e = hipStreamSynchronize(b.stream);
    if (rc == DPD_OK && e != hipSuccess) rc = fail(DPD_EDEVICE, "dpd_run_static: %s", hipGetErrorString(e));
    return rc;
}

// ---- batches ------------------------------------------------------------------

int dpd_batch_workspace_bytes(int32_t nboxes, size_t* bytes)
{
    if (nboxes < 1 || nboxes > 65536 || !bytes) return fail(DPD_EINVAL, "dpd_batch_workspace_bytes: bad arguments");
    *bytes = align256((size_t)nboxes * sizeof(dpd::BoxDesc)) + align256((size_t)dpd::kNumWork * (nboxes + 1) * sizeof(int));
    return DPD_OK;
}

}  // extern "C"

namespace {

// Copy the member boxes' descriptors into the batch table and rebuild the
// prefix tables (boxes' parameters may have changed since creation).
int batch_refresh(dpd_batch_s* bt)
{
    const int nb = (int)bt->boxes.size();
    std::vector<dpd::BoxDesc> h(nb);
    bt->pre.assign((size_t)dpd::kNumWork * (nb + 1), 0);
    int lds = 0;
    bool virial = false, species = false, walls = false;
    // one launch has one workgroup size: the first box's; the others are
    // laid out for it in the batch's copy of their descriptors
    const int threads = nb > 0 ? bt->boxes[0]->hd.tc.threads : dpd::kForceBlock;
    for (int i = 0; i < nb; ++i) {
        h[i] = bt->boxes[i]->hd;
        if (h[i].tc.threads != threads) h[i].tc = tile_for(bt->boxes[i], bt->boxes[i]->tile_req, threads);
        lds = std::max(lds, h[i].tc.lds_bytes);
        virial |= (h[i].flags & DPD_FLAG_VIRIAL) != 0;
        species |= bt->boxes[i]->lp.species;
        walls |= bt->boxes[i]->lp.walls;
        for (int k = 0; k < dpd::kNumWork; ++k)
            bt->pre[(size_t)k * (nb + 1) + i + 1] = bt->pre[(size_t)k * (nb + 1) + i] + dpd::box_work(h[i], k);
    }
    bool changed = bt->lp.lds_force != lds || bt->lp.any_virial != virial || bt->lp.species != species ||
                   bt->lp.walls != walls || bt->lp.force_threads != threads || !bt->lp.fuse;
    for (int k = 0; k < dpd::kNumWork; ++k) {
        const int tot = bt->pre[(size_t)k * (nb + 1) + nb];
        changed |= bt->lp.total[k] != tot;
        bt->lp.total[k] = tot;
    }
    bt->lp.desc = bt->d_desc;
    bt->lp.pre = bt->d_pre;
    bt->lp.nbox = nb;
    bt->lp.lds_force = lds;
    bt->lp.any_virial = virial;
    bt->lp.species = species;
    bt->lp.walls = walls;
    bt->lp.force_threads = threads;
    bt->lp.reference_force = false;     // reference boxes take the gather path inside the tile kernel
    bt->lp.fuse = true;
    if (changed) bt->graph_dirty = true;   // launch shape changed: capture again
    HIPCHK(dpd::force_tiled_prepare(lds));
    // the tables go through pinned memory, so the copies are queued behind
    // the work already on the batch stream without the host waiting for it
    const size_t desc_bytes = (size_t)nb * sizeof(dpd::BoxDesc), pre_bytes = bt->pre.size() * sizeof(int);
    const int k = bt->stage_next;
    bt->stage_next ^= 1;
    if (bt->stage_used[k]) HIPCHK(hipEventSynchronize(bt->stage_done[k]));   // its last copy has run
    if (bt->stage_bytes[k] < desc_bytes + pre_bytes) {
        if (bt->stage[k]) HIPCHK(hipHostFree(bt->stage[k]));
        bt->stage[k] = nullptr;
        bt->stage_bytes[k] = 0;
        HIPCHK(hipHostMalloc((void**)&bt->stage[k], desc_bytes + pre_bytes, hipHostMallocDefault));
        bt->stage_bytes[k] = desc_bytes + pre_bytes;
    }
    std::memcpy(bt->stage[k], h.data(), desc_bytes);
    std::memcpy(bt->stage[k] + desc_bytes, bt->pre.data(), pre_bytes);
    HIPCHK(hipMemcpyAsync(bt->d_desc, bt->stage[k], desc_bytes, hipMemcpyHostToDevice, bt->stream));
    HIPCHK(hipMemcpyAsync(bt->d_pre, bt->stage[k] + desc_bytes, pre_bytes, hipMemcpyHostToDevice, bt->stream));
    HIPCHK(hipEventRecord(bt->stage_done[k], bt->stream));
    bt->stage_used[k] = true;
    return DPD_OK;
}

// Release what a batch holds (after its stream has drained).
void batch_free(dpd_batch_s* bt)
{
    bt->graphs.release();
    for (int k = 0; k < 2; ++k) {
        if (bt->stage[k]) (void)hipHostFree(bt->stage[k]);
        if (bt->stage_done[k]) (void)hipEventDestroy(bt->stage_done[k]);
    }
    if (bt->done) (void)hipEventDestroy(bt->done);
    if (bt->pending) (void)hipEventDestroy(bt->pending);
    delete bt;
}

}  // namespace

extern "C" {

int dpd_batch_create(const dpd_box* boxes, int32_t nboxes, void* dev_ws, size_t ws_bytes, void* hip_stream,
                     dpd_batch* out)
{
    if (!out) return fail(DPD_EINVAL, "dpd_batch_create: null output");
    *out = nullptr;
    size_t need = 0;
    const int rc0 = dpd_batch_workspace_bytes(nboxes, &need);
    if (rc0) return rc0;
    if (!boxes) return fail(DPD_EINVAL, "dpd_batch_create: null box list");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(DPD_EINVAL, "dpd_batch_create: workspace null or misaligned");
    if (ws_bytes < need) return fail(DPD_ENOMEM, "dpd_batch_create: workspace of %zu bytes, %zu needed", ws_bytes, need);
    for (int i = 0; i < nboxes; ++i) {
        if (!boxes[i]) return fail(DPD_EINVAL, "dpd_batch_create: null box %d", i);
        for (int j = 0; j < i; ++j)
            if (boxes[j] == boxes[i]) return fail(DPD_EINVAL, "dpd_batch_create: box %d listed twice", i);
    }
    dpd_batch_s* bt = new (std::nothrow) dpd_batch_s();
    if (!bt) return fail(DPD_ENOMEM, "dpd_batch_create: host allocation failed");
    bt->boxes.assign(boxes, boxes + nboxes);
    // the tables are laid out for as many boxes as the workspace holds, so a
    // batch can later take other boxes (the request server's use)
    int cap = nboxes;
    for (int step = 32768; step > 0; step >>= 1) {
        size_t b = 0;
        if (cap + step <= 65536 && dpd_batch_workspace_bytes(cap + step, &b) == DPD_OK && b <= ws_bytes) cap += step;
    }
    bt->capacity = cap;
    bt->stream = (hipStream_t)hip_stream;
    bt->d_desc = (dpd::BoxDesc*)dev_ws;
    bt->d_pre = (int*)((char*)dev_ws + align256((size_t)cap * sizeof(dpd::BoxDesc)));
    bt->lp.lds_force = -1;
    hipError_t e = hipEventCreateWithFlags(&bt->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->pending, hipEventDisableTiming);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&bt->stage_done[k], hipEventDisableTiming);
    int rc = e == hipSuccess ? batch_refresh(bt) : fail(DPD_EDEVICE, "dpd_batch_create: %s", hipGetErrorString(e));
    if (rc) {
        (void)hipStreamSynchronize(bt->stream);
        batch_free(bt);
        return rc;
    }
    *out = bt;
    return DPD_OK;
}

int dpd_batch_tune(dpd_batch bt, int32_t reps, int32_t tile_out[3], double* ms_out)
{
    if (!bt || !tile_out) return fail(DPD_EINVAL, "dpd_batch_tune: null argument");
    if (reps < 1 || reps > 1000) return fail(DPD_EINVAL, "dpd_batch_tune: reps must be in 1..1000");
    for (size_t i = 0; i < bt->boxes.size(); ++i) {
        dpd_box_s* b = bt->boxes[i];
        if (!ready(b)) return fail(DPD_ESTATE, "dpd_batch_tune: box %zu lacks params, seed or state", i);
        if (b->binned) return fail(DPD_ESTATE, "dpd_batch_tune: box %zu holds a bare cell list", i);
        if (b->params.flags & DPD_FLAG_REFERENCE_FORCE)
            return fail(DPD_EINVAL, "dpd_batch_tune: box %zu takes the reference force path", i);
    }
    for (dpd_box_s* b : bt->boxes) HIPCHK(hipStreamSynchronize(b->stream));
    int rc = batch_refresh(bt);
    if (rc) return rc;
    HIPCHK(dpd::launch_bin(bt->lp, bt->stream));   // cell lists of the current state, for every timing
    for (dpd_box_s* b : bt->boxes) {
        b->binned = true;
        b->keys_valid = false;
        b->have_force = false;
        b->graph_dirty = true;
    }
    std::vector<std::array<int, 3>> saved;
    std::vector<int> saved_threads;
    for (dpd_box_s* b : bt->boxes) {
        saved.push_back({b->tile_req[0], b->tile_req[1], b->tile_req[2]});
        saved_threads.push_back(b->threads_req);
    }
    std::string key;
    if (tune_cache_on()) {
        key = tune_key_prefix(bt->stream) + "batch";
        for (size_t i = 0; i < bt->boxes.size(); ++i) {
            const dpd_box_s* b = bt->boxes[i];
            char own[48];
            std::snprintf(own, sizeof own, "/t%dx%dx%d@%d", b->tile_req[0], b->tile_req[1], b->tile_req[2],
                          b->threads_req);
            key += "|" + box_tune_part(b) + own;
        }
        TuneEntry e;
        bool usable = tune_lookup(key, &e) && (e.threads == 256 || e.threads == 512 || e.threads == 1024);
        const bool uniform = usable && e.tile[0] > 0;
        for (size_t i = 0; i < bt->boxes.size() && usable; ++i) {
            const int* t = uniform ? e.tile : saved[i].data();
            usable = (size_t)tile_for(bt->boxes[i], t, e.threads).lds_bytes <= kLdsLimit;
        }
        if (usable) {
            for (size_t i = 0; i < bt->boxes.size() && rc == DPD_OK; ++i) {
                dpd_box_s* b = bt->boxes[i];
                for (int k = 0; k < 3; ++k) b->tile_req[k] = uniform ? e.tile[k] : saved[i][k];
                b->threads_req = e.threads;
                rc = push_desc(b);
            }
            if (rc == DPD_OK) rc = batch_refresh(bt);
            if (rc) return rc;
            for (int k = 0; k < 3; ++k) tile_out[k] = uniform ? e.tile[k] : 0;
            if (ms_out) *ms_out = e.ms;
            return DPD_OK;
        }
    }
    // batches step with the fused kernel: timed with it, every box's state
    // and diagnostics put back afterwards
    const bool fused = bt->lp.fuse;
    std::vector<FusedKeep> keep(fused ? bt->boxes.size() : 0);
    if (fused) HIPCHK(hipStreamSynchronize(bt->stream));   // the binning above (and its fold) is done
    for (size_t i = 0; i < keep.size(); ++i) {
        const int rk = fused_keep(bt->boxes[i], keep[i]);
        if (rk) return rk;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    int bt3[3] = {0, 0, 0}, bthreads = 0;
    bool have_best = false;
    const int ncand = (int)(sizeof kTuneCand / sizeof kTuneCand[0]);
    for (const int threads : dpd::kForceBlocks)
    for (int ci = -1; ci < ncand && rc == DPD_OK; ++ci) {      // -1: the boxes' own tiles
        bool fits = true;
        for (size_t i = 0; i < bt->boxes.size() && fits; ++i) {
            dpd_box_s* b = bt->boxes[i];
            const int* t = ci < 0 ? saved[i].data() : kTuneCand[ci];
            fits = (size_t)tile_for(b, t, threads).lds_bytes <= kLdsLimit;
        }
        if (!fits) continue;
        for (size_t i = 0; i < bt->boxes.size() && rc == DPD_OK; ++i) {
            dpd_box_s* b = bt->boxes[i];
            const int* t = ci < 0 ? saved[i].data() : kTuneCand[ci];
            for (int k = 0; k < 3; ++k) b->tile_req[k] = t[k];
            b->threads_req = threads;
            rc = push_desc(b);
        }
        if (rc == DPD_OK) rc = batch_refresh(bt);
        if (rc) break;
        float ms = 0.0f;
        hipError_t e = dpd::launch_force(bt->lp, bt->stream, fused);     // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, bt->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = dpd::launch_force(bt->lp, bt->stream, fused);
        if (e == hipSuccess) e = hipEventRecord(e1, bt->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = fail(DPD_EDEVICE, "dpd_batch_tune: %s", hipGetErrorString(e));
            break;
        }
        const double per = ms / reps;
        if (per < best) {
            best = per;
            have_best = true;
            for (int k = 0; k < 3; ++k) bt3[k] = ci < 0 ? 0 : kTuneCand[ci][k];
            bthreads = threads;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (fused) {
        HIPCHK(hipStreamSynchronize(bt->stream));
        for (size_t i = 0; i < keep.size(); ++i) {
            const int rr = fused_restore(bt->boxes[i], keep[i]);
            if (rr) return rr;
        }
    }
    // apply the winner (or restore the boxes' own tiles)
    int rc2 = DPD_OK;
    for (size_t i = 0; i < bt->boxes.size() && rc2 == DPD_OK; ++i) {
        dpd_box_s* b = bt->boxes[i];
        const bool ok = rc == DPD_OK && have_best;
        const bool uniform = ok && bt3[0] > 0;
        for (int k = 0; k < 3; ++k) b->tile_req[k] = uniform ? bt3[k] : saved[i][k];
        b->threads_req = ok ? bthreads : saved_threads[i];
        rc2 = push_desc(b);
    }
    if (rc2 == DPD_OK) rc2 = batch_refresh(bt);
    if (rc) return rc;
    if (rc2) return rc2;
    if (have_best && !key.empty()) tune_store(key, bt3, bthreads, best);
    for (int k = 0; k < 3; ++k) tile_out[k] = bt3[k];
    if (ms_out) *ms_out = best;
    return DPD_OK;
}

int dpd_set_tune_cache(const char* path)
{
    TuneCacheFile& f = tune_file();
    std::lock_guard<std::mutex> lk(f.mu);
    f.path = path ? path : "";
    f.entries.clear();
    if (!f.path.empty()) tune_read(f);
    return DPD_OK;
}

int dpd_batch_step(dpd_batch bt, int64_t nsteps)
{
    if (!bt) return fail(DPD_EINVAL, "dpd_batch_step: null batch");
    if (nsteps < 0) return fail(DPD_EINVAL, "dpd_batch_step: nsteps < 0");
    size_t nbinned = 0;
    for (size_t i = 0; i < bt->boxes.size(); ++i) {
        dpd_box_s* b = bt->boxes[i];
        if (!ready(b)) return fail(DPD_ESTATE, "dpd_batch_step: box %zu lacks params, seed or state", i);
        nbinned += b->binned ? 1 : 0;
    }
    if (nbinned != 0 && nbinned != bt->boxes.size())
        return fail(DPD_ESTATE, "dpd_batch_step: %zu of %zu boxes hold a bare cell list; step them once alone",
                    nbinned, bt->boxes.size());
    if (nsteps == 0) return DPD_OK;
    // the run waits (on the device) for what is queued on the boxes' own streams
    for (dpd_box_s* b : bt->boxes)
        if (b->stream != bt->stream) {
            HIPCHK(hipEventRecord(bt->pending, b->stream));
            HIPCHK(hipStreamWaitEvent(bt->stream, bt->pending, 0));
        }
    int rc = batch_refresh(bt);
    if (rc) return rc;
    // One graph holds the whole run (up to kBatchGraphMax steps), so a run is
    // a single launch; longer runs replay it.  Short runs (a serving quantum
    // on a changing set of boxes) are launched directly.
    const int64_t left = nsteps - (nbinned ? 1 : 0);
    const bool graphs = nsteps >= kBatchGraphMin;
    const RunPlan rp = graphs ? plan_run(left, kBatchGraphMax) : RunPlan{};
    hipGraphExec_t gfull = nullptr, gtail = nullptr;
    if (rp.full && (rc = graph_for(bt->graphs, bt->graph_dirty, bt->lp, rp.g, &gfull))) return rc;
    if (rp.tail && (rc = graph_for(bt->graphs, bt->graph_dirty, bt->lp, rp.tail, &gtail))) return rc;
    if (nbinned) {                       // first step reuses the cell lists
        HIPCHK(enqueue_step_tail(bt->lp, bt->stream));
        for (dpd_box_s* b : bt->boxes) b->binned = false;
    }
    if (graphs) {
        for (int64_t k = 0; k < rp.full; ++k) HIPCHK(hipGraphLaunch(gfull, bt->stream));
        if (rp.tail) HIPCHK(hipGraphLaunch(gtail, bt->stream));
        if (left == 0) HIPCHK(dpd::launch_fold(bt->lp, bt->stream));
    } else {
        HIPCHK(enqueue_steps(bt->lp, left, bt->stream));
        HIPCHK(dpd::launch_fold(bt->lp, bt->stream));   // the last step's reductions
    }
    // later work on each box's own stream waits for the batch
    HIPCHK(hipEventRecord(bt->done, bt->stream));
    for (dpd_box_s* b : bt->boxes) {
        if (b->stream != bt->stream) HIPCHK(hipStreamWaitEvent(b->stream, bt->done, 0));
        b->keys_valid = true;
        b->have_force = true;
        b->binned = false;
    }
    return DPD_OK;
}

int dpd_batch_destroy(dpd_batch bt)
{
    if (!bt) return DPD_OK;
    hipError_t e = hipStreamSynchronize(bt->stream);
    batch_free(bt);
    if (e != hipSuccess) return fail(DPD_EDEVICE, "dpd_batch_destroy: %s", hipGetErrorString(e));
    return DPD_OK;
}

// ---- random-term diagnostics -----------------------------------------------

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

// ---- calls of the request server that do not synchronise (dpd_runtime.hpp) ----

namespace dpd {

int box_set_stream(dpd_box b, hipStream_t s)
{
    if (!b) return fail(DPD_EINVAL, "box_set_stream: null box");
    b->stream = s;
    b->graph_dirty = true;             // graphs are captured from the box stream's work
    return DPD_OK;
}

int box_enqueue_results(dpd_box b, float* pos_n3, float* vel_n3, DevStats* dev_stats)
{
    if (!b || !dev_stats || (b->n > 0 && (!pos_n3 || !vel_n3)))
        return fail(DPD_EINVAL, "box_enqueue_results: null argument");
    if (!b->have_state) return fail(DPD_ESTATE, "box_enqueue_results: no state loaded");
    const BoxDesc& d = b->hd;
    const size_t bytes = (size_t)b->n * 3 * sizeof(float);
    if (b->n > 0) {
        // both quantities pass through the box's staging rows in turn (stream order)
        HIPCHK(launch_to_rows(d.pos_a, nullptr, 0.0f, d.pos_a, b->n, b->out, b->stream));
        HIPCHK(hipMemcpyAsync(pos_n3, b->out, bytes, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(launch_to_rows(d.vel_a, nullptr, 0.0f, d.pos_a, b->n, b->out, b->stream));
        HIPCHK(hipMemcpyAsync(vel_n3, b->out, bytes, hipMemcpyDeviceToHost, b->stream));
    }
    HIPCHK(hipMemcpyAsync(dev_stats, d.st, sizeof(DevStats), hipMemcpyDeviceToHost, b->stream));
    return DPD_OK;
}

void stats_from_device(const DevStats& s, dpd_stats* out)
{
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
}

void box_release(dpd_box b)
{
    if (!b) return;
    b->graphs.release();
    delete b;
}

int batch_set_boxes(dpd_batch bt, const dpd_box* boxes, int32_t nboxes)
{
    if (!bt || (nboxes > 0 && !boxes)) return fail(DPD_EINVAL, "batch_set_boxes: null argument");
    if (nboxes < 1 || nboxes > bt->capacity)
        return fail(DPD_EINVAL, "batch_set_boxes: %d boxes, the tables hold 1..%d", nboxes, bt->capacity);
    for (int i = 0; i < nboxes; ++i)
        if (!boxes[i]) return fail(DPD_EINVAL, "batch_set_boxes: null box %d", i);
    bt->boxes.assign(boxes, boxes + nboxes);
    bt->graph_dirty = true;
    return batch_refresh(bt);
}

}  // namespace dpd
