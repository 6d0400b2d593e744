// dpd_internal.hpp -- data layout shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dpd_device.hpp"

namespace dpd {

constexpr int kBlock = 256;             // threads per block of the streaming kernels
constexpr int kForceBlock = 512;        // default threads per workgroup of the tiled pair-force kernel
constexpr int kForceBlocks[3] = {256, 512, 1024};   // the instantiated workgroup sizes
constexpr int kScanChunk = 512;         // cells per block of the cell-count scan (2 per thread)
constexpr int kSubChunk = 64;             // cells per device counter of the chunk sums
static_assert(kScanChunk % kSubChunk == 0, "chunks are whole sub-chunks");
constexpr int kIntegrateMaxBlocks = 2048;
constexpr int kProfileMaxBins = 4096;
constexpr int kPartials = 5;            // P_x, P_y, P_z, KE_half, KE_centred
constexpr int kFlagVirial = 1;          // DPD_FLAG_VIRIAL
constexpr int kFlagReference = 2;       // DPD_FLAG_REFERENCE_FORCE
constexpr int kMaxTypes = 8;            // species of one box (DPD_MAX_TYPES)
constexpr int kFrozenBit = 256;         // in the velocity's .w (an int): a frozen wall particle
constexpr int kFlagBodyUniform = 4;     // DPD_FLAG_BODY_UNIFORM

// Fixed-point scale of the flow-profile and virial accumulators.
constexpr double kProfScale = 16777216.0;      // 2^24 units per velocity unit
constexpr double kVirScale = 16777216.0;       // 2^24 units per virial unit

// Device-resident counters and reductions.  Written only by kernels after
// creation; read back by dpd_get_stats.
struct DevStats {
    unsigned long long step;        // force evaluations since set_state
    unsigned int fold_pending;      // integrate partials not yet folded into the reductions
    int nonfinite;
    int escaped;
    unsigned int fold_count;        // partials the pending fold adds up (integrate blocks or force tiles)
    double last[kPartials];         // reductions of the last step
    double sum_kT_centred;
    double sum_pressure;
    double sum_momentum[3];
    unsigned long long nsamples;
    long long virial_fx;            // conservative virial of the current step (fixed point)
    double last_virial;
    double last_pressure;
    double last_kT_centred;
};

// Per-step constants of the integrate kernel.
struct StepConst {
    float dt;          // time step
    float dtm;         // dt / m
    float half_dtm;    // dt / (2 m)
    float q;           // position grid
    float inv_q;
    float L[3];
    int cells[3];
    int flow_axis, grad_axis, nbins;
    float grad_scale;  // nbins / L_grad
    double mass;
    double inv_dof;    // 1 / (3 (N - 1)), N = particles not frozen  (0 when N < 2)
    double inv_vol;
    double rho;
    int wall_kind;     // DPD_WALL_*
    float wall_h;      // plate half-gap, pipe radius or outer cylinder radius
    float centre[3];   // L / 2
    float wall_r_in;   // inner cylinder radius
    float omega[2];    // angular velocities of the inner and outer cylinder
    float rot[2][2];   // (cos, sin) of omega dt: the per-step turn of each cylinder's frozen layer
};

// Signed distance to the wall surface: negative in the fluid.
__device__ __forceinline__ float wall_sdf(float x, float y, float z, const StepConst& sc)
{
    const float r[3] = {x - sc.centre[0], y - sc.centre[1], z - sc.centre[2]};
    if (sc.wall_kind == 1) return fabsf(r[sc.grad_axis]) - sc.wall_h;
    float q2 = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) q2 += k == sc.flow_axis ? 0.0f : r[k] * r[k];
    const float q = sqrtf(q2);
    return sc.wall_kind == 2 ? q - sc.wall_h : fmaxf(sc.wall_r_in - q, q - sc.wall_h);
}

// Offsets (c1, c2) of a point from the cylinders' axis along the two axes
// after flow_axis (right-handed about it), and which cylinder it belongs to
// (0 inner, 1 outer).  Selects, not indexed arrays, keep it in registers.
__device__ __forceinline__ float pick3(int k, float a, float b, float c) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ __forceinline__ int cylinder_of(float x, float y, float z, const StepConst& sc, float& c1, float& c2)
{
    const float rx = x - sc.centre[0], ry = y - sc.centre[1], rz = z - sc.centre[2];
    const int a1 = sc.flow_axis == 2 ? 0 : sc.flow_axis + 1;
    const int a2 = sc.flow_axis == 0 ? 2 : sc.flow_axis - 1;
    c1 = pick3(a1, rx, ry, rz);
    c2 = pick3(a2, rx, ry, rz);
    return sqrtf(c1 * c1 + c2 * c2) < 0.5f * (sc.wall_r_in + sc.wall_h) ? 0 : 1;
}

// Components along x, y, z of the vector (0 along flow_axis, c1, c2).
__device__ __forceinline__ float3 from_axes(const StepConst& sc, float c1, float c2)
{
    const int a1 = sc.flow_axis == 2 ? 0 : sc.flow_axis + 1;
    return make_float3(a1 == 0 ? c1 : (sc.flow_axis == 1 ? c2 : 0.0f),
                       a1 == 1 ? c1 : (sc.flow_axis == 2 ? c2 : 0.0f),
                       a1 == 2 ? c1 : (sc.flow_axis == 0 ? c2 : 0.0f));
}

// Velocity of the wall at a point: omega x r for the cylinders, else 0.
__device__ __forceinline__ float3 wall_velocity(float x, float y, float z, const StepConst& sc)
{
    if (sc.wall_kind != 3) return make_float3(0.0f, 0.0f, 0.0f);
    float c1, c2;
    const float om = sc.omega[cylinder_of(x, y, z, sc, c1, c2)];
    return from_axes(sc, -om * c2, om * c1);
}

struct ForceConst {
    PairConst pc;
    float L[3];
    int cells[3];
    float body_f;
    int flow_axis, grad_axis;
    float half_grad;   // L_grad / 2
    int body_uniform;  // 1: +body_f everywhere, 0: the two halves of Eq. 11
    int ntypes;        // species; > 1: each pair takes (a, gamma, sigma / sqrt(dt), 1 / r_c) from tab
    float4 tab[kMaxTypes * kMaxTypes];   // [s * kMaxTypes + t], symmetric
};

// Table entry of the species pair (s, t).  The species sit in the .w of the
// velocity (an int); the masks keep any value inside the table.
__device__ __forceinline__ int species_pair(int s, int t) { return ((s & (kMaxTypes - 1)) * kMaxTypes) | (t & (kMaxTypes - 1)); }

// Tiling of the box for the LDS pair-force kernel, with the byte offsets of
// its dynamic LDS buffers.
struct TileConst {
    int T[3];          // tile edge in cells (clamped to the box)
    int ntile[3];      // tiles per axis (the last one may be ragged)
    int ntiles;
    int ux;            // cells per home unit of the candidate search (consecutive in x)
    int smax;          // staged particles (tile + halo) that fit the LDS buffers
    int pmax;          // tile particles that fit the accumulators
    int lds_bytes;
    int off_sv, off_acc, off_cst, off_cg, off_rows, off_ut, off_q;
    int threads;       // workgroup size the queue region is laid out for (a kForceBlocks entry)
};

// Everything a kernel needs about one box, in device memory.  The step
// kernels read it at run time, so parameters can change between launches
// of a captured graph.  A single box is a batch of one.
struct BoxDesc {
    float4 *pos_a, *vel_a;     // state in the previous cell order (or id order)
    float4 *pos_b, *vel_b;     // state binned into cell order
    float4* force;             // total force of the last step, cell order
    int2* keyslot;             // (cell, arrival slot) of pos_a
    int* perm;                 // cell order -> index into pos_a (arrival order)
    int* cellof;               // cell order -> cell of that position
    int* count;                // particles per cell (zeroed by the scan)
    int* cell_start;           // nc + 1
    int* bsum;                 // particles per kSubChunk cells (zeroed by the scatter)
    double* partials;          // FP64 partials of the last step (kPartials per integrate block or force tile)
    long long* profile;        // flow profile accumulators (sum, count) per slab
    DevStats* st;
    int n, nc, nchunks, nsub;
    int nblk_int;              // integrate blocks of this box (depends on n only)
    int flags;                 // DPD_FLAG_* of the box
    int pad0;
    ForceConst fc;
    StepConst sc;
    TileConst tc;
};

// Work decomposition of one launch group (a box, or a batch of boxes): per
// kernel kind, the exclusive prefix over boxes of the workgroups each box
// needs; a workgroup finds its box by binary search.
enum WorkKind { kWChunk = 0, kWPart = 1, kWTile = 2, kWInt = 3, kNumWork = 4 };

struct LaunchPlan {
    const BoxDesc* desc;       // device array [nbox]
    const int* pre;            // device array [kNumWork][nbox + 1]
    int nbox;
    int total[kNumWork];       // workgroups per kind
    int lds_force;             // dynamic LDS of the tile kernel (max over boxes)
    int force_threads;         // workgroup size of the tile kernel (every box's tc.threads)
    bool species;              // some box has several species: the tile kernel reads the pair table
    bool walls;                // some box has walls or frozen particles: the wall kick-drift
    bool any_virial;
    bool reference_force;      // single box flagged DPD_FLAG_REFERENCE_FORCE
    bool fuse;                 // the tile kernel integrates each particle once its force is final
                               // (every launch of the tile kernel; not the reference force path)
};

// Layout of a box inside its caller-provided workspace.  All offsets are
// 256-byte aligned.
struct Layout {
    size_t pos_a, vel_a;      // float4[n]  state, previous cell order (or id order)
    size_t pos_b, vel_b;      // float4[n]  state binned into cell order
    size_t force;             // float4[n]  total force of the last step, cell order
    size_t keyslot;           // int2[n]    (cell, arrival slot) of pos_a
    size_t perm;              // int[n]     cell order -> index into pos_a (unstable)
    size_t cellof;            // int[n]     cell order -> cell
    size_t out;               // float[3n]  staging of reads and writes in id order
    size_t count;             // int[nc]    particles per cell
    size_t cell_start;        // int[nc+1]
    size_t bsum;              // int[nsub]
    size_t partials;          // double[max(kIntegrateMaxBlocks, nc) * kPartials]: per block or per tile
    size_t profile;           // long long[kProfileMaxBins * 2] (sum, count)
    size_t stats;             // DevStats
    size_t flags;             // int[4] scratch flags
    size_t desc;              // BoxDesc
    size_t pre;               // int[kNumWork * 2] launch prefixes of the box alone
    size_t total;
};

Layout make_layout(int64_t n, int64_t nc);
int set_error(int code, const char* msg);   // thread-local message behind dpd_last_error
int integrate_blocks(int n);
int box_work(const BoxDesc& d, int kind);

// ---- kernel launchers ------------------------------------------------------
hipError_t launch_fill_i32(int* p, int value, int64_t count, hipStream_t s);
hipError_t launch_load_state(const float* pos3, const float* vel3, int n, float4* pos, float4* vel,
                             float q, float inv_q, const float* L, int* bad, hipStream_t s);
hipError_t launch_init_random(int n, const float* L, float q, double vscale, uint64_t seed, float4* pos, float4* vel,
                              double* scratch, int scratch_doubles, hipStream_t s);
hipError_t launch_keys(const float4* pos, int n, const int* cells, int* count, int* bsum, int2* keyslot,
                       hipStream_t s);
// species by id -> vel[i].w of the particle whose id is pos[i].w, and back
hipError_t launch_set_types(const float4* pos, float4* vel, int n, const int* type_by_id, hipStream_t s);
hipError_t launch_get_types(const float4* pos, const float4* vel, int n, int* type_by_id, hipStream_t s);
// frozen marks by id <-> the frozen bit of vel[i].w (frozen velocities set to 0)
hipError_t launch_set_frozen(const float4* pos, float4* vel, int n, const unsigned char* frozen_by_id,
                             const StepConst& sc, hipStream_t s);
hipError_t launch_get_frozen(const float4* pos, const float4* vel, int n, unsigned char* frozen_by_id, hipStream_t s);
hipError_t launch_wall_sdf(const float4* pos, int n, const StepConst& sc, float* sdf_by_id, hipStream_t s);
// Stage launchers.  t0 / t1 (optional): events that the first kernel of the
// stage records as it starts and the last as it ends (hipExtLaunchKernel), so
// that the events time the stage's kernels alone; null in normal steps and
// in captured graphs.
hipError_t launch_bin(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// integrate: a step's force launch, which also integrates when lp.fuse (the
// tuners and timers pass false: forces only, the state is left alone)
hipError_t launch_force(const LaunchPlan& lp, hipStream_t s, bool integrate, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
hipError_t launch_virial(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_integrate(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// A kernel launch that records t0 when it starts and t1 when it ends (either
// may be null; both null is a plain launch).
template <typename K, typename... A>
inline void launch_timed(K kernel, dim3 grid, dim3 block, unsigned lds, hipStream_t s, hipEvent_t t0, hipEvent_t t1,
                         A... args)
{
    if (t0 || t1)
        hipExtLaunchKernelGGL(kernel, grid, block, lds, s, t0, t1, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}
hipError_t launch_fold(const LaunchPlan& lp, hipStream_t s);
// rho: particles per occupied cell (the density the tile capacities are sized for)
TileConst make_tile_const(const int* cells, double rho, const int* tile, int threads, int smax_override,
                          int pmax_override);
hipError_t launch_count_nonempty(const int* count, int nc, int* out, hipStream_t s);
hipError_t force_tiled_prepare(int lds_bytes);
hipError_t launch_to_rows(const float4* src, const float4* sub, float sub_scale, const float4* idsrc, int n,
                          float* out3, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr4, const uint32_t* key2, int64_t n, uint32_t* out4, hipStream_t s);
hipError_t launch_box_muller(const uint32_t* w0, const uint32_t* w1, int64_t n, float* xi, hipStream_t s);

// Arrival slot in a per-cell counter, aggregated over runs of equal keys in
// a wave: lanes l0..l1 holding the same key (consecutive lanes) take one
// atomicAdd of the run length and slots base + (l - l0).  Particles in cell
// order mostly stay in their cell, so runs are about rho long.  Lanes with
// valid == false must pass key = -1.  All lanes of the wave must call both
// halves (arrival_issue, then arrival_finish).
struct ArrivalTicket {
    int base;       // counter value taken by the run head (head lanes)
    int my_head;    // lane of this lane's run head
};

// First half: issue the run heads' atomics.  The returned
// value is not needed until arrival_finish, so other work can hide the
// atomic's round trip.
__device__ __forceinline__ ArrivalTicket arrival_issue(int key, bool valid, int* __restrict__ count)
{
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const bool head = valid && (lane == 0 || prev != key);
    const unsigned long long heads = __ballot(head);
    const unsigned long long live = __ballot(valid);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    ArrivalTicket t;
    t.my_head = 63 - __clzll(heads & upto);                         // valid lanes only
    int run_end = 64;
    const unsigned long long after = heads & ~upto;
    if (after) run_end = __ffsll((long long)after) - 1;
    const int nlive = __popcll(live);                               // valid lanes are a prefix
    if (run_end > nlive) run_end = nlive;
    t.base = 0;
    if (head) t.base = gatomic_add(&count[key], run_end - lane);
    return t;
}

// Particle counts per sub-chunk of kSubChunk cells, one device atomic per
// run of equal sub-chunks in a wave.  Same-address device atomics
// serialise, so the counters are kept small enough that only a few waves
// (about kSubChunk rho / 64) add to each.  Same contract as arrival_issue;
// nothing is returned.
__device__ __forceinline__ void chunk_add(int key, bool valid, int* __restrict__ bsum)
{
    const int lane = threadIdx.x & 63;
    const int ck = valid ? key / kSubChunk : -1;
    const int prev = __shfl_up(ck, 1, 64);
    const bool head = valid && (lane == 0 || prev != ck);
    const unsigned long long heads = __ballot(head);
    const int nlive = __popcll(__ballot(valid));                    // valid lanes are a prefix
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const unsigned long long after = heads & ~upto;
    int run_end = after ? __ffsll((long long)after) - 1 : 64;
    if (run_end > nlive) run_end = nlive;
    if (head) gatomic_add(&bsum[ck], run_end - lane);
}

// Second half: every lane of the wave must call it.
__device__ __forceinline__ int arrival_finish(const ArrivalTicket& t, bool valid)
{
    const int lane = threadIdx.x & 63;
    const int base = __shfl(t.base, valid ? t.my_head : lane, 64);
    return base + (lane - t.my_head);
}

// Kick and drift of one free particle of a box without walls (Sec. 3.1,
// time-stepping step 5: v^{n+1/2} = v^{n-1/2} + dt f^n / m, then
// x^{n+1} = x^n + dt v^{n+1/2}), the position rounded to the grid q and
// wrapped into [0, L).  Shared by the integrate kernel and the force kernel's
// fused epilogue, so both compute the same bits.  A non-finite result keeps
// the old position (fin = false); esc reports a move of a cell or more, or a
// position that still fell outside the box (clamped inside).
struct Kicked {
    float nx, ny, nz;      // x^{n+1}
    float vx, vy, vz;      // v^{n+1/2}
    float vcx, vcy, vcz;   // v^{n-1/2} + dt f^n / (2 m): the time-centred velocity
    bool fin, esc;
};

__device__ __forceinline__ Kicked kick_drift(float4 x, float4 v, float4 f, const StepConst& sc)
{
    Kicked k;
    k.vcx = fmaf(f.x, sc.half_dtm, v.x);
    k.vcy = fmaf(f.y, sc.half_dtm, v.y);
    k.vcz = fmaf(f.z, sc.half_dtm, v.z);
    k.vx = fmaf(f.x, sc.dtm, v.x);
    k.vy = fmaf(f.y, sc.dtm, v.y);
    k.vz = fmaf(f.z, sc.dtm, v.z);
    float nx = fmaf(k.vx, sc.dt, x.x), ny = fmaf(k.vy, sc.dt, x.y), nz = fmaf(k.vz, sc.dt, x.z);
    k.fin = isfinite(k.vx) && isfinite(k.vy) && isfinite(k.vz) && isfinite(nx) && isfinite(ny) && isfinite(nz);
    if (!k.fin) {
        nx = x.x;
        ny = x.y;
        nz = x.z;
    }
    k.esc = fabsf(nx - x.x) >= 1.0f || fabsf(ny - x.y) >= 1.0f || fabsf(nz - x.z) >= 1.0f;
    nx = rintf(nx * sc.inv_q) * sc.q;
    ny = rintf(ny * sc.inv_q) * sc.q;
    nz = rintf(nz * sc.inv_q) * sc.q;
    if (nx >= sc.L[0]) nx -= sc.L[0]; else if (nx < 0.0f) nx += sc.L[0];
    if (ny >= sc.L[1]) ny -= sc.L[1]; else if (ny < 0.0f) ny += sc.L[1];
    if (nz >= sc.L[2]) nz -= sc.L[2]; else if (nz < 0.0f) nz += sc.L[2];
    if (!(nx >= 0.0f && nx < sc.L[0] && ny >= 0.0f && ny < sc.L[1] && nz >= 0.0f && nz < sc.L[2])) {
        k.esc = true;
        nx = fminf(fmaxf(nx, 0.0f), sc.L[0] - sc.q);
        ny = fminf(fmaxf(ny, 0.0f), sc.L[1] - sc.q);
        nz = fminf(fmaxf(nz, 0.0f), sc.L[2] - sc.q);
    }
    k.nx = nx;
    k.ny = ny;
    k.nz = nz;
    return k;
}

constexpr int kBounceIters = 24;        // bisection steps of the bounce-back: t to 2^-24 of the drift

// Kick and drift of one particle of a box with walls (Sec. 3.1, time-stepping
// step 5, with the walls' conditions): a frozen wall particle keeps its place
// and velocity, or turns rigidly with its cylinder and takes the wall
// velocity there; a fluid particle whose drift ends inside a wall goes back
// to the last point of its drift on the fluid side (bisection on the
// position grid) with its velocity reversed in the wall's frame.  Shared by
// the integrate kernel and the force kernel's fused write-out, so both
// compute the same bits.
__device__ __forceinline__ Kicked kick_drift_walls(float4 x, float4 v, float4 f, bool live, bool frozen,
                                                   const StepConst& sc)
{
    Kicked k;
    k.vcx = fmaf(f.x, sc.half_dtm, v.x);
    k.vcy = fmaf(f.y, sc.half_dtm, v.y);
    k.vcz = fmaf(f.z, sc.half_dtm, v.z);
    float vx = fmaf(f.x, sc.dtm, v.x), vy = fmaf(f.y, sc.dtm, v.y), vz = fmaf(f.z, sc.dtm, v.z);
    if (frozen) { vx = v.x; vy = v.y; vz = v.z; }
    float nx = frozen ? x.x : fmaf(vx, sc.dt, x.x), ny = frozen ? x.y : fmaf(vy, sc.dt, x.y),
          nz = frozen ? x.z : fmaf(vz, sc.dt, x.z);
    bool turned = false;
    if (frozen && sc.wall_kind == 3) {
        // a turning cylinder turns its frozen layer rigidly by omega dt
        // about the axis (the particle takes the wall velocity at its
        // new, grid-rounded position below)
        float c1, c2;
        const int cyl = cylinder_of(x.x, x.y, x.z, sc, c1, c2);
        if (sc.omega[cyl] != 0.0f) {
            const float cs = sc.rot[cyl][0], sn = sc.rot[cyl][1];
            const float3 dd = from_axes(sc, fmaf(cs, c1, -sn * c2) - c1, fmaf(sn, c1, cs * c2) - c2);
            nx = x.x + dd.x;
            ny = x.y + dd.y;
            nz = x.z + dd.z;
            turned = true;
        }
    }
    k.fin = isfinite(vx) && isfinite(vy) && isfinite(vz) && isfinite(nx) && isfinite(ny) && isfinite(nz);
    if (!k.fin) {
        nx = x.x; ny = x.y; nz = x.z;
    }
    k.esc = fabsf(nx - x.x) >= 1.0f || fabsf(ny - x.y) >= 1.0f || fabsf(nz - x.z) >= 1.0f;
    nx = rintf(nx * sc.inv_q) * sc.q;
    ny = rintf(ny * sc.inv_q) * sc.q;
    nz = rintf(nz * sc.inv_q) * sc.q;
    if (turned) {               // the same velocity dpd_set_frozen gives a particle there
        const float3 u = wall_velocity(nx, ny, nz, sc);
        vx = u.x; vy = u.y; vz = u.z;
    }
    if (sc.wall_kind != 0 && live && !frozen && k.fin && wall_sdf(nx, ny, nz, sc) > 0.0f) {
        // bounce-back: bisection for the sdf's zero along the drift, every
        // probe on the position grid; the particle goes to the last probe
        // on the fluid side (the start, t = 0, if none) and its velocity is
        // reversed in the frame of the wall: v -> 2 u_wall - v
        const float dx = nx - x.x, dy = ny - x.y, dz = nz - x.z;
        float lo = 0.0f, hi = 1.0f;
        for (int it = 0; it < kBounceIters; ++it) {
            const float mid = 0.5f * (lo + hi);
            const bool in = wall_sdf(rintf(fmaf(mid, dx, x.x) * sc.inv_q) * sc.q,
                                     rintf(fmaf(mid, dy, x.y) * sc.inv_q) * sc.q,
                                     rintf(fmaf(mid, dz, x.z) * sc.inv_q) * sc.q, sc) > 0.0f;
            lo = in ? lo : mid;
            hi = in ? mid : hi;
        }
        nx = rintf(fmaf(lo, dx, x.x) * sc.inv_q) * sc.q;
        ny = rintf(fmaf(lo, dy, x.y) * sc.inv_q) * sc.q;
        nz = rintf(fmaf(lo, dz, x.z) * sc.inv_q) * sc.q;
        const float3 u = wall_velocity(nx, ny, nz, sc);           // reversal in the wall's frame
        vx = fmaf(2.0f, u.x, -vx); vy = fmaf(2.0f, u.y, -vy); vz = fmaf(2.0f, u.z, -vz);
    }
    if (nx >= sc.L[0]) nx -= sc.L[0]; else if (nx < 0.0f) nx += sc.L[0];
    if (ny >= sc.L[1]) ny -= sc.L[1]; else if (ny < 0.0f) ny += sc.L[1];
    if (nz >= sc.L[2]) nz -= sc.L[2]; else if (nz < 0.0f) nz += sc.L[2];
    if (!(nx >= 0.0f && nx < sc.L[0] && ny >= 0.0f && ny < sc.L[1] && nz >= 0.0f && nz < sc.L[2])) {
        k.esc = true;
        nx = fminf(fmaxf(nx, 0.0f), sc.L[0] - sc.q);
        ny = fminf(fmaxf(ny, 0.0f), sc.L[1] - sc.q);
        nz = fminf(fmaxf(nz, 0.0f), sc.L[2] - sc.q);
    }
    k.nx = nx; k.ny = ny; k.nz = nz;
    k.vx = vx; k.vy = vy; k.vz = vz;
    return k;
}

// FP64 sums of one moved particle into m[kPartials]: momentum and kinetic
// energy of v^{n+1/2}, kinetic energy of the time-centred velocity.
__device__ __forceinline__ void add_partials(double* m, const Kicked& k)
{
    m[0] += (double)k.vx;
    m[1] += (double)k.vy;
    m[2] += (double)k.vz;
    m[3] += (double)k.vx * k.vx + (double)k.vy * k.vy + (double)k.vz * k.vz;
    m[4] += (double)k.vcx * k.vcx + (double)k.vcy * k.vcy + (double)k.vcz * k.vcz;
}

// Flow-profile slab of a particle at x^n (grad_axis coordinate) and its
// fixed-point time-centred flow velocity.
__device__ __forceinline__ int profile_bin(float4 x, const StepConst& sc)
{
    const float g = sc.grad_axis == 0 ? x.x : (sc.grad_axis == 1 ? x.y : x.z);
    int b = (int)(g * sc.grad_scale);
    return b < 0 ? 0 : (b > sc.nbins - 1 ? sc.nbins - 1 : b);
}

// (the components come as separate values: a runtime pick from a struct
// would be compiled as an indexed load from a stack copy of it)
__device__ __forceinline__ long long profile_units(float vcx, float vcy, float vcz, const StepConst& sc)
{
    const float vflow = sc.flow_axis == 0 ? vcx : (sc.flow_axis == 1 ? vcy : vcz);
    return llrint((double)vflow * kProfScale);
}

// Box of workgroup `b` of a launch group (exclusive prefix pre[0..nbox]).
__device__ __forceinline__ int find_box(const int* __restrict__ pre, int nbox, int b)
{
    int lo = 0, hi = nbox;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace dpd
