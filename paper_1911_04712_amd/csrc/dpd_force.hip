// dpd_force.hip -- DPD pair forces on gfx950 (Sec. 2.1, Eqs. 2-5 of the
// Mirheo paper; periodic-Poiseuille body force of Sec. 4.2, Eq. 11).
//
// Two kernels compute the same bits:
//
//  k_force_gather  one thread per particle sums over all 27 neighbour cells
//                  straight from HBM (each pair evaluated from both sides).
//                  It is the reference kernel and the fallback for tiles
//                  whose particles do not fit the LDS buffers.
//
//  k_force_tiled   one workgroup per tile of cells.  The tile and its
//                  one-cell halo are staged in LDS (rows of cells are
//                  contiguous in cell order, so each row is a contiguous copy,
//                  with the periodic image shift applied on the way in).  Each
//                  tile particle walks the half stencil: forward neighbour
//                  cells, later particles of its own cell, and backward cells
//                  that lie in the halo.  Home units (one or two cells of a
//                  tile row) go to the waves from an LDS counter as the waves
//                  free up.  Candidates with r < r_c are compacted into a
//                  per-wave queue (ballot + popcount) and evaluated 64 at a
//                  time with every lane busy.  Both halves
//                  of a pair inside the tile are accumulated (F_ij to i,
//                  -F_ij to j); a pair that crosses the tile boundary is
//                  evaluated once from each side and only the tile particle is
//                  updated, so every force is written exactly once.
//
// Bitwise agreement of the two kernels follows from the rules in
// dpd_device.hpp: exact displacements, exactly antisymmetric pair forces and
// order-independent fixed-point sums.
#include <climits>
#include <cmath>

#include "dpd_internal.hpp"

namespace dpd {

// Load through the global address space (see gmem).
__device__ __forceinline__ float4 gload4(const float4* p, int i)
{
    typedef float __attribute__((ext_vector_type(4))) v4;
    const v4 t = ((const DPD_GLOBAL v4*)p)[i];
    return make_float4(t.x, t.y, t.z, t.w);
}

__device__ __forceinline__ int wrap_cell(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

__device__ __forceinline__ float body_force_of(float4 p, const ForceConst& fc)
{
    if (fc.body_uniform) return fc.body_f;
    const float g = fc.grad_axis == 0 ? p.x : (fc.grad_axis == 1 ? p.y : p.z);
    return g <= fc.half_grad ? -fc.body_f : fc.body_f;
}

__device__ __forceinline__ float4 finish_force(long long ax, long long ay, long long az, float4 p, const ForceConst& fc)
{
    double f[3] = {(double)ax * kFxInv, (double)ay * kFxInv, (double)az * kFxInv};
    if (fc.body_f != 0.0f) f[fc.flow_axis] += (double)body_force_of(p, fc);
    return make_float4((float)f[0], (float)f[1], (float)f[2], 0.0f);
}

// Pair (i, j) given both particles' (image-shifted) positions and
// velocities: adds the fixed-point force on i to a[0..2].  Returns false if
// the force is outside the fixed-point range (reported as non-finite).
// kCut: the pair has its own cutoff r_c <= 1; the displacement is measured
// in units of it (inv_rc = 1 / r_c: w = 1 - r / r_c, and the direction and
// the velocity projection do not change), and pairs beyond it add nothing.
// The negated displacement scales to the negated value, so F_ji = -F_ij
// still holds bit for bit; inv_rc = 1 leaves every bit as it is.
template <bool kCut = false>
__device__ __forceinline__ bool pair_fx(float4 pi, float4 vi, float4 pj, float4 vj, uint32_t step, const PairConst& pc,
                                        long long& fx, long long& fy, long long& fz, float inv_rc = 1.0f)
{
    float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    if constexpr (kCut) {
        dx *= inv_rc;
        dy *= inv_rc;
        dz *= inv_rc;
    }
    const float r2 = dist2(dx, dy, dz);
    const float xi = pair_xi(__float_as_uint(pi.w), __float_as_uint(pj.w), step, pc.k0, pc.k1);
    float rinv;
    const float fs = pair_scalar(r2, dx, dy, dz, vi.x - vj.x, vi.y - vj.y, vi.z - vj.z, rinv, xi, pc);
    // coincident particles exert no force on each other; with a pair cutoff
    // the candidate test (r < 1) lets through pairs beyond it
    const bool live = r2 > 0.0f && (!kCut || r2 < 1.0f);
    // the scalar force in fixed-point units (a power-of-two scale: each
    // component below is 2^31 times its FP32 value F = fs (d / r), bit for
    // bit).  |e| <= 1 up to an ulp, so |fs| < 2^19 keeps every component
    // inside the conversion's range; beyond it (or NaN) the pair adds
    // nothing and is reported (selects, not a branch)
    const float g = fs * kFxScale;
    const bool ok = !live || fabsf(g) < kFxLimit * kFxScale;
    const float gs = (live && ok) ? g : 0.0f;
    const float ri = live ? rinv : 0.0f;
    fx = fx_of_units(gs * (dx * ri));
    fy = fx_of_units(gs * (dy * ri));
    fz = fx_of_units(gs * (dz * ri));
    return ok;
}

// Force on particle i (cell order) by gathering over its 27 neighbour cells;
// kSp: each pair takes its species pair's entry of the table.
template <bool kSp>
__device__ float4 gather_force_one(int i, const float4* __restrict__ pos, const float4* __restrict__ vel,
                                   const int* __restrict__ cell_start, const ForceConst& fc, uint32_t step, bool& bad)
{
    const float4 pi = pos[i], vi = vel[i];
    const int Lx = fc.cells[0], Ly = fc.cells[1], Lz = fc.cells[2];
    const int cx = cell_coord(pi.x, Lx), cy = cell_coord(pi.y, Ly), cz = cell_coord(pi.z, Lz);
    long long ax = 0, ay = 0, az = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        int nz = cz + dz;
        float sz = 0.0f;
        if (nz < 0) { nz += Lz; sz = -fc.L[2]; } else if (nz >= Lz) { nz -= Lz; sz = fc.L[2]; }
        for (int dy = -1; dy <= 1; ++dy) {
            int ny = cy + dy;
            float sy = 0.0f;
            if (ny < 0) { ny += Ly; sy = -fc.L[1]; } else if (ny >= Ly) { ny -= Ly; sy = fc.L[1]; }
            for (int dx = -1; dx <= 1; ++dx) {
                int nx = cx + dx;
                float sx = 0.0f;
                if (nx < 0) { nx += Lx; sx = -fc.L[0]; } else if (nx >= Lx) { nx -= Lx; sx = fc.L[0]; }
                const int cell = nx + Lx * (ny + Ly * nz);
                const int s = cell_start[cell], e = cell_start[cell + 1];
                for (int j = s; j < e; ++j) {
                    if (j == i) continue;
                    float4 pj = pos[j];
                    pj.x += sx;
                    pj.y += sy;
                    pj.z += sz;
                    const float r2 = dist2(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z);
                    if (!(r2 < 1.0f) || r2 == 0.0f) continue;
                    long long fx, fy, fz;
                    const float4 vj = vel[j];
                    if constexpr (kSp) {
                        PairConst pc = fc.pc;
                        const float4 c = fc.tab[species_pair(__float_as_int(vi.w), __float_as_int(vj.w))];
                        pc.a = c.x;
                        pc.gamma = c.y;
                        pc.sig_rdt = c.z;
                        bad |= !pair_fx<true>(pi, vi, pj, vj, step, pc, fx, fy, fz, c.w);
                    } else {
                        bad |= !pair_fx(pi, vi, pj, vj, step, fc.pc, fx, fy, fz);
                    }
                    ax += fx;
                    ay += fy;
                    az += fz;
                }
            }
        }
    }
    return finish_force(ax, ay, az, pi, fc);
}

__global__ __launch_bounds__(kBlock) void k_force_gather(const BoxDesc* __restrict__ desc,
                                                         const int* __restrict__ pre, int nbox)
{
    const int* __restrict__ pre_ = pre + kWPart * (nbox + 1);
    const int box = nbox == 1 ? 0 : find_box(pre_, nbox, (int)blockIdx.x);
    const BoxDesc& d = desc[box];
    const int i = ((int)blockIdx.x - pre_[box]) * kBlock + threadIdx.x;
    if (i >= d.n) return;
    bool bad = false;
    const uint32_t step = (uint32_t)d.st->step;
    d.force[i] = d.fc.ntypes > 1 ? gather_force_one<true>(i, d.pos_b, d.vel_b, d.cell_start, d.fc, step, bad)
                                 : gather_force_one<false>(i, d.pos_b, d.vel_b, d.cell_start, d.fc, step, bad);
    if (bad) gatomic_or(&d.st->nonfinite, 1);
}

// ---------------------------------------------------------------------------
// tiled kernel
// ---------------------------------------------------------------------------
constexpr int kQueueLive = 192; // per-wave hit queue: < 64 pending + up to 2 x 64 new; after the
                                // waves' queues, 64 slots that lanes without a hit write to (shared
                                // by all waves: nothing reads them)
constexpr int kUnitSlots = 16;  // run-table entries per home unit (14 runs, own_e, the list length)

// Inclusive prefix sum inside each row of 16 lanes (DPP row shifts).
__device__ __forceinline__ int row16_incl_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    return v;
}

__device__ __forceinline__ int lane_val(int v, int src_lane) { return __builtin_amdgcn_ds_bpermute(src_lane << 2, v); }

// floor(x / d) for 0 <= x < 2^22, d >= 1, with inv = 1.0f / d rounded to
// nearest: (x + 0.5) / d lies at least 0.5 / d from an integer, and the
// float product (x + 0.5) * inv is within about x 2^-23 / d of it.
__device__ __forceinline__ int small_div(int x, float inv)
{
    return (int)(((float)x + 0.5f) * inv);
}

// 64-bit value moved by a DPP row operation (both halves with the same
// control); lanes whose source lies outside their row of 16 get 0.
template <int kCtrl>
__device__ __forceinline__ long long dpp_i64(long long v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), kCtrl, 0xf, 0xf, true);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Levels of the home-side pre-combine in a flush (0: every lane adds its own
// pair force to its home particle).  The hits of one home particle sit
// together in the queue, so a flush's lanes target a few home accumulators
// many times over, and LDS atomics to one address serialise.  Level k adds,
// inside aligned groups of 2^levels lanes, the partial sum of the lanes
// 2^(k-1) below when no run of another home starts in between (a segmented
// scan by DPP row shifts); then only the last lane of each run of one home
// inside a group adds the run's sum.  Integer sums: the bits do not change.
#ifndef DPD_HOME_COMBINE
#define DPD_HOME_COMBINE 3
#endif
constexpr int kHomeCombine = DPD_HOME_COMBINE;
static_assert(kHomeCombine >= 0 && kHomeCombine <= 4, "groups of at most one DPP row (16 lanes)");

// Lanes that open a group of 2^levels lanes, as a wave mask.
constexpr unsigned long long group_first_lanes(int levels)
{
    unsigned long long m = 0;
    for (int l = 0; l < 64; l += 1 << levels) m |= 1ull << l;
    return m;
}

// One level of the segmented scan at distance kDist (DPP row_shr:kDist):
// a lane whose run started more than kDist lanes back adds the partial sums
// kDist lanes below.  The run heads are a wave mask (bit l for lane l); after
// the level a lane's bit says "a run starts within the last 2 kDist lanes",
// which is its bit or the bit kDist lanes below (a lane whose source lies in
// the row of 16 below counts as a head: rows are never crossed).  The mask
// arithmetic runs on the scalar unit.
template <int kDist>
__device__ __forceinline__ void combine_level(long long& hx, long long& hy, long long& hz, unsigned long long& heads)
{
    constexpr int ctrl = 0x110 + kDist;                      // row_shr:kDist
    constexpr unsigned long long kRowLow = ((1ull << kDist) - 1ull) * 0x0001000100010001ull;   // l % 16 < kDist
    const long long tx = dpp_i64<ctrl>(hx), ty = dpp_i64<ctrl>(hy), tz = dpp_i64<ctrl>(hz);
    const bool add = !__builtin_amdgcn_inverse_ballot_w64(heads);
    hx += add ? tx : 0ll;
    hy += add ? ty : 0ll;
    hz += add ? tz : 0ll;
    heads |= ((heads << kDist) & ~kRowLow) | kRowLow;
}

// Staged velocity .w: the tile index (-1 outside the tile); with species
// (kSp) its low 24 bits hold the tile index and the top 8 bits the species.
// Every lane of the wave calls it; `live` marks the lanes that hold a queue
// entry (the others take entry 0, a coincident pair that adds nothing, and
// skip the atomics).
template <bool kSp>
__device__ __forceinline__ void flush_hit(unsigned e, bool live, const float4* sp, const float4* sv, long long* acc,
                                          uint32_t step, const PairConst& pc, const float4* tab, bool& bad)
{
    if (!live) e = 0u;
    const int a = (int)(e >> 16), b = (int)(e & 0xffffu);
    const float4 va = sv[a], vb = sv[b];
    long long fx, fy, fz;
    const int wa = __float_as_int(va.w), wb = __float_as_int(vb.w);
    int ia, ib;
    if constexpr (kSp) {
        PairConst q = pc;
        const float4 c = tab[species_pair((int)((unsigned)wa >> 24), (int)((unsigned)wb >> 24))];
        q.a = c.x;
        q.gamma = c.y;
        q.sig_rdt = c.z;
        bad |= !pair_fx<true>(sp[a], va, sp[b], vb, step, q, fx, fy, fz, c.w);
        ia = wa & 0xffffff;
        ib = (wb << 8) >> 8;
    } else {
        bad |= !pair_fx(sp[a], va, sp[b], vb, step, pc, fx, fy, fz);
        ia = wa;
        ib = wb;
    }
    long long hx = fx, hy = fy, hz = fz;
    bool home_add = live;
    if constexpr (kHomeCombine > 0) {
        constexpr int last = (1 << kHomeCombine) - 1;        // lanes per group - 1
        const int g = (int)(threadIdx.x & 63) & last;
        const int key = live ? ia : -1 - (int)(threadIdx.x & 63);   // dead lanes never match
        const int kp1 = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x111, 0xf, 0xf, false);   // row_shr:1
        const int kn1 = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x101, 0xf, 0xf, false);   // row_shl:1
        // a run of one home starts here: a group's first lane, or a new key
        unsigned long long heads = __builtin_amdgcn_ballot_w64(kp1 != key) | group_first_lanes(kHomeCombine);
        combine_level<1>(hx, hy, hz, heads);
        if constexpr (kHomeCombine > 1) combine_level<2>(hx, hy, hz, heads);
        if constexpr (kHomeCombine > 2) combine_level<4>(hx, hy, hz, heads);
        if constexpr (kHomeCombine > 3) combine_level<8>(hx, hy, hz, heads);
        home_add = live && (g == last || kn1 != key);
    }
    if (home_add) {
        // tile indices are below 2^24: 24-bit multiplies for the LDS offsets
        unsigned long long* pa = (unsigned long long*)((char*)acc + __umul24((unsigned)ia, 24u));
        atomicAdd(pa, (unsigned long long)hx);
        atomicAdd(pa + 1, (unsigned long long)hy);
        atomicAdd(pa + 2, (unsigned long long)hz);
    }
    if (live && ib >= 0) {               // both ends in the tile: apply the reaction too (LDS subtract)
        unsigned long long* pb = (unsigned long long*)((char*)acc + __umul24((unsigned)ib, 24u));
        __hip_atomic_fetch_sub(pb, (unsigned long long)fx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_sub(pb + 1, (unsigned long long)fy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_sub(pb + 2, (unsigned long long)fz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

constexpr int kProfSlots = 64;  // flow-profile slabs one tile sums in LDS before its global atomics

// Write-out of tile t: each tile particle's total force, once, in cell
// order.  With kFuse (1; 2 for a launch with walls: frozen particles, the
// bounce-back, the velocity's .w read whole from the cell-ordered state) the
// particle's kick-drift follows at once (Sec. 3.1,
// time-stepping step 5, done here because the force is final): the next
// position and velocity go to pos_a / vel_a, its next cell and arrival slot
// to keyslot and the cell counters, and the tile's FP64 sums (fixed order:
// lanes, then waves) to its own entry of `partials`, which the fold adds
// up in tile order.  The nt tile particles are taken flat, thread k with
// particles k, k + threads, ..., so a tile of a few hundred particles is one
// pass of the whole workgroup with one round trip of the arrival atomics;
// the row of a particle comes from a binary search over the rows' tile
// starts.  src(rw, k, x, v, f) gives particle k of tile row rw: its position
// x^n, stored velocity (w = species) and force.  scr is LDS the kernel no
// longer uses (at least kProfSlots * 12 + waves * 40 bytes).  Every thread
// of the workgroup calls it.
template <int kFuse, int kThreads, typename Src>
__device__ __forceinline__ void write_tile(const BoxDesc& d, int t, const int4* rows, int nrows, int nt, int o_grad,
                                           unsigned char* scr, Src src)
{
    constexpr int nw = kThreads >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    long long* p_sum = (long long*)scr;
    int* p_cnt = (int*)(scr + kProfSlots * 8);
    double* s_red = (double*)(scr + kProfSlots * 12);
    const StepConst& sc = d.sc;
    const int nbins = kFuse != 0 ? sc.nbins : 0;
    const int blo = nbins > 0 ? max(0, min((int)((float)o_grad * sc.grad_scale), nbins - 1)) : 0;
    if (nbins > 0) {                                    // uniform; 0 without kFuse
        for (int k = tid; k < kProfSlots; k += kThreads) {
            p_sum[k] = 0;
            p_cnt[k] = 0;
        }
        __syncthreads();
    }
    int top = 1;                                        // binary search over the rows' tile starts
    while (top * 2 <= nrows) top *= 2;
    double m[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool bad = false, esc = false;
    for (int ti0 = wave * 64; ti0 < nt; ti0 += kThreads) {   // wave-uniform: every lane reaches the atomics
        const int ti = ti0 + lane;
        const bool live = ti < nt;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f), v = x, f = x;
        int g = 0, wfull = 0;
        if (live) {
            int r = 0;
            for (int st = top; st > 0; st >>= 1)
                if (r + st < nrows && rows[r + st].w <= ti) r += st;
            const int4 rw = rows[r];
            const int k = ti - rw.w;
            g = rw.z + k;
            src(rw, k, x, v, f);
            gstore(d.force + g, f);
            if constexpr (kFuse == 2) wfull = gmem(reinterpret_cast<const int*>(d.vel_b))[4 * g + 3];   // species | frozen
        }
        if constexpr (kFuse != 0) {
            const bool frozen = kFuse == 2 && (wfull & kFrozenBit) != 0;   // wall particles never move
            Kicked kk;
            if constexpr (kFuse == 2)
                kk = kick_drift_walls(x, v, f, live, frozen, sc);
            else
                kk = kick_drift(x, v, f, sc);
            bad |= !kk.fin;
            esc |= kk.esc;
            const int c = live ? cell_of(kk.nx, kk.ny, kk.nz, sc.cells[0], sc.cells[1], sc.cells[2]) : -1;
            const ArrivalTicket tk = arrival_issue(c, live, d.count);   // atomic in flight meanwhile
            chunk_add(c, live, d.bsum);
            if (live) {
                gstore(d.pos_a + g, make_float4(kk.nx, kk.ny, kk.nz, x.w));
                gstore(d.vel_a + g, make_float4(kk.vx, kk.vy, kk.vz, kFuse == 2 ? __int_as_float(wfull) : v.w));
            }
            if (live && kk.fin && !frozen) {
                add_partials(m, kk);
                if (nbins > 0) {
                    const int b = profile_bin(x, sc);
                    const long long q = profile_units(kk.vcx, kk.vcy, kk.vcz, sc);
                    const int sl = b - blo;
                    if (sl >= 0 && sl < kProfSlots) {
                        atomicAdd((unsigned long long*)&p_sum[sl], (unsigned long long)q);
                        atomicAdd(&p_cnt[sl], 1);
                    } else {
                        gatomic_add((unsigned long long*)&d.profile[2 * b], (unsigned long long)q);
                        gatomic_add((unsigned long long*)&d.profile[2 * b + 1], 1ull);
                    }
                }
            }
            const int slot = arrival_finish(tk, live);
            if (live) gstore(d.keyslot + g, make_int2(c, slot));
        }
    }
    if constexpr (kFuse != 0) {
        if (bad) gatomic_or(&d.st->nonfinite, 1);
        if (esc) gatomic_or(&d.st->escaped, 1);
        // only the waves that took particles hold sums: the others' are +0.0,
        // which leaves a sum started at +0.0 unchanged, so they are skipped
        const int nwl = min(nw, (nt + 63) >> 6);
        if (wave < nwl) {                               // wave-uniform
#pragma unroll
            for (int k = 0; k < kPartials; ++k) {
                const double w = wave_sum(m[k]);
                if (lane == 0) s_red[wave * kPartials + k] = w;
            }
        }
        __syncthreads();
        if (tid < kPartials) {
            double sum = 0.0;
            for (int w = 0; w < nwl; ++w) sum += s_red[w * kPartials + tid];
            gmem(d.partials)[(size_t)t * kPartials + tid] = sum;
        }
        if (nbins > 0)
            for (int k = tid; k < kProfSlots; k += kThreads)
                if (p_cnt[k]) {
                    gatomic_add((unsigned long long*)&d.profile[2 * (blo + k)], (unsigned long long)p_sum[k]);
                    gatomic_add((unsigned long long*)&d.profile[2 * (blo + k) + 1], (unsigned long long)p_cnt[k]);
                }
        if (t == 0 && tid == 0) {      // the fold adds up one partial per tile
            gmem(&d.st->fold_count)[0] = (unsigned)d.tc.ntiles;
            gmem(&d.st->fold_pending)[0] = 1;
        }
    }
}

// 1024-thread workgroups: at most 64 VGPRs, so that two fit a CU (8 waves
// per SIMD); the smaller ones fit their LDS-bound count of workgroups anyway
template <bool kSp, int kThreads, int kFuse>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kThreads == 1024 ? 8 : 1))) void k_force_tiled(const BoxDesc* __restrict__ desc,
                                                             const int* __restrict__ pre, int nbox)
{
    const int* __restrict__ pre_ = pre + kWTile * (nbox + 1);
    const int box = nbox == 1 ? 0 : find_box(pre_, nbox, (int)blockIdx.x);
    const BoxDesc& d = desc[box];
    const ForceConst& fc = d.fc;
    const TileConst& tc = d.tc;
    const float4* __restrict__ pos = d.pos_b;
    const float4* __restrict__ vel = d.vel_b;
    const int* __restrict__ cell_start = d.cell_start;
    float4* __restrict__ force = d.force;
    int* __restrict__ nonfinite = &d.st->nonfinite;
    // constants the loops use, read once: after an LDS or global atomic the
    // compiler would otherwise fetch them from the descriptor again
    const PairConst pc = fc.pc;
    const float Lf0 = fc.L[0], Lf1 = fc.L[1], Lf2 = fc.L[2];
    const int ux = tc.ux;
    extern __shared__ __align__(16) unsigned char lds[];
    float4* sp = (float4*)lds;                                  // staged positions (image-shifted), w = id
    float4* sv = (float4*)(lds + tc.off_sv);                    // staged velocities, w = tile index or -1 (+ species)
    long long* acc = (long long*)(lds + tc.off_acc);            // fixed-point force of tile particles
    int* cst = (int*)(lds + tc.off_cst);                        // staged cell offsets in LDS (ncs + 1)
    int* cg = (int*)(lds + tc.off_cg);                          // staged cell start in HBM (cell order)
    int4* rows = (int4*)(lds + tc.off_rows);                    // tile rows: (lds start, len, HBM start, tile start)
    unsigned* qall = (unsigned*)(lds + tc.off_q);               // per-wave hit queues
    unsigned* utab = (unsigned*)(lds + tc.off_ut);              // run table of every home unit
    __shared__ int s_scr[kThreads / 64];
    __shared__ int s_unit;                                      // next home unit to hand out
    const float4* tab = nullptr;                                // species pair table (kSp)
    if constexpr (kSp) {
        __shared__ float4 s_tab[kMaxTypes * kMaxTypes];
        for (int k = threadIdx.x; k < kMaxTypes * kMaxTypes; k += kThreads) s_tab[k] = fc.tab[k];
        tab = s_tab;                                            // visible after the first barrier below
    }

    // Consecutive tiles go to the same XCD (workgroups are dealt to the 8
    // XCDs round-robin and every box's range starts at a multiple of 8), so
    // neighbouring tiles share halo cells in one L2.
    const int lb = (int)blockIdx.x - pre_[box];
    const int per_xcd = (pre_[box + 1] - pre_[box]) >> 3;
    const int t = (lb & 7) * per_xcd + (lb >> 3);
    if (t >= tc.ntiles) return;
    const int L0 = fc.cells[0], L1 = fc.cells[1], L2 = fc.cells[2];
    const int tx = t % tc.ntile[0], ty = (t / tc.ntile[0]) % tc.ntile[1], tz = t / (tc.ntile[0] * tc.ntile[1]);
    const int o0 = tx * tc.T[0], o1 = ty * tc.T[1], o2 = tz * tc.T[2];
    const int P0 = min(tc.T[0], L0 - o0), P1 = min(tc.T[1], L1 - o1), P2 = min(tc.T[2], L2 - o2);
    const int S0 = P0 + 2, S1 = P1 + 2, S2 = P2 + 2;
    const int ncs = S0 * S1 * S2;
    const int tid = threadIdx.x, lane = tid & 63, nw = kThreads >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float inv_s0 = 1.0f / (float)S0, inv_s1 = 1.0f / (float)S1, inv_p1 = 1.0f / (float)P1;
    const uint32_t step = (uint32_t)d.st->step;

    // 1. HBM start and particle count of every staged cell (the only
    //    dependent HBM round trip before the copy), scanned into LDS offsets
    for (int lc = tid; lc < ncs; lc += kThreads) {
        const int rr = small_div(lc, inv_s0);                  // staged row
        const int lz = small_div(rr, inv_s1), ly = rr - lz * S1, lx = lc - rr * S0;
        const int g = wrap_cell(o0 - 1 + lx, L0) + L0 * (wrap_cell(o1 - 1 + ly, L1) + L1 * wrap_cell(o2 - 1 + lz, L2));
        const int gs = gmem(cell_start)[g];
        cg[lc] = gs;
        cst[lc] = gmem(cell_start)[g + 1] - gs;
    }
    __syncthreads();
    const int S = block_excl_scan(cst, ncs, s_scr);

    // 2. tile rows (cells lx = 1..P0 of a row are contiguous in LDS and in HBM)
    const int nrows = P1 * P2;
    if (wave == 0) {
        int carry = 0;
        for (int r0 = 0; r0 < nrows; r0 += 64) {
            const int r = r0 + lane;
            int len = 0, ls = 0, gs = 0;
            if (r < nrows) {
                const int qz = small_div(r, inv_p1);
                const int ly = 1 + r - qz * P1, lz = 1 + qz;
                const int lc1 = 1 + S0 * (ly + S1 * lz);
                ls = cst[lc1];
                len = cst[lc1 + P0] - ls;
                gs = cg[lc1];
            }
            const int incl = wave_incl_scan(len);
            if (r < nrows) rows[r] = make_int4(ls, len, gs, carry + incl - len);
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) s_scr[0] = carry;
    }
    __syncthreads();
    const int nt = s_scr[0];

    const int o_grad = fc.grad_axis == 0 ? o0 : (fc.grad_axis == 1 ? o1 : o2);   // tile origin along the profile axis
    unsigned char* scr = lds + tc.off_q;                // the queues' LDS, free again at write-out

    if (S > tc.smax || nt > tc.pmax || (d.flags & kFlagReference)) {
        // Overfull tile (or the box asks for the reference path): gather
        // from HBM, same arithmetic and same bits.
        bool bad = false;
        for (int r = wave; r < nrows; r += nw) {
            const int4 rw = rows[r];
            for (int k = lane; k < rw.y; k += 64)
                gstore(force + rw.z + k, gather_force_one<kSp>(rw.z + k, pos, vel, cell_start, fc, step, bad));
        }
        if (bad) gatomic_or(nonfinite, 1);
        // the write-out takes the particles in another order: the barrier
        // makes every force written above visible to the whole workgroup
        __syncthreads();
        if constexpr (kFuse != 0)
            write_tile<kFuse, kThreads>(d, t, rows, nrows, nt, o_grad, scr,
                                        [&](const int4& rw, int k, float4& x, float4& v, float4& f) {
                                            const int g = rw.z + k;
                                            x = pos[g];
                                            v = vel[g];
                                            f = force[g];
                                        });
        return;
    }

    // 3. stage the region, one staged particle per thread.  A staged row
    //    (S0 cells) is at most three runs contiguous in HBM: cell lx = 0,
    //    cells 1..S0-2 and cell S0-1; only the end cells can wrap, and they
    //    take the periodic image shift on the way in.  Each thread finds its
    //    row by binary search over the row starts, so all loads of a pass
    //    are in flight together.
    {
        const int nsrows = S1 * S2;
        int top = 1;
        while (top * 2 <= nsrows) top *= 2;
        const float shx_lo = o0 == 0 ? -Lf0 : 0.0f, shx_hi = o0 + P0 == L0 ? Lf0 : 0.0f;
        for (int s0 = tid; s0 < S; s0 += 2 * kThreads) {
            int src[2], tiv[2];
            float shx[2], shy[2], shz[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int s = min(s0 + u * kThreads, S - 1);
                int r = 0;
                for (int st = top; st > 0; st >>= 1)
                    if (r + st < nsrows && cst[(r + st) * S0] <= s) r += st;
                const int c0 = r * S0;
                const int lz = small_div(r, inv_s1), ly = r - lz * S1;
                const int b1 = cst[c0 + 1], b2 = cst[c0 + S0 - 1];
                const int seg = s < b1 ? 0 : (s < b2 ? 1 : 2);
                const int cs = seg == 0 ? c0 : (seg == 1 ? c0 + 1 : c0 + S0 - 1);
                src[u] = cg[cs] + (s - cst[cs]);
                shx[u] = seg == 0 ? shx_lo : (seg == 2 ? shx_hi : 0.0f);
                const int gy = o1 - 1 + ly, gz = o2 - 1 + lz;
                shy[u] = gy < 0 ? -Lf1 : (gy >= L1 ? Lf1 : 0.0f);
                shz[u] = gz < 0 ? -Lf2 : (gz >= L2 ? Lf2 : 0.0f);
                const bool tile_row = ly >= 1 && ly <= P1 && lz >= 1 && lz <= P2;
                tiv[u] = (tile_row && seg == 1) ? rows[(ly - 1) + P1 * (lz - 1)].w + (s - b1) : -1;
            }
            const float4 p0 = gload4(pos, src[0]), v0 = gload4(vel, src[0]);
            const float4 p1 = gload4(pos, src[1]), v1 = gload4(vel, src[1]);
            sp[s0] = make_float4(p0.x + shx[0], p0.y + shy[0], p0.z + shz[0], p0.w);
            if constexpr (kSp) {
                tiv[0] = (tiv[0] & 0xffffff) | (int)((unsigned)__float_as_int(v0.w) << 24);   // species bits
                tiv[1] = (tiv[1] & 0xffffff) | (int)((unsigned)__float_as_int(v1.w) << 24);
            }
            sv[s0] = make_float4(v0.x, v0.y, v0.z, __int_as_float(tiv[0]));
            const int s1 = s0 + kThreads;
            if (s1 < S) {
                sp[s1] = make_float4(p1.x + shx[1], p1.y + shy[1], p1.z + shz[1], p1.w);
                sv[s1] = make_float4(v1.x, v1.y, v1.z, __int_as_float(tiv[1]));
            }
        }
    }
    // 4a. the candidate list of every home unit (ux consecutive cells x ..
    //     x+w-1 of a tile row, w = ux or fewer at the row's end), sixteen
    //     lanes per unit with every lane busy: up to 14 runs of consecutive
    //     staged particles, one per slot,
    //       slot 0      the unit and cell x+w (so the unit comes first)
    //       slots 1-4   forward rows, cells x-1 .. x+w
    //       slots 5-8   backward rows (y-1, z), (y+1, z-1), (y, z-1),
    //                   (y-1, z-1): cells x-1 .. x+w when the row lies in the
    //                   halo, else cell x-1 when it is a halo cell
    //       slots 9-12  the same backward rows: cell x+w when it is a halo cell
    //       slot 13     cell x-1 of the own row when it is a halo cell
    //     Each entry holds the run's staged start (high 16 bits) and its
    //     position in the list (low 16 bits, an exclusive scan over the
    //     unit's sixteen lanes, which are one DPP row); slot 14 holds the
    //     end of the unit's own particles in place of a run start, and the
    //     position of slots 14 and 15 is the list length.  Staged indices
    //     are below smax <= 65535, so both halves fit.
    const int upr = (P0 + ux - 1) / ux;                 // units per tile row
    const int nunits = upr * nrows;
    {
        const int sl = lane & (kUnitSlots - 1);
        const int rj = (sl - 1) & 3;                    // stencil row of slots 1..12
        const int fdy = (rj == 0 || rj == 3) ? 1 : (rj == 1 ? -1 : 0), fdz = rj == 0 ? 0 : 1;
        const int rsgn = (sl == 0 || sl >= 13) ? 0 : (sl < 5 ? 1 : -1);
        const int roff = rsgn * S0 * (fdy + S1 * fdz);  // staged-cell offset of the slot's row
        const float inv_upr = 1.0f / (float)upr;
        // whole units per pass (kThreads is a multiple of 16): the scan's
        // row of sixteen lanes is all active or all idle
        for (int e = tid; e < kUnitSlots * nunits; e += kThreads) {
            const int un = e / kUnitSlots;
            const int row = small_div(un, inv_upr);     // row (y, z) of the unit, y fastest
            const int rz = small_div(row, inv_p1), ry = row - rz * P1;
            const int lx = 1 + (un - row * upr) * ux, ly = ry + 1, lz = rz + 1;
            const int w = min(ux, P0 + 1 - lx);         // cells in this unit
            const int cown = lx + S0 * (ly + S1 * lz);
            // which backward rows (slots 5-8, and 9-12) leave the tile
            const bool yl = ly == 1, yh = ly == P1, zl = lz == 1;
            const unsigned outB = ((unsigned)yl << 5) | ((unsigned)(yh || zl) << 6) | ((unsigned)zl << 7) |
                                  ((unsigned)(yl || zl) << 8);
            const bool xl = lx == 1, xh = lx + w - 1 == P0;
            const unsigned mLeft = xl ? ((0x1E0u & ~outB) | (1u << 13)) : 0u;
            const unsigned mRight = xh ? (0x1E00u & ~(outB << 4)) : 0u;
            const unsigned mOn = 0x1Fu | outB | mLeft | mRight;
            const bool left = (mLeft >> sl) & 1u, right = (mRight >> sl) & 1u, on = (mOn >> sl) & 1u;
            // run of this slot: cells x0..x1 relative to the unit's first cell
            const int x0 = right ? w : (sl == 0 ? 0 : -1);
            const int x1 = left ? -1 : w;
            const int rbase = cown + roff;
            const int rs = cst[rbase + x0];
            const int rl = on ? cst[rbase + x1 + 1] - rs : 0;
            const int rpre = row16_incl_scan(rl) - rl;
            const int start = sl == 14 ? cst[cown + w] : rs;
            utab[e] = ((unsigned)start << 16) | (unsigned)rpre;
        }
    }
    for (int k = tid; k < 3 * nt; k += kThreads) acc[k] = 0;
    if (tid == 0) s_unit = nw;                          // units 0 .. nw-1 start the waves
    __syncthreads();

    // 4b. candidates, one home unit per wave at a time.  All particles of a
    //    unit share one candidate list: the unit itself and its half stencil
    //    (cell x+w, rows (y+1, z) and (y-1..y+1, z+1) over x-1 .. x+w), plus
    //    the backward cells that lie in the halo (pairs that cross the tile
    //    boundary are evaluated from both tiles, each updating only its own
    //    particle), as laid out in the run table above.  Entries out of
    //    reach of a given particle fail the distance test.
    //    List entries are spread over the lanes, each home particle is tested
    //    against all of them, and hits with r < r_c are compacted into a
    //    per-wave queue (ballot + popcount) and evaluated 64 at a time with
    //    every lane busy.  A pair inside the tile adds F_ij to i and -F_ij to
    //    j.  Pairs inside the unit are taken once (b after a): the unit heads
    //    the list in cell order, so that is list position > index of a.
    unsigned* q = qall + wave * kQueueLive;             // queue, entries [0, qt); qt is wave-uniform
    int qt = 0;
    bool bad = false;
    // each wave takes the next unit when it is done with one (face rows
    // cost about twice an interior row, so a fixed deal of units to waves
    // leaves waves idle while the slowest finishes)
    auto next_unit = [&]() {
        int v = 0;
        if (lane == 0) v = atomicAdd(&s_unit, 1);
        return __builtin_amdgcn_readfirstlane(v);
    };
    for (int un = wave; un < nunits; un = next_unit()) {
        const unsigned ent = utab[un * kUnitSlots + (lane & (kUnitSlots - 1))];
        const int rs = (int)(ent >> 16), rpre = (int)(ent & 0xffffu);
        const int own_s = __builtin_amdgcn_readlane(rs, 0);
        const int own_e = __builtin_amdgcn_readlane(rs, 14);
        if (own_s == own_e) continue;
        const int M = __builtin_amdgcn_readlane(rpre, 15);
        const int delta = rs - rpre;                // staged index = list position + delta
        for (int u0 = 0; u0 < M; u0 += 64) {
            // a last stretch of at most 32 entries is tested by lane groups
            // of 8, 16 or 32 lanes, one home particle per group
            const int rem = M - u0;
            const int gbits = rem <= 8 ? 3 : (rem <= 16 ? 4 : (rem <= 32 ? 5 : 6));   // wave-uniform
            const int u = u0 + (lane & ((1 << gbits) - 1));
            int k = 0;
#pragma unroll
            for (int st = 8; st > 0; st >>= 1)
                if (lane_val(rpre, k + st) <= u) k += st;
            const int dk = lane_val(delta, k);      // every lane takes part: source lanes must be active
            const bool valid = u < M;
            const int b = valid ? u + dk : own_s;
            const float4 xb = sp[b];
            const float bx = valid ? xb.x : 1e30f;
            const unsigned ub = (unsigned)u;
            const unsigned qdummy = (unsigned)((nw - wave) * kQueueLive + lane);   // the shared slots
            // flush whole waves of hits once 64 or more are queued
            auto drain = [&]() {
                if (qt >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    int fh = 0;
                    do {
                        flush_hit<kSp>(q[fh + lane], true, sp, sv, acc, step, pc, tab, bad);
                        fh += 64;
                    } while (qt - fh >= 64);
                    const unsigned rest = q[fh + lane];          // move what is left (< 64) to the front
                    __builtin_amdgcn_wave_barrier();
                    q[lane] = rest;
                    __builtin_amdgcn_wave_barrier();
                    qt -= fh;
                }
            };
            if (gbits < 6) {
                const int g = lane >> gbits, G = 64 >> gbits;
                for (int a = own_s; a < own_e; a += G) {
                    const int ah = a + g;
                    const bool hv = ah < own_e;
                    const float4 xa = sp[hv ? ah : a];
                    const float r2 = dist2(xa.x - bx, xa.y - xb.y, xa.z - xb.z);
                    const unsigned long long m = __builtin_amdgcn_ballot_w64(r2 < 1.0f) &
                                                 __builtin_amdgcn_ballot_w64(hv && ub > (unsigned)(ah - own_s));
                    const unsigned sl = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m, (unsigned)qt));
                    q[__builtin_amdgcn_inverse_ballot_w64(m) ? sl : qdummy] = ((unsigned)ah << 16) | (unsigned)b;
                    qt += __popcll(m);
                    drain();
                }
                continue;
            }
            // home particles two at a time (the pair loop carries no odd-tail
            // logic), then the odd one
            int a = own_s;
            for (; a + 1 < own_e; a += 2) {
                const float4* pa = sp + a;          // same address on every lane
                const float4 xa0 = pa[0];
                const float4 xa1 = pa[1];
                const float r20 = dist2(xa0.x - bx, xa0.y - xb.y, xa0.z - xb.z);
                const float r21 = dist2(xa1.x - bx, xa1.y - xb.y, xa1.z - xb.z);
                // r2 < 1 (r2 == 0 adds nothing: see pair_fx), and list position
                // after a (the unit heads the list)
                const unsigned ia = (unsigned)(a - own_s);
                const unsigned long long m0 = __builtin_amdgcn_ballot_w64(r20 < 1.0f) &
                                              __builtin_amdgcn_ballot_w64(ub > ia);
                const unsigned long long m1 = __builtin_amdgcn_ballot_w64(r21 < 1.0f) &
                                              __builtin_amdgcn_ballot_w64(ub > ia + 1u);
                const int c0 = __popcll(m0);
                const unsigned s0 = __builtin_amdgcn_mbcnt_hi((unsigned)(m0 >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((unsigned)m0, (unsigned)qt));
                const unsigned s1 = __builtin_amdgcn_mbcnt_hi((unsigned)(m1 >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((unsigned)m1, (unsigned)(qt + c0)));
                q[__builtin_amdgcn_inverse_ballot_w64(m0) ? s0 : qdummy] = ((unsigned)a << 16) | (unsigned)b;
                q[__builtin_amdgcn_inverse_ballot_w64(m1) ? s1 : qdummy] = ((unsigned)(a + 1) << 16) | (unsigned)b;
                qt += c0 + __popcll(m1);
                drain();
            }
            if (a < own_e) {
                const float4 xa0 = sp[a];
                const float r20 = dist2(xa0.x - bx, xa0.y - xb.y, xa0.z - xb.z);
                const unsigned long long m0 = __builtin_amdgcn_ballot_w64(r20 < 1.0f) &
                                              __builtin_amdgcn_ballot_w64(ub > (unsigned)(a - own_s));
                const unsigned s0 = __builtin_amdgcn_mbcnt_hi((unsigned)(m0 >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((unsigned)m0, (unsigned)qt));
                q[__builtin_amdgcn_inverse_ballot_w64(m0) ? s0 : qdummy] = ((unsigned)a << 16) | (unsigned)b;
                qt += __popcll(m0);
                drain();
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (qt > 0) flush_hit<kSp>(q[lane], lane < qt, sp, sv, acc, step, pc, tab, bad);
    if (bad) gatomic_or(nonfinite, 1);
    __syncthreads();

    // 5. each tile particle's force is written once, in cell order (a tile
    //    particle is staged without an image shift, so sp holds x^n); with
    //    kFuse its kick-drift follows
    write_tile<kFuse, kThreads>(d, t, rows, nrows, nt, o_grad, scr,
                                [&](const int4& rw, int k, float4& x, float4& v, float4& f) {
                                    const int ti = rw.w + k;
                                    x = sp[rw.x + k];
                                    v = sv[rw.x + k];
                                    // the staged .w holds the tile index (and the species in
                                    // its top 8 bits with kSp); a launch without kSp has only
                                    // species-0 particles
                                    v.w = __int_as_float(kSp ? (int)((unsigned)__float_as_int(v.w) >> 24) : 0);
                                    f = finish_force(acc[3 * ti], acc[3 * ti + 1], acc[3 * ti + 2], x, fc);
                                });
}

TileConst make_tile_const(const int* cells, double rho, const int* tile, int threads, int smax_override,
                          int pmax_override)
{
    TileConst tc{};
    tc.threads = threads;
    for (int k = 0; k < 3; ++k) {
        tc.T[k] = tile[k] < cells[k] ? tile[k] : cells[k];
        tc.ntile[k] = (cells[k] + tc.T[k] - 1) / tc.T[k];
    }
    tc.ntiles = tc.ntile[0] * tc.ntile[1] * tc.ntile[2];
    const int ncs_max = (tc.T[0] + 2) * (tc.T[1] + 2) * (tc.T[2] + 2);
    const int ntc = tc.T[0] * tc.T[1] * tc.T[2];
    // capacities: mean + 6 standard deviations of a uniform fluid, rounded up
    auto cap = [](double mean) { int c = (int)std::ceil(mean + 6.0 * std::sqrt(mean + 1.0) + 16.0); return (c + 63) & ~63; };
    // two-cell home units keep a dilute fluid's candidate list near one wave
    // (about 19 rho entries, against 14 rho + 1 for a single cell)
    tc.ux = (rho <= 4.5 && tc.T[0] >= 2) ? 2 : 1;
    tc.smax = smax_override > 0 ? smax_override : cap(rho * ncs_max);
    tc.pmax = pmax_override > 0 ? pmax_override : cap(rho * ntc);
    if (tc.smax > 65535) tc.smax = 65535;
    size_t off = (size_t)tc.smax * 16;
    tc.off_sv = (int)off;
    off += (size_t)tc.smax * 16;
    tc.off_acc = (int)off;
    off += (size_t)tc.pmax * 24;
    tc.off_cst = (int)off;
    off += ((size_t)(ncs_max + 1) * 4 + 15) & ~(size_t)15;
    tc.off_cg = (int)off;
    off += ((size_t)ncs_max * 4 + 15) & ~(size_t)15;
    tc.off_rows = (int)off;
    off += (size_t)tc.T[1] * tc.T[2] * 16;
    tc.off_ut = (int)off;
    off += (size_t)((tc.T[0] + tc.ux - 1) / tc.ux) * tc.T[1] * tc.T[2] * kUnitSlots * 4;
    tc.off_q = (int)off;
    off += ((size_t)(threads / 64) * kQueueLive + 64) * 4;
    tc.lds_bytes = (int)off;
    return tc;
}

template <bool kSp, int kFuse>
static void launch_tiled(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    const dim3 grid(lp.total[kWTile]);
    switch (lp.force_threads) {
    case 256:
        launch_timed(k_force_tiled<kSp, 256, kFuse>, grid, dim3(256), lp.lds_force, s, t0, t1, lp.desc, lp.pre, lp.nbox);
        break;
    case 1024:
        launch_timed(k_force_tiled<kSp, 1024, kFuse>, grid, dim3(1024), lp.lds_force, s, t0, t1, lp.desc, lp.pre,
                     lp.nbox);
        break;
    default:
        launch_timed(k_force_tiled<kSp, 512, kFuse>, grid, dim3(512), lp.lds_force, s, t0, t1, lp.desc, lp.pre, lp.nbox);
        break;
    }
}

hipError_t launch_force(const LaunchPlan& lp, hipStream_t s, bool integrate, hipEvent_t t0, hipEvent_t t1)
{
    if (lp.reference_force) {
        if (lp.total[kWPart] > 0)
            launch_timed(k_force_gather, dim3(lp.total[kWPart]), dim3(kBlock), 0, s, t0, t1, lp.desc, lp.pre, lp.nbox);
    } else if (lp.total[kWTile] > 0) {
        // 0: forces only; 1: the kick-drift fused; 2: fused, with walls
        const int fuse = integrate && lp.fuse ? (lp.walls ? 2 : 1) : 0;
        if (lp.species)
            fuse == 2 ? launch_tiled<true, 2>(lp, s, t0, t1)
                      : (fuse == 1 ? launch_tiled<true, 1>(lp, s, t0, t1) : launch_tiled<true, 0>(lp, s, t0, t1));
        else
            fuse == 2 ? launch_tiled<false, 2>(lp, s, t0, t1)
                      : (fuse == 1 ? launch_tiled<false, 1>(lp, s, t0, t1) : launch_tiled<false, 0>(lp, s, t0, t1));
    }
    return hipGetLastError();
}

hipError_t force_tiled_prepare(int lds_bytes)
{
    if (lds_bytes <= 65536) return hipSuccess;
    const void* fns[] = {
        (const void*)k_force_tiled<false, 256, 0>, (const void*)k_force_tiled<false, 512, 0>,
        (const void*)k_force_tiled<false, 1024, 0>, (const void*)k_force_tiled<true, 256, 0>,
        (const void*)k_force_tiled<true, 512, 0>, (const void*)k_force_tiled<true, 1024, 0>,
        (const void*)k_force_tiled<false, 256, 1>, (const void*)k_force_tiled<false, 512, 1>,
        (const void*)k_force_tiled<false, 1024, 1>, (const void*)k_force_tiled<true, 256, 1>,
        (const void*)k_force_tiled<true, 512, 1>, (const void*)k_force_tiled<true, 1024, 1>,
        (const void*)k_force_tiled<false, 256, 2>, (const void*)k_force_tiled<false, 512, 2>,
        (const void*)k_force_tiled<false, 1024, 2>, (const void*)k_force_tiled<true, 256, 2>,
        (const void*)k_force_tiled<true, 512, 2>, (const void*)k_force_tiled<true, 1024, 2>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dpd
