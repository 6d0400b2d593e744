// dpd_kernels.hip -- gfx950 kernels of the DPD step: cell binning, pair
// forces, fused velocity-Verlet with FP64 reductions, and read-back helpers.
//
// Binning (Sec. 3.2 of the Mirheo paper: cells of edge r_c, particles sorted
// by cell) is a counting sort made stable and deterministic:
//   keys    -- cell of each particle and an arrival slot from an atomic
//              per-cell counter, plus particle counts per kSubChunk cells
//              from a second counter (fused into the kick-drift: the force
//              kernel's write-out, or k_integrate on the reference force
//              path; after a state load, k_keys and k_sub_sums);
//   scan    -- each block scans its chunk after a block-wide reduction of the
//              chunk sums before it, giving cell_start; counters are zeroed;
//   scatter -- perm[cell_start + slot] = particle (slot order is arbitrary),
//              and the cell of that position beside it (so the gather looks up
//              the cell's bounds while it loads the particle); the sub-chunk
//              counts are zeroed for the next step;
//   gather  -- each particle's final place is cell_start + its rank by
//              previous index among the cell's members, so the order inside a
//              cell is the previous array order whatever the atomics did.
#include "dpd_internal.hpp"

namespace dpd {

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int* p, int value, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_i32(int* p, int value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, value, count);
    return hipGetLastError();
}

// Load n rows (id order) of positions and velocities, round positions to the
// grid q and flag rows outside [0, L) or non-finite.
__global__ void k_load_state(const float* __restrict__ pos3, const float* __restrict__ vel3, int n,
                             float4* __restrict__ pos, float4* __restrict__ vel, float q, float inv_q,
                             float Lx, float Ly, float Lz, int* bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = pos3[3 * i], y = pos3[3 * i + 1], z = pos3[3 * i + 2];
    const float vx = vel3[3 * i], vy = vel3[3 * i + 1], vz = vel3[3 * i + 2];
    const bool ok = (x >= 0.0f && x < Lx) && (y >= 0.0f && y < Ly) && (z >= 0.0f && z < Lz) &&
                    isfinite(vx) && isfinite(vy) && isfinite(vz);
    if (!ok) {
        atomicOr(bad, 1);
        x = y = z = 0.0f;
    }
    x = rintf(x * inv_q) * q;
    y = rintf(y * inv_q) * q;
    z = rintf(z * inv_q) * q;
    if (x >= Lx) x -= Lx;
    if (y >= Ly) y -= Ly;
    if (z >= Lz) z -= Lz;
    pos[i] = make_float4(x, y, z, __int_as_float(i));
    vel[i] = make_float4(vx, vy, vz, 0.0f);
}

hipError_t launch_load_state(const float* pos3, const float* vel3, int n, float4* pos, float4* vel, float q,
                             float inv_q, const float* L, int* bad, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_state, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos3, vel3, n, pos,
                       vel, q, inv_q, L[0], L[1], L[2], bad);
    return hipGetLastError();
}

// Random initial state on the device: positions uniform on [0, L) on the
// grid q, velocities N(0, kT/m) per component (Box-Muller), from Philox with
// counters (i, 0xffffffff, k, 1) -- the last word keeps these streams apart
// from the pair-noise counters, whose last word is 0.  Per-block FP64 sums
// of the velocities go to `partials` for the centre-of-mass removal.
__global__ __launch_bounds__(kBlock) void k_init_random(int n, float Lx, float Ly, float Lz, float q, float inv_q,
                                                        float vscale, uint32_t k0, uint32_t k1,
                                                        float4* __restrict__ pos, float4* __restrict__ vel,
                                                        double* __restrict__ partials)
{
    __shared__ double s_red[kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double sv[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const uint4 a = philox10(make_uint4((uint32_t)i, 0xffffffffu, 0u, 1u), k0, k1);
        const uint4 b = philox10(make_uint4((uint32_t)i, 0xffffffffu, 1u, 1u), k0, k1);
        const uint4 c = philox10(make_uint4((uint32_t)i, 0xffffffffu, 2u, 1u), k0, k1);
        const float L[3] = {Lx, Ly, Lz};
        const uint32_t w[3] = {a.x, a.y, a.z};
        float x[3];
        for (int k = 0; k < 3; ++k) {
            const float u = (float)(w[k] >> 8) * 0x1p-24f;                 // [0, 1)
            float v = floorf(u * L[k] * inv_q) * q;
            x[k] = v >= L[k] ? 0.0f : v;
        }
        const float g0 = box_muller(b.x, b.y), g1 = box_muller(b.z, b.w), g2 = box_muller(c.x, c.y);
        const float v3[3] = {g0 * vscale, g1 * vscale, g2 * vscale};
        pos[i] = make_float4(x[0], x[1], x[2], __int_as_float(i));
        vel[i] = make_float4(v3[0], v3[1], v3[2], 0.0f);
        for (int k = 0; k < 3; ++k) sv[k] = (double)v3[k];
    }
    for (int k = 0; k < 3; ++k) {
        const double t = block_sum(sv[k], s_red);
        if (threadIdx.x == 0) partials[blockIdx.x * 3 + k] = t;
    }
}

// Mean velocity from the per-block sums (fixed order), subtracted from every
// particle (FP32).
__global__ __launch_bounds__(kBlock) void k_remove_com(int n, int nblocks, const double* __restrict__ partials,
                                                       float4* __restrict__ vel)
{
    __shared__ double s_mean[3];
    __shared__ double s_red[kBlock / 64];
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) t += partials[b * 3 + k];
        t = block_sum(t, s_red);
        if (threadIdx.x == 0) s_mean[k] = n > 0 ? t / (double)n : 0.0;
    }
    __syncthreads();
    const float mx = (float)s_mean[0], my = (float)s_mean[1], mz = (float)s_mean[2];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        float4 v = vel[i];
        v.x -= mx;
        v.y -= my;
        v.z -= mz;
        vel[i] = v;
    }
}

hipError_t launch_init_random(int n, const float* L, float q, double vscale, uint64_t seed, float4* pos, float4* vel,
                              double* scratch, int scratch_doubles, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (n + kBlock - 1) / kBlock;
    if (blocks * 3 > scratch_doubles) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_init_random, dim3(blocks), dim3(kBlock), 0, s, n, L[0], L[1], L[2], q, 1.0f / q,
                       (float)vscale, (uint32_t)seed, (uint32_t)(seed >> 32), pos, vel, scratch);
    hipLaunchKernelGGL(k_remove_com, dim3(blocks < 1024 ? blocks : 1024), dim3(kBlock), 0, s, n, blocks, scratch, vel);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
// count must be zero on entry.
__global__ void k_keys(const float4* __restrict__ pos, int n, int Lx, int Ly, int Lz, int* __restrict__ count,
                       int2* __restrict__ keyslot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;                      // a prefix of each wave; every lane takes part below
    int c = -1;
    if (live) {
        const float4 p = pos[i];
        c = cell_of(p.x, p.y, p.z, Lx, Ly, Lz);
    }
    const ArrivalTicket tk = arrival_issue(c, live, count);
    const int slot = arrival_finish(tk, live);
    if (live) keyslot[i] = make_int2(c, slot);
}

// Sub-chunk counts from the cell counts, one wave per sub-chunk.  A state
// load is in no particular cell order, so counting through chunk_add would
// put every particle's atomic on a few hundred addresses.
__global__ __launch_bounds__(kBlock) void k_sub_sums(const int* __restrict__ count, int nc, int nsub,
                                                     int* __restrict__ bsum)
{
    static_assert(kSubChunk == 64, "one lane per cell of a sub-chunk");
    const int k = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int c = k * kSubChunk + (int)(threadIdx.x & 63);
    const int t = wave_sum(c < nc ? count[c] : 0);   // uniform per wave: every lane takes part
    if (k < nsub && (threadIdx.x & 63) == 0) bsum[k] = t;
}

hipError_t launch_keys(const float4* pos, int n, const int* cells, int* count, int* bsum, int2* keyslot,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, n, cells[0], cells[1],
                       cells[2], count, keyslot);
    const int nc = cells[0] * cells[1] * cells[2];
    const int nsub = (nc + kSubChunk - 1) / kSubChunk;
    const int per = kBlock / 64;
    hipLaunchKernelGGL(k_sub_sums, dim3((nsub + per - 1) / per), dim3(kBlock), 0, s, count, nc, nsub, bsum);
    return hipGetLastError();
}

// Number of cells holding at least one particle (added to *out).
__global__ __launch_bounds__(kBlock) void k_count_nonempty(const int* __restrict__ count, int nc, int* __restrict__ out)
{
    __shared__ long long scratch[kBlock / 64];
    long long k = 0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock) k += count[c] > 0 ? 1 : 0;
    k = block_sum(k, scratch);
    if (threadIdx.x == 0 && k) atomicAdd(out, (int)k);
}

hipError_t launch_count_nonempty(const int* count, int nc, int* out, hipStream_t s)
{
    if (nc <= 0) return hipSuccess;
    const int blocks = (nc + kBlock - 1) / kBlock < 1024 ? (nc + kBlock - 1) / kBlock : 1024;
    hipLaunchKernelGGL(k_count_nonempty, dim3(blocks), dim3(kBlock), 0, s, count, nc, out);
    return hipGetLastError();
}

// Species by particle id into the .w of the velocity row holding that id.
__global__ void k_set_types(const float4* __restrict__ pos, float4* __restrict__ vel, int n,
                            const int* __restrict__ type_by_id)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int id = __float_as_int(pos[i].w);
    const int w = __float_as_int(vel[i].w);
    vel[i].w = __int_as_float(type_by_id[id] | (w & kFrozenBit));
}

__global__ void k_get_types(const float4* __restrict__ pos, const float4* __restrict__ vel, int n,
                            int* __restrict__ type_by_id)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    type_by_id[__float_as_int(pos[i].w)] = __float_as_int(vel[i].w) & 0xff;
}

__global__ void k_set_frozen(const float4* __restrict__ pos, float4* __restrict__ vel, int n,
                             const unsigned char* __restrict__ frozen_by_id, StepConst sc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 p = pos[i];
    float4 v = vel[i];
    const int w = __float_as_int(v.w) & ~kFrozenBit;
    if (frozen_by_id[__float_as_int(p.w)]) {
        const float3 u = wall_velocity(p.x, p.y, p.z, sc);         // the wall's own velocity
        v = make_float4(u.x, u.y, u.z, __int_as_float(w | kFrozenBit));
    } else {
        v.w = __int_as_float(w);
    }
    vel[i] = v;
}

__global__ void k_get_frozen(const float4* __restrict__ pos, const float4* __restrict__ vel, int n,
                             unsigned char* __restrict__ frozen_by_id)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    frozen_by_id[__float_as_int(pos[i].w)] = (__float_as_int(vel[i].w) & kFrozenBit) ? 1 : 0;
}

__global__ void k_wall_sdf(const float4* __restrict__ pos, int n, StepConst sc, float* __restrict__ sdf_by_id)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 p = pos[i];
    sdf_by_id[__float_as_int(p.w)] = wall_sdf(p.x, p.y, p.z, sc);
}

hipError_t launch_set_types(const float4* pos, float4* vel, int n, const int* type_by_id, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_types, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, vel, n, type_by_id);
    return hipGetLastError();
}

hipError_t launch_get_types(const float4* pos, const float4* vel, int n, int* type_by_id, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_get_types, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, vel, n, type_by_id);
    return hipGetLastError();
}

hipError_t launch_set_frozen(const float4* pos, float4* vel, int n, const unsigned char* frozen_by_id,
                             const StepConst& sc, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_frozen, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, vel, n, frozen_by_id,
                       sc);
    return hipGetLastError();
}

hipError_t launch_get_frozen(const float4* pos, const float4* vel, int n, unsigned char* frozen_by_id, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_get_frozen, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, vel, n, frozen_by_id);
    return hipGetLastError();
}

hipError_t launch_wall_sdf(const float4* pos, int n, const StepConst& sc, float* sdf_by_id, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wall_sdf, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pos, n, sc, sdf_by_id);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// step kernels: each workgroup finds its box in the launch group, then works
// on that box exactly as it would alone (same partition, same order)
// ---------------------------------------------------------------------------
#define DPD_BOX_OF(kind)                                                       \
    const int* __restrict__ pre_ = pre + (kind) * (nbox + 1);                  \
    const int box_ = nbox == 1 ? 0 : find_box(pre_, nbox, (int)blockIdx.x);   \
    const BoxDesc& d = desc[box_];                                             \
    const int lb = (int)blockIdx.x - pre_[box_];

int integrate_blocks(int n)
{
    int b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return b > kIntegrateMaxBlocks ? kIntegrateMaxBlocks : b;
}

// Blocks of the per-particle kernels: every particle, and every chunk sum
// that k_scatter zeroes.  The gather launch has one block more, which folds
// the previous step's reductions (hidden behind the gather's own work).
__host__ __device__ inline int part_blocks(const BoxDesc& d)
{
    const int np = (d.n + kBlock - 1) / kBlock, nk = (d.nsub + kBlock - 1) / kBlock;
    return np > nk ? np : nk;
}

int box_work(const BoxDesc& d, int kind)
{
    switch (kind) {
    case kWChunk: return d.nchunks;
    case kWPart: return part_blocks(d) + 1;                   // + one block that folds the reductions

    case kWTile: return ((d.tc.ntiles + 7) / 8) * 8;       // padded for the XCD swizzle
    default: return d.nblk_int;
    }
}

__device__ void fold_stats(const BoxDesc& d);

__global__ __launch_bounds__(kBlock) void k_scan(const BoxDesc* __restrict__ desc, const int* __restrict__ pre, int nbox)
{
    DPD_BOX_OF(kWChunk)
    constexpr int per = kScanChunk / kBlock;   // consecutive cells per thread
    __shared__ int scratch[kBlock / 64];
    __shared__ int wtot[kBlock / 64];
    const int nc = d.nc;
    int* __restrict__ count = d.count;
    // this chunk's counts first: their loads overlap the prefix below
    const int c0 = lb * kScanChunk + threadIdx.x * per;
    int v[per];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = (c0 + k < nc) ? count[c0 + k] : 0;
        tsum += v[k];
    }
    // prefix of this chunk: sum of the sub-chunk counts before it
    // (a whole number of int4s: chunks are 8 sub-chunks, the array 256-byte aligned)
    static_assert((kScanChunk / kSubChunk) % 4 == 0, "int4 reads of whole chunks");
    const int4* __restrict__ b4 = reinterpret_cast<const int4*>(d.bsum);
    const int nk4 = lb * (kScanChunk / kSubChunk / 4);
    int p0 = 0, p1 = 0;
    int j = threadIdx.x;
    for (; j + kBlock < nk4; j += 2 * kBlock) {
        const int4 q0 = b4[j], q1 = b4[j + kBlock];
        p0 += (q0.x + q0.y) + (q0.z + q0.w);
        p1 += (q1.x + q1.y) + (q1.z + q1.w);
    }
    if (j < nk4) {
        const int4 q0 = b4[j];
        p0 += (q0.x + q0.y) + (q0.z + q0.w);
    }
    int prefix = p0 + p1;
    prefix = block_sum(prefix, scratch);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int incl = wave_incl_scan(tsum);
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wtot[w];
    int run = prefix + wpre + incl - tsum;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (c0 + k < nc) {
            d.cell_start[c0 + k] = run;
            count[c0 + k] = 0;
        }
        run += v[k];
    }
    if (lb == d.nchunks - 1 && threadIdx.x == 0) d.cell_start[nc] = d.n;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const BoxDesc* __restrict__ desc, const int* __restrict__ pre,
                                                    int nbox)
{
    DPD_BOX_OF(kWPart)
    const int i = lb * kBlock + threadIdx.x;
    if (i < d.nsub) d.bsum[i] = 0;               // the scan has read them; the next keys add to zero
    if (i >= d.n) return;
    const int2 ks = d.keyslot[i];
    const int p = d.cell_start[ks.x] + ks.y;
    d.perm[p] = i;
    d.cellof[p] = ks.x;
}

__global__ __launch_bounds__(kBlock) void k_gather(const BoxDesc* __restrict__ desc, const int* __restrict__ pre,
                                                   int nbox)
{
    DPD_BOX_OF(kWPart)
    if (lb == part_blocks(d)) {                 // the extra block: the previous step's reductions
        fold_stats(d);
        return;
    }
    const int p = lb * kBlock + threadIdx.x;
    if (p >= d.n) return;
    const int* __restrict__ perm = d.perm;
    const int i = perm[p], c = d.cellof[p];
    const float4 x = d.pos_a[i], v = d.vel_a[i];     // in flight during the rank search
    const int s = d.cell_start[c], e = d.cell_start[c + 1];
    // the first eight members in one round of independent loads (a cell
    // rarely holds more), then the rest one by one
    int rank = 0;
    const int last = d.n - 1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int o = perm[min(s + k, last)];
        rank += (s + k < e && o < i) ? 1 : 0;
    }
    for (int t = s + 8; t < e; ++t) rank += perm[t] < i;
    d.pos_b[s + rank] = x;
    d.vel_b[s + rank] = v;
}

hipError_t launch_bin(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    const bool parts = lp.total[kWPart] > 0;
    if (lp.total[kWChunk] > 0)
        launch_timed(k_scan, dim3(lp.total[kWChunk]), dim3(kBlock), 0, s, t0, parts ? nullptr : t1, lp.desc, lp.pre,
                     lp.nbox);
    if (parts) {
        launch_timed(k_scatter, dim3(lp.total[kWPart]), dim3(kBlock), 0, s, lp.total[kWChunk] > 0 ? nullptr : t0,
                     nullptr, lp.desc, lp.pre, lp.nbox);
        launch_timed(k_gather, dim3(lp.total[kWPart]), dim3(kBlock), 0, s, nullptr, t1, lp.desc, lp.pre, lp.nbox);
    }
    return hipGetLastError();
}

// Conservative virial sum_{i<j} r_ij . F^C_ij = sum_i sum_{j != i} a w r / 2,
// per particle in FP64, then added as fixed point (order-independent).
__global__ __launch_bounds__(kBlock) void k_virial(const BoxDesc* __restrict__ desc, const int* __restrict__ pre,
                                                   int nbox)
{
    DPD_BOX_OF(kWPart)
    if (!(d.flags & kFlagVirial)) return;
    __shared__ long long scratch[kBlock / 64];
    const ForceConst& fc = d.fc;
    const float4* __restrict__ pos = d.pos_b;
    const float4* __restrict__ vel = d.vel_b;
    const int* __restrict__ cell_start = d.cell_start;
    const int i = lb * kBlock + threadIdx.x;
    const bool species = fc.ntypes > 1;
    double acc = 0.0;
    if (i < d.n) {
        const float4 pi = pos[i];
        const int ti = species ? __float_as_int(vel[i].w) : 0;
        const int Lx = fc.cells[0], Ly = fc.cells[1], Lz = fc.cells[2];
        const int cx = cell_coord(pi.x, Lx), cy = cell_coord(pi.y, Ly), cz = cell_coord(pi.z, Lz);
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
                    for (int j = cell_start[cell]; j < cell_start[cell + 1]; ++j) {
                        if (j == i) continue;
                        const float4 pj = pos[j];
                        const double ddx = (double)(pi.x - (pj.x + sx));
                        const double ddy = (double)(pi.y - (pj.y + sy));
                        const double ddz = (double)(pi.z - (pj.z + sz));
                        const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        if (!(r2 < 1.0) || r2 == 0.0) continue;
                        const double r = sqrt(r2);
                        if (species) {          // the pair's a and cutoff
                            const float4 c = fc.tab[species_pair(ti, __float_as_int(vel[j].w))];
                            const double w = 1.0 - r * (double)c.w;
                            if (w > 0.0) acc += 0.5 * (double)c.x * w * r;
                        } else {
                            acc += 0.5 * (double)fc.pc.a * (1.0 - r) * r;
                        }
                    }
                }
            }
        }
    }
    long long v = (long long)llrint(acc * kVirScale);
    v = block_sum(v, scratch);
    if (threadIdx.x == 0 && v != 0) atomicAdd((unsigned long long*)&d.st->virial_fx, (unsigned long long)v);
}

hipError_t launch_virial(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    if (!lp.any_virial || lp.total[kWPart] <= 0) return hipSuccess;
    launch_timed(k_virial, dim3(lp.total[kWPart]), dim3(kBlock), 0, s, t0, t1, lp.desc, lp.pre, lp.nbox);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused velocity-Verlet + next keys + FP64 reductions, as a kernel of its own:
// the step of the reference force path (every other step runs the same
// kick-drift in the force kernel's write-out)
// ---------------------------------------------------------------------------
constexpr int kLdsBins = 1024;

// kWalls: some box of the launch has walls (bounce-back and frozen particles);
// the plain instantiation keeps the register budget of the wall-free step.
template <bool kWalls>
__global__ __launch_bounds__(kBlock) void k_integrate(const BoxDesc* __restrict__ desc, const int* __restrict__ pre,
                                                      int nbox)
{
    DPD_BOX_OF(kWInt)
    __shared__ long long s_psum[kLdsBins];
    __shared__ int s_pcnt[kLdsBins];
    __shared__ double s_red[kBlock / 64][kPartials];
    const StepConst& sc = d.sc;
    const int n = d.n;
    const float4* __restrict__ pos_s = d.pos_b;
    const float4* __restrict__ vel_s = d.vel_b;
    const float4* __restrict__ force = d.force;
    float4* __restrict__ pos_a = d.pos_a;
    float4* __restrict__ vel_a = d.vel_a;
    int2* __restrict__ keyslot = d.keyslot;
    long long* __restrict__ profile = d.profile;
    const int nbins = sc.nbins;
    const bool lds_prof = nbins > 0 && nbins <= kLdsBins;
    if (lds_prof)
        for (int b = threadIdx.x; b < nbins; b += kBlock) { s_psum[b] = 0; s_pcnt[b] = 0; }
    __syncthreads();

    double m[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool bad = false, esc = false;
    const int stride = d.nblk_int * kBlock;
    for (int i0 = lb * kBlock; i0 < n; i0 += stride) {   // uniform per block: all lanes reach arrival_slot
        const int i = i0 + threadIdx.x;
        const bool live = i < n;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f), v = x, f = x;
        if (live) {
            x = pos_s[i];
            v = vel_s[i];
            f = force[i];
        }
        const bool frozen = kWalls && (__float_as_int(v.w) & kFrozenBit) != 0;   // wall particles never move
        Kicked k;
        if constexpr (!kWalls) {
            k = kick_drift(x, v, f, sc);
        } else {
            k = kick_drift_walls(x, v, f, live, frozen, sc);
        }
        bad |= !k.fin;
        esc |= k.esc;
        const int c = live ? cell_of(k.nx, k.ny, k.nz, sc.cells[0], sc.cells[1], sc.cells[2]) : -1;
        const ArrivalTicket tk = arrival_issue(c, live, d.count);     // atomic in flight meanwhile
        chunk_add(c, live, d.bsum);
        if (live) {
            pos_a[i] = make_float4(k.nx, k.ny, k.nz, x.w);
            vel_a[i] = make_float4(k.vx, k.vy, k.vz, v.w);          // .w: species
        }
        if (live && k.fin && !frozen) {
            add_partials(m, k);
            if (nbins > 0) {
                const int b = profile_bin(x, sc);
                const long long q = profile_units(k.vcx, k.vcy, k.vcz, sc);
                if (lds_prof) {
                    atomicAdd((unsigned long long*)&s_psum[b], (unsigned long long)q);
                    atomicAdd(&s_pcnt[b], 1);
                } else {
                    atomicAdd((unsigned long long*)&profile[2 * b], (unsigned long long)q);
                    atomicAdd((unsigned long long*)&profile[2 * b + 1], 1ull);
                }
            }
        }
        const int slot = arrival_finish(tk, live);
        if (live) keyslot[i] = make_int2(c, slot);
    }
    if (bad) atomicOr(&d.st->nonfinite, 1);
    if (esc) atomicOr(&d.st->escaped, 1);
    if (lb == 0 && threadIdx.x == 0) {   // the fold adds up this kernel's block partials
        d.st->fold_count = (unsigned)d.nblk_int;
        d.st->fold_pending = 1;
    }
    // block partials: lane tree inside each wave, then waves in index order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < kPartials; ++kk) {
        const double t = wave_sum(m[kk]);
        if (lane == 0) s_red[wave][kk] = t;
    }
    __syncthreads();
    if (threadIdx.x < kPartials) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += s_red[w][threadIdx.x];
        d.partials[lb * kPartials + threadIdx.x] = t;
    }
    if (lds_prof)
        for (int b = threadIdx.x; b < nbins; b += kBlock)
            if (s_pcnt[b]) {
                atomicAdd((unsigned long long*)&profile[2 * b], (unsigned long long)s_psum[b]);
                atomicAdd((unsigned long long*)&profile[2 * b + 1], (unsigned long long)s_pcnt[b]);
            }
}

// Fold of a box's integrate partials into the step's reductions, in block
// order.  The whole workgroup calls it; it does nothing unless the integrate
// kernel left partials to fold.  It runs in the first block of the next
// step's scan kernel, or as its own kernel at the end of a run of steps.
__device__ void fold_stats(const BoxDesc& d)
{
    __shared__ double s_red[kBlock / 64][kPartials];
    DevStats* st = d.st;
    if (!st->fold_pending) return;                 // uniform: written by an earlier kernel
    const double* __restrict__ partials = d.partials;
    const int nblocks = (int)st->fold_count;
    const StepConst& sc = d.sc;
    // running sums the first thread updates, fetched while the partials load
    long long vir_fx = 0;
    double sum_kT = 0.0, sum_p = 0.0, sum_m[3] = {0.0, 0.0, 0.0};
    unsigned long long ns = 0;
    if (threadIdx.x == 0) {
        vir_fx = st->virial_fx;
        sum_kT = st->sum_kT_centred;
        sum_p = st->sum_pressure;
        sum_m[0] = st->sum_momentum[0];
        sum_m[1] = st->sum_momentum[1];
        sum_m[2] = st->sum_momentum[2];
        ns = st->nsamples;
    }
    // per thread: blocks b, b + kBlock, ... in four interleaved chains; then
    // the lane tree of each wave and the waves in index order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kPartials; ++k) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        int b = threadIdx.x;
        for (; b + 3 * kBlock < nblocks; b += 4 * kBlock) {
            t0 += partials[b * kPartials + k];
            t1 += partials[(b + kBlock) * kPartials + k];
            t2 += partials[(b + 2 * kBlock) * kPartials + k];
            t3 += partials[(b + 3 * kBlock) * kPartials + k];
        }
        for (; b < nblocks; b += kBlock) t0 += partials[b * kPartials + k];
        const double w = wave_sum((t0 + t1) + (t2 + t3));
        if (lane == 0) s_red[wave][k] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kPartials];
        for (int k = 0; k < kPartials; ++k) {
            double t = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) t += s_red[w][k];
            tot[k] = t;
        }
        const double mass = sc.mass;
        const double ke_half = 0.5 * mass * tot[3];
        const double ke_c = 0.5 * mass * tot[4];
        const double kT_c = 2.0 * ke_c * sc.inv_dof;
        const double vir = (double)vir_fx / kVirScale;
        st->virial_fx = 0;
        const double press = sc.rho * kT_c + vir * sc.inv_vol / 3.0;
        st->last[0] = mass * tot[0];
        st->last[1] = mass * tot[1];
        st->last[2] = mass * tot[2];
        st->last[3] = ke_half;
        st->last[4] = ke_c;
        st->last_kT_centred = kT_c;
        st->last_virial = vir;
        st->last_pressure = press;
        st->sum_kT_centred = sum_kT + kT_c;
        st->sum_pressure = sum_p + press;
        st->sum_momentum[0] = sum_m[0] + mass * tot[0];
        st->sum_momentum[1] = sum_m[1] + mass * tot[1];
        st->sum_momentum[2] = sum_m[2] + mass * tot[2];
        st->nsamples = ns + 1;
        // the step is complete: the next force evaluation takes the next
        // step's noise (no kernel of this step reads the counter any more)
        st->step += 1;
        st->fold_pending = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_fold_stats(const BoxDesc* __restrict__ desc)
{
    fold_stats(desc[blockIdx.x]);
}

hipError_t launch_integrate(const LaunchPlan& lp, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    if (lp.walls)
        launch_timed(k_integrate<true>, dim3(lp.total[kWInt]), dim3(kBlock), 0, s, t0, t1, lp.desc, lp.pre, lp.nbox);
    else
        launch_timed(k_integrate<false>, dim3(lp.total[kWInt]), dim3(kBlock), 0, s, t0, t1, lp.desc, lp.pre, lp.nbox);
    return hipGetLastError();
}

hipError_t launch_fold(const LaunchPlan& lp, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold_stats, dim3(lp.nbox), dim3(kBlock), 0, s, lp.desc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// read-back: rows in id order
// ---------------------------------------------------------------------------
__global__ void k_to_rows(const float4* __restrict__ src, const float4* __restrict__ sub, float sub_scale,
                          const float4* __restrict__ idsrc, int n, float* __restrict__ out3)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 v = src[i];
    if (sub) {
        const float4 u = sub[i];
        v.x = fmaf(u.x, sub_scale, v.x);
        v.y = fmaf(u.y, sub_scale, v.y);
        v.z = fmaf(u.z, sub_scale, v.z);
    }
    const int id = __float_as_int(idsrc[i].w);
    if (id < 0 || id >= n) return;
    out3[3 * id] = v.x;
    out3[3 * id + 1] = v.y;
    out3[3 * id + 2] = v.z;
}

hipError_t launch_to_rows(const float4* src, const float4* sub, float sub_scale, const float4* idsrc, int n,
                          float* out3, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_rows, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, sub, sub_scale, idsrc, n,
                       out3);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// random-term diagnostics
// ---------------------------------------------------------------------------
__global__ void k_philox(const uint32_t* __restrict__ ctr4, const uint32_t* __restrict__ key2, int64_t n,
                         uint32_t* __restrict__ out4)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = make_uint4(ctr4[4 * i], ctr4[4 * i + 1], ctr4[4 * i + 2], ctr4[4 * i + 3]);
    const uint32_t k0 = key2[2 * i], k1 = key2[2 * i + 1];
    // a wave whose lanes share one key takes the force kernels' variant
    const uint32_t u0 = __builtin_amdgcn_readfirstlane(k0), u1 = __builtin_amdgcn_readfirstlane(k1);
    const bool same = __builtin_amdgcn_ballot_w64(k0 != u0 || k1 != u1) == 0;
    const uint4 w = same ? philox10_uniform_key(c, u0, u1) : philox10(c, k0, k1);
    out4[4 * i] = w.x;
    out4[4 * i + 1] = w.y;
    out4[4 * i + 2] = w.z;
    out4[4 * i + 3] = w.w;
}

hipError_t launch_philox(const uint32_t* ctr4, const uint32_t* key2, int64_t n, uint32_t* out4, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, ctr4, key2, n, out4);
    return hipGetLastError();
}

__global__ void k_box_muller(const uint32_t* __restrict__ w0, const uint32_t* __restrict__ w1, int64_t n,
                             float* __restrict__ xi)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) xi[i] = box_muller(w0[i], w1[i]);
}

hipError_t launch_box_muller(const uint32_t* w0, const uint32_t* w1, int64_t n, float* xi, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_box_muller, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, w0, w1, n, xi);
    return hipGetLastError();
}

}  // namespace dpd
