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
//                  that lie in the halo.  Candidates with r < r_c are
//                  compacted into a per-wave queue (ballot + popcount) and
//                  evaluated 64 at a time with every lane busy.  Both halves
//                  of a pair inside the tile are accumulated (F_ij to i,
//                  -F_ij to j); a pair that crosses the tile boundary is
//                  evaluated once from each side and only the tile particle is
//                  updated, so every force is written exactly once.
//
// Bitwise agreement of the two kernels follows from the rules in
// dpd_device.hpp: exact displacements, exactly antisymmetric pair forces and
// order-independent fixed-point sums.
#include <cmath>

#include "dpd_internal.hpp"

namespace dpd {

__device__ __forceinline__ int wrap_cell(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

__device__ __forceinline__ float body_force_of(float4 p, const ForceConst& fc)
{
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
__device__ __forceinline__ bool pair_fx(float4 pi, float4 vi, float4 pj, float4 vj, uint32_t step, const PairConst& pc,
                                        long long& fx, long long& fy, long long& fz)
{
    const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const float r2 = dist2(dx, dy, dz);
    const float xi = pair_xi(__float_as_uint(pi.w), __float_as_uint(pj.w), step, pc.k0, pc.k1);
    float rinv;
    const float fs = pair_scalar(r2, dx, dy, dz, vi.x - vj.x, vi.y - vj.y, vi.z - vj.z, rinv, xi, pc);
    const float Fx = fs * (dx * rinv), Fy = fs * (dy * rinv), Fz = fs * (dz * rinv);
    if (!(fabsf(Fx) < kFxLimit && fabsf(Fy) < kFxLimit && fabsf(Fz) < kFxLimit)) {
        fx = fy = fz = 0;
        return false;
    }
    fx = fx_of(Fx);
    fy = fx_of(Fy);
    fz = fx_of(Fz);
    return true;
}

// Force on particle i (cell order) by gathering over its 27 neighbour cells.
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
                    bad |= !pair_fx(pi, vi, pj, vel[j], step, fc.pc, fx, fy, fz);
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
    d.force[i] = gather_force_one(i, d.pos_b, d.vel_b, d.cell_start, d.fc, (uint32_t)d.st->step, bad);
    if (bad) atomicOr(&d.st->nonfinite, 1);
}

// ---------------------------------------------------------------------------
// tiled kernel
// ---------------------------------------------------------------------------
constexpr int kQueue = 256;     // per-wave hit ring buffer (< 64 pending + up to 128 new)
constexpr int kMaxSeg = 14;     // candidate runs per tile particle

__device__ __forceinline__ void flush_hit(unsigned e, const float4* sp, const float4* sv, long long* acc,
                                          uint32_t step, const PairConst& pc, bool& bad)
{
    const int a = (int)(e >> 16), b = (int)(e & 0xffffu);
    const float4 va = sv[a], vb = sv[b];
    long long fx, fy, fz;
    bad |= !pair_fx(sp[a], va, sp[b], vb, step, pc, fx, fy, fz);
    const int ia = __float_as_int(va.w), ib = __float_as_int(vb.w);
    atomicAdd((unsigned long long*)&acc[3 * ia], (unsigned long long)fx);
    atomicAdd((unsigned long long*)&acc[3 * ia + 1], (unsigned long long)fy);
    atomicAdd((unsigned long long*)&acc[3 * ia + 2], (unsigned long long)fz);
    if (ib >= 0) {                       // both ends in the tile: apply the reaction too
        atomicAdd((unsigned long long*)&acc[3 * ib], (unsigned long long)(-fx));
        atomicAdd((unsigned long long*)&acc[3 * ib + 1], (unsigned long long)(-fy));
        atomicAdd((unsigned long long*)&acc[3 * ib + 2], (unsigned long long)(-fz));
    }
}

__global__ __launch_bounds__(kBlock) void k_force_tiled(const BoxDesc* __restrict__ desc, const int* __restrict__ pre,
                                                        int nbox)
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
    extern __shared__ __align__(16) unsigned char lds[];
    float4* sp = (float4*)lds;                                  // staged positions (image-shifted), w = id
    float4* sv = (float4*)(lds + tc.off_sv);                    // staged velocities, w = tile index or -1
    long long* acc = (long long*)(lds + tc.off_acc);            // fixed-point force of tile particles
    unsigned short* ps = (unsigned short*)(lds + tc.off_ps);    // tile index -> staged index
    int* cst = (int*)(lds + tc.off_cst);                        // staged cell offsets in LDS (ncs + 1)
    int* cg = (int*)(lds + tc.off_cg);                          // staged cell start in HBM (cell order)
    int4* rows = (int4*)(lds + tc.off_rows);                    // tile rows: (lds start, len, HBM start, tile start)
    unsigned* qall = (unsigned*)(lds + tc.off_q);               // per-wave hit queues
    unsigned* segall = (unsigned*)(lds + tc.off_seg);           // per-wave candidate segments [slot][lane]
    __shared__ int s_scr[kBlock / 64];

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
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const uint32_t step = (uint32_t)d.st->step;

    // 1. HBM start and particle count of every staged cell (the only
    //    dependent HBM round trip before the copy), scanned into LDS offsets
    for (int lc = tid; lc < ncs; lc += blockDim.x) {
        const int lx = lc % S0, ly = (lc / S0) % S1, lz = lc / (S0 * S1);
        const int g = wrap_cell(o0 - 1 + lx, L0) + L0 * (wrap_cell(o1 - 1 + ly, L1) + L1 * wrap_cell(o2 - 1 + lz, L2));
        const int gs = cell_start[g];
        cg[lc] = gs;
        cst[lc] = cell_start[g + 1] - gs;
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
                const int ly = 1 + r % P1, lz = 1 + r / P1;
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

    if (S > tc.smax || nt > tc.pmax || (d.flags & kFlagReference)) {
        // Overfull tile (or the box asks for the reference path): gather
        // from HBM, same arithmetic and same bits.
        bool bad = false;
        for (int r = wave; r < nrows; r += nw) {
            const int4 rw = rows[r];
            for (int k = lane; k < rw.y; k += 64)
                force[rw.z + k] = gather_force_one(rw.z + k, pos, vel, cell_start, fc, step, bad);
        }
        if (bad) atomicOr(nonfinite, 1);
        return;
    }

    // 3. stage the region: each staged row is at most three runs of cells
    //    contiguous in HBM (low wrap, interior, high wrap), copied with the
    //    periodic image shift
    const int nsrows = S1 * S2;
    for (int sr = wave; sr < nsrows; sr += nw) {
        const int ly = sr % S1, lz = sr / S1;
        const int gy = o1 - 1 + ly, gz = o2 - 1 + lz;
        const float sy = gy < 0 ? -fc.L[1] : (gy >= L1 ? fc.L[1] : 0.0f);
        const float sz = gz < 0 ? -fc.L[2] : (gz >= L2 ? fc.L[2] : 0.0f);
        const bool tile_row = ly >= 1 && ly <= P1 && lz >= 1 && lz <= P2;
        int4 rw = make_int4(0, 0, 0, 0);
        if (tile_row) rw = rows[(ly - 1) + P1 * (lz - 1)];
        const int lcrow = S0 * (ly + S1 * lz);
        for (int seg = 0; seg < 3; ++seg) {
            int lx0, lx1;
            float sx = 0.0f;
            if (seg == 0) {                       // lx = 0 when it wraps to the top of the box
                if (o0 != 0) continue;
                lx0 = 0; lx1 = 1; sx = -fc.L[0];
            } else if (seg == 1) {                // cells inside [0, L0)
                lx0 = (o0 == 0) ? 1 : 0;
                lx1 = (o0 + P0 == L0) ? S0 - 1 : S0;
            } else {                              // lx = S0-1 when it wraps to the bottom
                if (o0 + P0 != L0) continue;
                lx0 = S0 - 1; lx1 = S0; sx = fc.L[0];
            }
            const int gsrc = cg[lcrow + lx0];
            const int dst0 = cst[lcrow + lx0];
            const int cnt = cst[lcrow + lx1] - dst0;
            for (int k = lane; k < cnt; k += 64) {
                float4 p = pos[gsrc + k];
                float4 v = vel[gsrc + k];
                const int dst = dst0 + k;
                p.x += sx;
                p.y += sy;
                p.z += sz;
                int ti = -1;
                if (tile_row && dst >= rw.x && dst < rw.x + rw.y) {
                    ti = rw.w + (dst - rw.x);
                    ps[ti] = (unsigned short)dst;
                }
                v.w = __int_as_float(ti);
                sp[dst] = p;
                sv[dst] = v;
            }
        }
    }
    for (int k = tid; k < 3 * nt; k += blockDim.x) acc[k] = 0;
    __syncthreads();

    // 4. candidates.  The half stencil of a tile particle, as runs of
    //    consecutive staged particles (a row of three neighbour cells is
    //    contiguous in LDS): own cell after i plus cell x+1; the forward rows
    //    (y+1, z) and (y-1..y+1, z+1); and, only where they are halo cells,
    //    the backward rows (y-1, z) and (y-1..y+1, z-1) and cell x-1.
    //    A row or an end cell is dropped when its distance from i is >= r_c;
    //    the bound is evaluated with the same FP32 operations as r^2 on exact
    //    gaps, so it never drops a pair with r^2 < 1.
    unsigned* q = qall + wave * kQueue;                 // ring buffer
    unsigned* seg = segall + wave * (kMaxSeg * 64) + lane;
    int qh = 0, qt = 0;                                 // wave-uniform head and tail
    bool bad = false;
    for (int pb = wave * 64; pb < nt; pb += blockDim.x) {
        const int p = pb + lane;
        int si = 0, nseg = 0;
        float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < nt) {
            si = ps[p];
            xi = sp[si];
            const float cxf = floorf(xi.x), cyf = floorf(xi.y), czf = floorf(xi.z);
            const int lx = min(max((int)cxf - o0 + 1, 1), P0);
            const int ly = min(max((int)cyf - o1 + 1, 1), P1);
            const int lz = min(max((int)czf - o2 + 1, 1), P2);
            // exact gaps to the lower and upper faces of i's cell
            const float gxl = xi.x - cxf, gxr = (cxf + 1.0f) - xi.x;
            const float gyl = xi.y - cyf, gyr = (cyf + 1.0f) - xi.y;
            const float gzl = xi.z - czf, gzr = (czf + 1.0f) - xi.z;
            auto add = [&](int a, int b) {
                if (a < b) {
                    seg[nseg * 64] = (unsigned)a | ((unsigned)b << 16);
                    ++nseg;
                }
            };
            // row (dy, dz) relative to i; `mid` = include the cells of the row
            // inside the tile, otherwise only its halo end cells
            auto row = [&](int dy, int dz, bool mid) {
                const float gy = dy > 0 ? gyr : (dy < 0 ? gyl : 0.0f);
                const float gz = dz > 0 ? gzr : (dz < 0 ? gzl : 0.0f);
                const float gyz = gy * gy;
                if (!(fmaf(gz, gz, gyz) < 1.0f)) return;
                const bool left = fmaf(gz, gz, fmaf(gy, gy, gxl * gxl)) < 1.0f;
                const bool right = fmaf(gz, gz, fmaf(gy, gy, gxr * gxr)) < 1.0f;
                const int r = S0 * ((ly + dy) + S1 * (lz + dz));
                if (mid) {
                    add(cst[r + (left ? lx - 1 : lx)], cst[r + (right ? lx + 2 : lx + 1)]);
                } else {
                    if (lx == 1 && left) add(cst[r], cst[r + 1]);
                    if (lx == P0 && right) add(cst[r + P0 + 1], cst[r + P0 + 2]);
                }
            };
            const int lcr = S0 * (ly + S1 * lz);
            add(si + 1, cst[lcr + (gxr * gxr < 1.0f ? lx + 2 : lx + 1)]);   // own cell tail, cell x+1
            row(1, 0, true);
            row(-1, 1, true);
            row(0, 1, true);
            row(1, 1, true);
            const int by[4] = {-1, -1, 0, 1}, bz[4] = {0, -1, -1, -1};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ny = ly + by[k], nz = lz + bz[k];
                row(by[k], bz[k], ny < 1 || ny > P1 || nz < 1 || nz > P2);
            }
            if (lx == 1) add(cst[lcr], cst[lcr + 1]);                         // cell x-1 (halo)
        }
        const unsigned tag = (unsigned)si << 16;
        int k = 0, j = 0, je = 0;
        unsigned nxt = nseg > 0 ? seg[0] : 0u;
        while (true) {
            if (j >= je && k < nseg) {
                j = (int)(nxt & 0xffffu);
                je = (int)(nxt >> 16);
                ++k;
                if (k < nseg) nxt = seg[k * 64];
            }
            const bool a0 = j < je, a1 = j + 1 < je;
            if (__ballot(a0) == 0ull) break;
            const float4 x0 = sp[a0 ? j : 0];
            const float4 x1 = sp[a1 ? j + 1 : 0];
            const float r0 = dist2(xi.x - x0.x, xi.y - x0.y, xi.z - x0.z);
            const float r1 = dist2(xi.x - x1.x, xi.y - x1.y, xi.z - x1.z);
            const bool h0 = a0 && r0 < 1.0f && r0 > 0.0f;
            const bool h1 = a1 && r1 < 1.0f && r1 > 0.0f;
            const unsigned long long m0 = __ballot(h0), m1 = __ballot(h1);
            const int c0 = __popcll(m0);
            if (h0) q[(qt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m0, 0u))) & (kQueue - 1)] = tag | (unsigned)j;
            if (h1) q[(qt + c0 + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m1, 0u))) & (kQueue - 1)] = tag | (unsigned)(j + 1);
            qt += c0 + __popcll(m1);
            j += (int)a0 + (int)a1;
            while (qt - qh >= 64) {
                __builtin_amdgcn_wave_barrier();
                flush_hit(q[(qh + lane) & (kQueue - 1)], sp, sv, acc, step, fc.pc, bad);
                __builtin_amdgcn_wave_barrier();
                qh += 64;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < qt - qh) flush_hit(q[(qh + lane) & (kQueue - 1)], sp, sv, acc, step, fc.pc, bad);
    if (bad) atomicOr(nonfinite, 1);
    __syncthreads();

    // 5. each tile particle's force is written once, in cell order
    for (int r = wave; r < nrows; r += nw) {
        const int4 rw = rows[r];
        for (int k = lane; k < rw.y; k += 64) {
            const int ti = rw.w + k;
            force[rw.z + k] = finish_force(acc[3 * ti], acc[3 * ti + 1], acc[3 * ti + 2], sp[rw.x + k], fc);
        }
    }
}

TileConst make_tile_const(const int* cells, int64_t n, const int* tile, int smax_override, int pmax_override)
{
    TileConst tc{};
    int64_t nc = 1;
    for (int k = 0; k < 3; ++k) {
        tc.T[k] = tile[k] < cells[k] ? tile[k] : cells[k];
        tc.ntile[k] = (cells[k] + tc.T[k] - 1) / tc.T[k];
        nc *= cells[k];
    }
    tc.ntiles = tc.ntile[0] * tc.ntile[1] * tc.ntile[2];
    const double rho = nc > 0 ? (double)n / (double)nc : 0.0;
    const int ncs_max = (tc.T[0] + 2) * (tc.T[1] + 2) * (tc.T[2] + 2);
    const int ntc = tc.T[0] * tc.T[1] * tc.T[2];
    // capacities: mean + 6 standard deviations of a uniform fluid, rounded up
    auto cap = [](double mean) { int c = (int)std::ceil(mean + 6.0 * std::sqrt(mean + 1.0) + 16.0); return (c + 63) & ~63; };
    tc.smax = smax_override > 0 ? smax_override : cap(rho * ncs_max);
    tc.pmax = pmax_override > 0 ? pmax_override : cap(rho * ntc);
    if (tc.smax > 65535) tc.smax = 65535;
    size_t off = (size_t)tc.smax * 16;
    tc.off_sv = (int)off;
    off += (size_t)tc.smax * 16;
    tc.off_acc = (int)off;
    off += (size_t)tc.pmax * 24;
    tc.off_ps = (int)off;
    off += ((size_t)tc.pmax * 2 + 15) & ~(size_t)15;
    tc.off_cst = (int)off;
    off += ((size_t)(ncs_max + 1) * 4 + 15) & ~(size_t)15;
    tc.off_cg = (int)off;
    off += ((size_t)ncs_max * 4 + 15) & ~(size_t)15;
    tc.off_rows = (int)off;
    off += (size_t)tc.T[1] * tc.T[2] * 16;
    tc.off_q = (int)off;
    off += (size_t)(kBlock / 64) * kQueue * 4;
    tc.off_seg = (int)off;
    off += (size_t)(kBlock / 64) * kMaxSeg * 64 * 4;
    tc.lds_bytes = (int)off;
    return tc;
}

hipError_t launch_force(const LaunchPlan& lp, hipStream_t s)
{
    if (lp.reference_force) {
        if (lp.total[kWPart] > 0)
            hipLaunchKernelGGL(k_force_gather, dim3(lp.total[kWPart]), dim3(kBlock), 0, s, lp.desc, lp.pre, lp.nbox);
    } else if (lp.total[kWTile] > 0) {
        hipLaunchKernelGGL(k_force_tiled, dim3(lp.total[kWTile]), dim3(kBlock), lp.lds_force, s, lp.desc, lp.pre,
                           lp.nbox);
    }
    return hipGetLastError();
}

hipError_t force_tiled_prepare(int lds_bytes)
{
    if (lds_bytes > 65536)
        return hipFuncSetAttribute((const void*)k_force_tiled, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    return hipSuccess;
}

}  // namespace dpd
