// dpd_device.hpp -- device-side building blocks of the DPD step on gfx950.
//
// Pair arithmetic is FP32 with explicit fmaf and the library is compiled
// with -ffp-contract=off, so every kernel that evaluates a pair evaluates it
// with the same instruction sequence.  Three design rules make the result
// independent of which thread, tile or kernel evaluates a pair:
//
//  * positions live on the grid q = ulp_f32(L_max) (see include/dpd.h), so a
//    periodic image x +- L and every neighbour displacement r_i - r_j are
//    exact in FP32; hence r_ji == -r_ij bit for bit;
//  * the pair force is an odd function of (r_ij, v_ij) in FP32: negating both
//    negates every product feeding e_ij . v_ij exactly, so F_ji == -F_ij;
//  * forces are accumulated in 64-bit fixed point (2^31 units per force
//    unit) with a round-to-nearest-even, odd-symmetric conversion, so sums are exact
//    integers whose value does not depend on summation order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpd {

// Global-memory view of a device pointer.  A box's arrays reach the kernels
// as plain pointers inside its descriptor, which the compiler must treat as
// generic and access with FLAT instructions.  A FLAT access also counts
// against the LDS wait counter, so every later LDS wait of the wave (a
// shuffle, a barrier) waits until the access is done, stores included.
// Through the global view the compiler emits global_* instructions, which
// only the vector-memory counter tracks.
#define DPD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ DPD_GLOBAL T* gmem(T* p)
{
    return (DPD_GLOBAL T*)p;
}

// Stores of HIP's vector types through the global view (their assignment
// operators are declared for generic memory only).
__device__ __forceinline__ void gstore(float4* p, float4 v)
{
    typedef float __attribute__((ext_vector_type(4))) v4;
    const v4 t = {v.x, v.y, v.z, v.w};
    *(DPD_GLOBAL v4*)p = t;
}
__device__ __forceinline__ void gstore(int2* p, int2 v)
{
    typedef int __attribute__((ext_vector_type(2))) i2;
    const i2 t = {v.x, v.y};
    *(DPD_GLOBAL i2*)p = t;
}

// Device-scope relaxed atomics (what atomicAdd / atomicOr are) on global
// memory.
template <typename T>
__device__ __forceinline__ T gatomic_add(T* p, T v)
{
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T gatomic_or(T* p, T v)
{
    return __hip_atomic_fetch_or(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): round multipliers and
// Weyl key increments.
constexpr uint32_t kPhM0 = 0xD2511F53u;
constexpr uint32_t kPhM1 = 0xCD9E8D57u;
constexpr uint32_t kPhW0 = 0x9E3779B9u;
constexpr uint32_t kPhW1 = 0xBB67AE85u;

__host__ __device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhM1 * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += kPhW0;
        k1 += kPhW1;
    }
    return c;
}

// a ^ b ^ k in one instruction: gfx950's three-input bitwise operation with
// the truth table of a three-way xor (0x96, symmetric in its inputs).  k must
// be the same on every lane of the wave (it is passed in a scalar register).
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// philox10 for a key that is the same on every lane of the wave (the pair
// term's seed): the same words, with each round's two xors into the key
// fused into one instruction per word.
__device__ __forceinline__ uint4 philox10_uniform_key(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhM1 * c.z;
        c = make_uint4(xor3_uniform((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                       xor3_uniform((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
        k0 += kPhW0;
        k1 += kPhW1;
    }
    return c;
}

// Gaussian xi from the first two Philox words (Box-Muller on 24-bit
// uniforms u1 in (0, 1], u2 in [0, 1)).  v_log_f32 returns log2 and
// v_cos_f32 takes its argument in revolutions, so cos(2 pi u2) needs no
// argument scaling.
__device__ __forceinline__ float box_muller(uint32_t w0, uint32_t w1)
{
    const float u1 = (float)((w0 >> 8) + 1u) * 0x1p-24f;
    const float u2 = (float)(w1 >> 8) * 0x1p-24f;
    const float minus_2ln2 = -1.3862943611198906f;
    const float rad = __builtin_amdgcn_sqrtf(minus_2ln2 * __builtin_amdgcn_logf(u1));
    return rad * __builtin_amdgcn_cosf(u2);
}

// k0, k1 (the seed) are the same on every lane of the wave.
__device__ __forceinline__ float pair_xi(uint32_t id_i, uint32_t id_j, uint32_t step, uint32_t k0,
                                         uint32_t k1)
{
    const uint32_t lo = min(id_i, id_j), hi = max(id_i, id_j);
    const uint4 w = philox10_uniform_key(make_uint4(lo, hi, step, 0u), k0, k1);
    return box_muller(w.x, w.y);
}

// ---- fixed point ---------------------------------------------------------
constexpr float kFxScale = 0x1p31f;        // units per force unit
constexpr double kFxInv = 0x1p-31;
constexpr float kFxLimit = 0x1p19f;        // a pair force of |F| >= 2^19 is reported as non-finite
constexpr double kFxMagic = 0x1.8p52;      // 1.5 * 2^52
constexpr int kFxMagicHi = 0x43380000;     // its high word (the low word is 0)

// Fixed-point value of a force already scaled to units, g = F * 2^31 with
// |g| < 2^51: the nearest integer, ties to even, so fx(-g) == -fx(g).  In
// [2^52, 2^53) doubles are spaced by 1, so g + 1.5 * 2^52 rounds g to an
// integer held in the low mantissa bits; taking off the magic number's bits
// leaves that integer (two's complement, since |g| < 2^51).
__device__ __forceinline__ long long fx_of_units(float g)
{
    const long long b = __double_as_longlong((double)g + kFxMagic);
    const int hi = (int)(b >> 32) - kFxMagicHi;
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)b);
}

struct PairConst {
    float a;          // conservative amplitude
    float gamma;      // dissipative coefficient
    float sig_rdt;    // sigma / sqrt(dt)
    uint32_t k0, k1;  // Philox key = seed
    float kexp;       // exponent k of the random-term kernel w_R = w^k
    int kgen;         // 0: k = 1 (w_R = w), 1: general k
};

// Error-free sum a + b = s + e (Knuth's TwoSum).
__device__ __forceinline__ float two_sum(float a, float b, float& e)
{
    const float s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

// 1 - r for a pair at r < 1, accurate to a few ulp of itself even near the
// cutoff: 1 - r^2 from the exact squares of the (exact) displacement
// components (fma two-products and TwoSum), then divided by 1 + r.  The
// plain 1 - r2 * rsqrt(r2) has an absolute error of ~1e-7, which a kernel
// w^k with k < 1 amplifies by k w^(k-1) near the cutoff.
__device__ __forceinline__ float one_minus_r(float dx, float dy, float dz, float r)
{
    const float p0 = dx * dx, p1 = dy * dy, p2 = dz * dz;
    const float e0 = fmaf(dx, dx, -p0), e1 = fmaf(dy, dy, -p1), e2 = fmaf(dz, dz, -p2);
    float c1, c2;
    const float s1 = two_sum(p0, p1, c1);
    const float s2 = two_sum(s1, p2, c2);
    // 1 - s2 is exact for s2 in [1/2, 1] (Sterbenz); below 1/2, w > 0.29 and
    // its rounding is already relatively small
    const float t = (1.0f - s2) - (((e0 + e1) + e2) + (c1 + c2));
    return t * __builtin_amdgcn_rcpf(1.0f + r);
}

// Scalar pair force along e_ij for r2 in (0, 1): returns F_ij / e_ij
// (the vector force is ret * d * rinv).  d = r_i - r_j, dv = v_i - v_j.
// F = a w - gamma w_R^2 (e.v) + sigma w_R xi / sqrt(dt), w = 1 - r,
// w_R = w^k (Sec. 2.1); k = 1 keeps the one-multiply form.  For general k,
// w_R = 2^(k log2 w) with the hardware log2 / exp2 on an accurate w.
__device__ __forceinline__ float pair_scalar(float r2, float dx, float dy, float dz, float dvx, float dvy,
                                             float dvz, float& rinv, float xi, const PairConst& pc)
{
    rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    const float w = 1.0f - r;
    const float ev = fmaf(dz, dvz, fmaf(dy, dvy, dx * dvx)) * rinv;   // e_ij . v_ij
    if (!pc.kgen) {
        const float inner = fmaf(pc.sig_rdt, xi, fmaf(-pc.gamma * w, ev, pc.a));
        return w * inner;
    }
    const float wa = fmaxf(one_minus_r(dx, dy, dz, r), 0.0f);   // an exact r^2 >= 1 rounded below gives 0
    const float wr = __builtin_amdgcn_exp2f(pc.kexp * __builtin_amdgcn_logf(wa));
    return fmaf(wr, fmaf(pc.sig_rdt, xi, (-pc.gamma * wr) * ev), pc.a * w);
}

__device__ __forceinline__ float dist2(float dx, float dy, float dz)
{
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// ---- cells and wave/block reductions --------------------------------------
__device__ __forceinline__ int cell_coord(float x, int L)
{
    int c = (int)x;                 // x >= 0 after the wrap: truncation is floor
    c = c < 0 ? 0 : c;
    return c > L - 1 ? L - 1 : c;
}

__device__ __forceinline__ int cell_of(float x, float y, float z, int Lx, int Ly, int Lz)
{
    return cell_coord(x, Lx) + Lx * (cell_coord(y, Ly) + Ly * cell_coord(z, Lz));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A double moved by a DPP row shift (kCtrl = row_shr:n) inside rows of 16
// lanes; lanes whose source lies outside their row get 0.
template <int kCtrl>
__device__ __forceinline__ double dpp_row_shr(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum of a double over the 64 lanes of a wave in a fixed order, with no LDS
// round trips: a tree inside each row of 16 lanes (DPP row shifts by 1, 2, 4
// and 8, which leave the row's sum in its last lane), then the four row sums
// as (r0 + r1) + (r2 + r3).  Every lane of the wave must be active; every lane
// gets the sum.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_row_shr<0x111>(v);
    v += dpp_row_shr<0x112>(v);
    v += dpp_row_shr<0x114>(v);
    v += dpp_row_shr<0x118>(v);
    return (readlane_f64(v, 15) + readlane_f64(v, 31)) + (readlane_f64(v, 47) + readlane_f64(v, 63));
}

// Block-wide sum in a fixed order (lane tree inside each wave, then waves in
// index order).  All threads of the block must call it.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch /* >= blockDim/64 */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    T t = T(0);
    for (int w = 0; w < nw; ++w) t += scratch[w];
    return t;
}

// Inclusive scan inside a wave of 64.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan of a[0..n) in place (LDS), a[n] = total; returns the total.
// scr needs blockDim/64 ints.  All threads of the block must call it.
__device__ __forceinline__ int block_excl_scan(int* a, int n, int* scr)
{
    const int bd = blockDim.x, tid = threadIdx.x;
    const int per = (n + bd - 1) / bd;
    const int b0 = tid * per;
    int sum = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < n) sum += a[b0 + k];
    const int lane = tid & 63, wave = tid >> 6;
    const int incl = wave_incl_scan(sum);
    __syncthreads();
    if (lane == 63) scr[wave] = incl;
    __syncthreads();
    int wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += scr[w];
    int run = wpre + incl - sum;
    for (int k = 0; k < per; ++k)
        if (b0 + k < n) {
            const int v = a[b0 + k];
            a[b0 + k] = run;
            run += v;
        }
    if (tid == bd - 1) a[n] = run;
    __syncthreads();
    return a[n];
}

}  // namespace dpd
