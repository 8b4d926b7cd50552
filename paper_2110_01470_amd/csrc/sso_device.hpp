// Device building blocks shared by the SSO kernels (gfx950, wave64).
//
// Counter-based random words, the interval rule of Eq. (2.1), the FP32
// objective terms and the orderable (fitness, index) key that turns the gBest
// search of Algorithm 4 into one 64-bit atomicMin.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sso_layout.hpp"

namespace sso {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key lives in scalar
// registers (it is a kernel argument); the counter is (chunk, particle,
// generation, swarm), so generation and swarm are wave-uniform and the first
// round's second product is a scalar multiply.
// ---------------------------------------------------------------------------

// a ^ b ^ k in one VALU instruction (gfx950's three-input bitwise op; 0x96 is
// the truth table of the three-way parity, whatever the operand order).  k
// must be wave-uniform: it is read from a scalar register.
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        if (r < 2) {
            // Rounds 1 and 2 xor wave-uniform words (generation, swarm, the
            // low half of a uniform product), which the compiler folds into
            // the key with scalar instructions.
            c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                           (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        } else {
            c = make_uint4(xor3_vvs((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                           xor3_vvs((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
        }
    }
    return c;
}

// Words of variables 4q .. 4q+3 of particle i at generation t.
__device__ __forceinline__ uint4 words4(const SwarmDev &S, uint32_t q, uint32_t i, uint32_t t)
{
    return philox4x32_10(make_uint4(q, i, t, S.swarm), S.key0, S.key1);
}

// Native 4-vector: arrays of these stay in registers (HIP's float4 struct
// arrays do not always).
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Eq. (2.1).  Word k stands for rand() = k 2^-32; thresholds are
// ceil(c 2^32), so the interval test is an exact integer compare.  A fresh
// value reuses the word: (k - th2) is uniform on [0, 2^32 - th2) and
// mulhi(k - th2, r), r = floor(2^56 / (2^32 - th2)), rescales it to 24 bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float draw24(const SwarmDev &S, uint32_t u24)
{
    // lo + u24 * (span 2^-24) with one rounding: u24 < 2^24 converts exactly
    // (as a signed int, which gives a single conversion instruction) and the
    // fma forms the product exactly before rounding.
    return __builtin_fmaf((float)(int32_t)u24, S.span24, S.lo);
}

__device__ __forceinline__ float init_value(const SwarmDev &S, uint32_t k)
{
    return draw24(S, k >> 8);
}

__device__ __forceinline__ f4 init4(const SwarmDev &S, uint4 k)
{
    return f4{init_value(S, k.x), init_value(S, k.y), init_value(S, k.z), init_value(S, k.w)};
}

template <bool EQ21>
__device__ __forceinline__ float select_one(const SwarmDev &S, uint32_t k, float g, float p,
                                            float x)
{
    // Interval sources: GPS order (g, p, self, fresh); Eq. (2.1) order
    // (self, p, g, fresh).
    const float first = EQ21 ? x : g;
    const float third = EQ21 ? g : x;
    float v = draw24(S, __umulhi(k - S.th2, S.r));
    v = (k < S.th2) ? third : v;
    v = (k < S.th1) ? p : v;
    v = (k < S.th0) ? first : v;
    return v;
}

template <bool EQ21>
__device__ __forceinline__ f4 select4(const SwarmDev &S, uint4 k, f4 g, f4 p, f4 x)
{
    return f4{select_one<EQ21>(S, k.x, g.x, p.x, x.x), select_one<EQ21>(S, k.y, g.y, p.y, x.y),
              select_one<EQ21>(S, k.z, g.z, p.z, x.z), select_one<EQ21>(S, k.w, g.w, p.w, x.w)};
}

// ---------------------------------------------------------------------------
// Row storage policies for the generation kernels (see sso_layout.hpp).
// T is the in-register form of one chunk of 4 variables; value() gives the
// FP32 positions the objective is evaluated on.
// ---------------------------------------------------------------------------
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

struct U24x4 {
    uint32_t w0, w1, w2;
};

struct StoreF32 {
    using T = f4;
    static constexpr bool kPacked = false;
    using R = f4;
    __device__ static R load_raw(const uint32_t *row, uint32_t c) { return reinterpret_cast<const f4 *>(row)[c]; }
    __device__ static T unpack(R v) { return v; }
    __device__ static T load(const uint32_t *row, uint32_t c) { return load_raw(row, c); }
    __device__ static void store(uint32_t *row, uint32_t c, T v) { reinterpret_cast<f4 *>(row)[c] = v; }
    __device__ static T init(const SwarmDev &S, uint4 k) { return init4(S, k); }
    template <bool EQ21>
    __device__ static T select(const SwarmDev &S, uint4 k, T g, T p, T x)
    {
        return select4<EQ21>(S, k, g, p, x);
    }
    __device__ static f4 value(const SwarmDev &, T v) { return v; }
};

template <bool EQ21>
__device__ __forceinline__ uint32_t select_u(const SwarmDev &S, uint32_t k, uint32_t g, uint32_t p,
                                             uint32_t x)
{
    const uint32_t first = EQ21 ? x : g;
    const uint32_t third = EQ21 ? g : x;
    uint32_t v = __umulhi(k - S.th2, S.r);  // fresh grid index
    v = (k < S.th2) ? third : v;
    v = (k < S.th1) ? p : v;
    v = (k < S.th0) ? first : v;
    return v;
}

struct StoreU24 {
    using T = u4v;
    static constexpr bool kPacked = true;
    // R is the chunk as stored (loaded early, unpacked when used).
    using R = U24x4;
    __device__ static R load_raw(const uint32_t *row, uint32_t c) { return reinterpret_cast<const U24x4 *>(row)[c]; }
    __device__ static T unpack(R q)
    {
        return T{q.w0 & 0xFFFFFFu, __builtin_amdgcn_alignbit(q.w1, q.w0, 24) & 0xFFFFFFu,
                 __builtin_amdgcn_alignbit(q.w2, q.w1, 16) & 0xFFFFFFu, q.w2 >> 8};
    }
    __device__ static T load(const uint32_t *row, uint32_t c) { return unpack(load_raw(row, c)); }
    __device__ static void store(uint32_t *row, uint32_t c, T u)
    {
        reinterpret_cast<U24x4 *>(row)[c] =
            U24x4{u.x | (u.y << 24), (u.y >> 8) | (u.z << 16), (u.z >> 16) | (u.w << 8)};
    }
    __device__ static T init(const SwarmDev &, uint4 k)
    {
        return T{k.x >> 8, k.y >> 8, k.z >> 8, k.w >> 8};
    }
    template <bool EQ21>
    __device__ static T select(const SwarmDev &S, uint4 k, T g, T p, T x)
    {
        return T{select_u<EQ21>(S, k.x, g.x, p.x, x.x), select_u<EQ21>(S, k.y, g.y, p.y, x.y),
                 select_u<EQ21>(S, k.z, g.z, p.z, x.z), select_u<EQ21>(S, k.w, g.w, p.w, x.w)};
    }
    __device__ static f4 value(const SwarmDev &S, T u)
    {
        return f4{draw24(S, u.x), draw24(S, u.y), draw24(S, u.z), draw24(S, u.w)};
    }
};

// ---------------------------------------------------------------------------
// Separable objectives: FP32 terms of four variables starting at column j0;
// columns >= d are padding and contribute nothing.
//
// sin(3u) is taken in revolutions: r = u * 3/(2 pi), reduced exactly to
// [-1/2, 1/2] by r - rint(r), then the hardware sine of 2 pi r.  Measured on
// gfx950 against FP64 sin this is within 1.9e-5 absolute for |3u| <= 460 and
// 1e-6 relative for small arguments; both are below 1e-6 of the term
// w u^2 + sin^2(3u)/2 it feeds (w >= 1), whatever u is.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ float term1(float x, float s, float w)
{
    const float u = x - s;
    if constexpr (KIND == OBJ_SPHERE) {
        return u * u;
    } else {
        const float r = u * 0.477464829275686f;  // 3 / (2 pi)
        const float sn = __builtin_amdgcn_sinf(r - __builtin_rintf(r));
        return w * (u * u) + 0.5f * (sn * sn);
    }
}

template <int KIND>
__device__ __forceinline__ float terms4(f4 x, f4 s, f4 w, uint32_t j0, uint32_t d)
{
    float t0 = term1<KIND>(x.x, s.x, w.x);
    float t1 = term1<KIND>(x.y, s.y, w.y);
    float t2 = term1<KIND>(x.z, s.z, w.z);
    float t3 = term1<KIND>(x.w, s.w, w.w);
    t0 = (j0 + 0 < d) ? t0 : 0.0f;
    t1 = (j0 + 1 < d) ? t1 : 0.0f;
    t2 = (j0 + 2 < d) ? t2 : 0.0f;
    t3 = (j0 + 3 < d) ? t3 : 0.0f;
    return (t0 + t1) + (t2 + t3);
}

// All four columns real (d is a multiple of 4): no padding masks.
template <int KIND>
__device__ __forceinline__ float terms4_full(f4 x, f4 s, f4 w)
{
    const float t0 = term1<KIND>(x.x, s.x, w.x);
    const float t1 = term1<KIND>(x.y, s.y, w.y);
    const float t2 = term1<KIND>(x.z, s.z, w.z);
    const float t3 = term1<KIND>(x.w, s.w, w.w);
    return (t0 + t1) + (t2 + t3);
}

// ---------------------------------------------------------------------------
// Table 3.2's benchmark functions, unshifted, over the d variables of a
// particle (F3, F5, F6 and F8 in the textbook forms the garbled entries name:
// the running sums of Schwefel 1.2, Rastrigin's cosine, Ackley with
// a = 20, b = 0.2, c = 2 pi and + a + e, Powell's four terms per group of
// four).  A particle's L lanes accumulate their chunks into PaperAcc; F3 needs
// running sums across the lanes (a scan of chunk totals plus a carry from
// the previous pass) and F4 the last variable of the previous chunk (the
// lane below, or for lane 0 the carry from the previous pass).  All lanes of
// a particle call paper_chunk together for the chunks c = c0 + ln of one
// pass; a lane whose chunk does not exist has left the loop, and its values
// are never needed.
// ---------------------------------------------------------------------------
struct PaperAcc {
    float a = 0.0f, b = 0.0f, p = 1.0f, carry = 0.0f;
};

// The functions below keep every product and sum a separate rounding (no
// fused multiply-add contraction), so the value does not depend on how the
// compiler schedules them in a given kernel: the STREAM and RESIDENT kernels
// evaluate them identically.
__device__ __forceinline__ float rosen_pair(float xi, float xn)
{
#pragma clang fp contract(off)
    const float q = xn - xi * xi, r = 1.0f - xi;
    return 100.0f * (q * q) + r * r;
}

__device__ __forceinline__ void paper_chunk(PaperAcc &q, f4 x, uint32_t c, uint32_t d, uint32_t L,
                                            uint32_t ln, int kind)
{
#pragma clang fp contract(off)
    const uint32_t j0 = 4u * c;
    const float v[4] = {x.x, x.y, x.z, x.w};
    switch (kind) {
    case OBJ_F1 + 0:  // sphere
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) q.a += v[e] * v[e];
        break;
    case OBJ_F1 + 1:  // hyper-ellipsoid: the square of variable j weighs j + 1
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) q.a += (float)(j0 + e + 1) * (v[e] * v[e]);
        break;
    case OBJ_F1 + 2: {  // Schwefel 1.2: squares of the running sums
        float pre[4], r = 0.0f;
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e) {
            r += (j0 + e < d) ? v[e] : 0.0f;
            pre[e] = r;
        }
        float incl = r;  // inclusive scan of the chunk totals over the lanes
        for (uint32_t off = 1; off < L; off <<= 1) {
            const float u = __shfl_up(incl, off, L);
            if (ln >= off) incl += u;
        }
        // Shuffles run in every lane before any select: a lane whose
        // execution bit is off does not supply its value to a permute, so a
        // shuffle inside the ln != 0 branch would read nothing from lane 0.
        const float up1 = __shfl_up(incl, 1, L);
        const float excl = ln ? up1 : 0.0f;
        const float base = q.carry + excl;
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) {
                const float run = base + pre[e];
                q.a += run * run;
            }
        q.carry += __shfl(incl, L - 1, L);
        break;
    }
    case OBJ_F1 + 3: {  // Rosenbrock: pairs (x_j, x_{j+1})
#pragma unroll
        for (uint32_t e = 0; e < 3; ++e)
            if (j0 + e + 1 < d) q.a += rosen_pair(v[e], v[e + 1]);
        // The pair that straddles chunks c-1 and c belongs to chunk c.  The
        // lane below (a DPP shift of the whole wave by one lane) is active
        // whenever this lane is; lane 0 of a particle ignores what it gets.
        const float below = __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(v[3]), 0x138, 0xF, 0xF, false));  // wave_shr:1
        const float prev = ln ? below : q.carry;
        if (c > 0 && j0 < d) q.a += rosen_pair(prev, v[0]);
        q.carry = __shfl(v[3], L - 1, L);
        break;
    }
    case OBJ_F1 + 4:  // Rastrigin (10 d is added at the end)
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) q.a += v[e] * v[e] - 10.0f * cospif(2.0f * v[e]);
        break;
    case OBJ_F1 + 5:  // Ackley: sum of squares, sum of cos(2 pi x)
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) {
                q.a += v[e] * v[e];
                q.b += cospif(2.0f * v[e]);
            }
        break;
    case OBJ_F1 + 6:  // Griewank: sum of squares, product of cos(x_j / sqrt(j + 1))
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) {
                q.a += v[e] * v[e];
                q.p *= cosf(v[e] / sqrtf((float)(j0 + e + 1)));
            }
        break;
    case OBJ_F1 + 7:  // Powell: chunk c is group c; only whole groups count
        if (j0 + 3 < d) {
            const float a1 = v[0] + 10.0f * v[1], a2 = v[2] - v[3];
            const float a3 = v[1] - 2.0f * v[2], a4 = v[0] - v[3];
            const float a3s = a3 * a3, a4s = a4 * a4;
            q.a += a1 * a1 + 5.0f * (a2 * a2) + a3s * a3s + 10.0f * (a4s * a4s);
        }
        break;
    default:  // F9, Schwefel 2.26: 418.9829 d is added at the end
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
            if (j0 + e < d) q.a += v[e] * sinf(sqrtf(fabsf(v[e])));
        break;
    }
}

// The particle's value from its lanes' accumulators (a butterfly over the
// L lanes, then the function's outer terms).
__device__ __forceinline__ float paper_finish(PaperAcc q, uint32_t L, uint32_t d, int kind)
{
#pragma clang fp contract(off)
    // Only Ackley uses the second sum and only Griewank the product; the
    // others skip their (unused) reductions.
    const bool need_b = kind == OBJ_F1 + 5, need_p = kind == OBJ_F1 + 6;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        if ((uint32_t)m < L) {
            q.a += __shfl_xor(q.a, m, 64);
            if (need_b) q.b += __shfl_xor(q.b, m, 64);
            if (need_p) q.p *= __shfl_xor(q.p, m, 64);
        }
    const float P = (float)d;
    switch (kind) {
    case OBJ_F1 + 4: return 10.0f * P + q.a;
    case OBJ_F1 + 5:
        return -20.0f * expf(-0.2f * sqrtf(q.a / P)) - expf(q.b / P) + 20.0f + 2.718281828459045f;
    case OBJ_F1 + 6: return q.a / 4000.0f - q.p + 1.0f;
    case OBJ_F1 + 8: return 418.9829f * P - q.a;
    default: return q.a;
    }
}

// ---------------------------------------------------------------------------
// gBest key: (orderable FP32 bits << 32) | (particle << 1) | pBest row.
// Smaller fitness wins; equal fitness goes to the lower particle index; NaN
// sorts above every number; -0 and +0 are the same.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t orderable(float f)
{
    uint32_t b = __float_as_uint(f);
    if (f != f) return 0xFFFFFFFFu;
    if (f == 0.0f) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Algorithm 3's strict improvement in the same order as the gBest key: NaN
// sorts above every number, so a NaN pBest fitness is replaced by any number
// and a NaN fitness never replaces a pBest; -0 and +0 are equal.
__device__ __forceinline__ bool improves(float f, float fp)
{
    return f < fp || (fp != fp && f == f);
}

__device__ __forceinline__ unsigned long long gbest_key(float f, uint32_t i, uint32_t row)
{
    return ((unsigned long long)orderable(f) << 32) | ((unsigned long long)i << 1) | row;
}

__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b)
{
    return a < b ? a : b;
}

// min(x, x of the lane the DPP control CTRL names), both halves moved by the
// same row-local pattern.  A lane whose source is off keeps its own value.
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_min_u64(unsigned long long x)
{
    const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
    const uint32_t plo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const uint32_t phi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return min_u64(x, ((unsigned long long)phi << 32) | plo);
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

// Minimum of x over the 64 lanes of the wave, the same value in every lane;
// called with every lane of the wave active.  A minimum does not depend on
// the order it is taken in, so this is the shuffle butterfly's result with
// row-local DPP moves (pairs, quads, half rows, rows of 16) instead of LDS
// permutes, and the four row minima read out as wave-uniform values.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x)
{
    x = dpp_min_u64<0xB1>(x);   // quad_perm(1, 0, 3, 2)
    x = dpp_min_u64<0x4E>(x);   // quad_perm(2, 3, 0, 1)
    x = dpp_min_u64<0x141>(x);  // row_half_mirror
    x = dpp_min_u64<0x140>(x);  // row_mirror
    return min_u64(min_u64(readlane_u64(x, 0), readlane_u64(x, 16)),
                   min_u64(readlane_u64(x, 32), readlane_u64(x, 48)));
}

__device__ __forceinline__ unsigned long long *sub_key(const SwarmDev &S, uint32_t group,
                                                       uint32_t j)
{
    return S.sub + ((size_t)group * kSubSlots + j) * kSubStride;
}

__device__ __forceinline__ uint32_t *sub_cnt(const SwarmDev &S, uint32_t group, uint32_t j)
{
    return reinterpret_cast<uint32_t *>(sub_key(S, group, j) + 1);
}

// The gBest key of generation t - 1 as lane l of wave 0 holds it before the
// reduction: sub-slot l of group (t - 1) mod 3 (all ones for unused lanes
// and other waves).  A separate call so that a kernel can issue this load
// ahead of its other loads: it heads the longest dependent chain of a
// generation (key, then gBest row, then the first select).
__device__ __forceinline__ unsigned long long generation_key_load(const SwarmDev &S, uint32_t t)
{
    const uint32_t lane = threadIdx.x & 63u;
    return (threadIdx.x < 64u && lane < S.nsub) ? *sub_key(S, (t - 1u) % kGroups, lane) : ~0ull;
}

// Start of generation t >= 1 (all threads of the workgroup call it; it holds
// one barrier).  Wave 0 reduces the sub-slots of generation t - 1 (k from
// generation_key_load; nsub <= 64) and shares the gBest key through LDS.
// Workgroup 0 of the swarm (blk == 0) also records that key and the
// improvement count in the trace ring and clears the group generation t + 1
// will commit into.
__device__ __forceinline__ unsigned long long generation_begin(const SwarmDev &S, uint32_t t,
                                                               uint32_t blk,
                                                               unsigned long long k)
{
    __shared__ unsigned long long s_best;
    const uint32_t lane = threadIdx.x & 63u;
    if (threadIdx.x < 64u) {
        const uint32_t g = (t - 1u) % kGroups;
        const bool used = lane < S.nsub;
        k = wave_min_u64(k);
        if (lane == 0) s_best = k;
        if (blk == 0) {
            uint32_t c = used ? *sub_cnt(S, g, lane) : 0u;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
            if (lane == 0) {
                S.keys[(t - 1u) % S.trace_cap] = k;
                S.cnt[(t - 1u) % S.trace_cap] = c;
            }
            const uint32_t gn = (t + 1u) % kGroups;
            if (used) {
                *sub_key(S, gn, lane) = ~0ull;
                *sub_cnt(S, gn, lane) = 0u;
            }
        }
    }
    __syncthreads();
    return s_best;
}

__device__ __forceinline__ unsigned long long generation_begin(const SwarmDev &S, uint32_t t,
                                                               uint32_t blk)
{
    return generation_begin(S, t, blk, generation_key_load(S, t));
}

// End of generation t for one wave (no barrier): the wave's minimum key and
// improvement count folded into sub-slot (wave_id mod nsub) of group t % 3.
__device__ __forceinline__ void wave_commit(const SwarmDev &S, uint32_t t, uint32_t wave_id,
                                            unsigned long long key, uint32_t improved)
{
    key = wave_min_u64(key);
    const uint32_t cnt = (uint32_t)__popcll(__ballot(improved != 0u));
    if ((threadIdx.x & 63u) == 0u) {
        const uint32_t g = t % kGroups, j = wave_id & (S.nsub - 1u);
        if (key != ~0ull) atomicMin(sub_key(S, g, j), key);
        if (cnt) atomicAdd(sub_cnt(S, g, j), cnt);
    }
}

// End of generation t: minimum key and improvement count over the workgroup's
// NW waves, folded into sub-slot (blk mod nsub) of group t % 3 with one atomic
// each (thread 0).
template <int NW>
__device__ __forceinline__ void generation_commit(const SwarmDev &S, uint32_t t, uint32_t blk,
                                                  unsigned long long key, uint32_t improved)
{
    __shared__ unsigned long long s_key[NW];
    __shared__ uint32_t s_cnt[NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    key = wave_min_u64(key);
    const uint32_t cnt = (uint32_t)__popcll(__ballot(improved != 0u));
    if (lane == 0) {
        s_key[wave] = key;
        s_cnt[wave] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = s_key[0];
        uint32_t c = s_cnt[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            k = min_u64(k, s_key[w]);
            c += s_cnt[w];
        }
        const uint32_t g = t % kGroups, j = blk & (S.nsub - 1u);
        if (k != ~0ull) atomicMin(sub_key(S, g, j), k);
        if (c) atomicAdd(sub_cnt(S, g, j), c);
    }
}

}  // namespace sso
