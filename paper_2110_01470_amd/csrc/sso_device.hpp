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
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    }
    return c;
}

// Words of variables 4q .. 4q+3 of particle i at generation t.
__device__ __forceinline__ uint4 words4(const SwarmDev &S, uint32_t q, uint32_t i, uint32_t t)
{
    return philox4x32_10(make_uint4(q, i, t, S.swarm), S.key0, S.key1);
}

// ---------------------------------------------------------------------------
// Eq. (2.1).  Word k stands for rand() = k 2^-32; thresholds are
// ceil(c 2^32), so the interval test is an exact integer compare.  A fresh
// value reuses the word: (k - th2) is uniform on [0, 2^32 - th2) and
// mulhi(k - th2, r), r = floor(2^56 / (2^32 - th2)), rescales it to 24 bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float draw24(const SwarmDev &S, uint32_t u24)
{
    // u24 * 2^-24 is exact; the fma rounds once.
    return __builtin_fmaf((float)u24 * 0x1p-24f, S.span, S.lo);
}

__device__ __forceinline__ float init_value(const SwarmDev &S, uint32_t k)
{
    return draw24(S, k >> 8);
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
__device__ __forceinline__ float4 select4(const SwarmDev &S, uint4 k, float4 g, float4 p,
                                          float4 x)
{
    return make_float4(select_one<EQ21>(S, k.x, g.x, p.x, x.x),
                       select_one<EQ21>(S, k.y, g.y, p.y, x.y),
                       select_one<EQ21>(S, k.z, g.z, p.z, x.z),
                       select_one<EQ21>(S, k.w, g.w, p.w, x.w));
}

// ---------------------------------------------------------------------------
// Separable objectives: FP32 terms of four variables starting at column j0;
// columns >= d are padding and contribute nothing.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ float term1(float x, float s, float w)
{
    const float u = x - s;
    if constexpr (KIND == OBJ_SPHERE) {
        return u * u;
    } else {
        const float sn = sinf(3.0f * u);
        return w * (u * u) + 0.5f * (sn * sn);
    }
}

template <int KIND>
__device__ __forceinline__ float terms4(float4 x, float4 s, float4 w, uint32_t j0, uint32_t d)
{
    float acc = 0.0f;
    acc += (j0 + 0 < d) ? term1<KIND>(x.x, s.x, w.x) : 0.0f;
    acc += (j0 + 1 < d) ? term1<KIND>(x.y, s.y, w.y) : 0.0f;
    acc += (j0 + 2 < d) ? term1<KIND>(x.z, s.z, w.z) : 0.0f;
    acc += (j0 + 3 < d) ? term1<KIND>(x.w, s.w, w.w) : 0.0f;
    return acc;
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

__device__ __forceinline__ unsigned long long gbest_key(float f, uint32_t i, uint32_t row)
{
    return ((unsigned long long)orderable(f) << 32) | ((unsigned long long)i << 1) | row;
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b)
{
    return a < b ? a : b;
}

// Minimum key and improvement count over one workgroup of NW waves, folded
// into the generation's trace slot with one atomic each (thread 0).
template <int NW>
__device__ __forceinline__ void workgroup_commit(unsigned long long key, uint32_t improved,
                                                 unsigned long long *slot_key,
                                                 uint32_t *slot_cnt)
{
    __shared__ unsigned long long s_key[NW];
    __shared__ uint32_t s_cnt[NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) key = min_u64(key, shfl_xor_u64(key, m));
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
        atomicMin(slot_key, k);
        if (c) atomicAdd(slot_cnt, c);
    }
}

}  // namespace sso
