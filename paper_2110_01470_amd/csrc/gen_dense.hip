// Dense objective f(x) = ||A (x - s)||^2: one fused kernel per generation
// with the contraction on FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Work split: a workgroup of eight waves owns 64 particles in four groups
// of 16.  The two waves of a group split the inner index: wave half h
// selects (Eq. 2.1) and contracts the variables of K-chunks
// [h NB/2, (h+1) NB/2), each K-chunk being 16 variables.  Per wave the kernel
// forms a partial Y^T = A[:, its chunks] * D^T[its chunks, :] (rows: output
// index k of A, columns: the group's 16 particles), where D = X' - s comes
// straight out of the select of the same generation.  At the end the upper
// half adds its partial Y^T into the lower half's through LDS, and the
// fitness of particle p is the sum over k of Y^T[k][p]^2.  Two waves per
// SIMD let one wave's select (VALU, memory) run under the other's MFMAs.
//
// MFMA operand layout (16x16x4, one block): lane l supplies A-operand
// element (row l%16, inner l/16) and B-operand element (inner l/16,
// column l%16); the 16x16 result leaves rows 4(l/16)+r, column l%16 in
// accumulator register r.  The inner index is free to permute, so MFMA step
// m = 4M + e pairs lane group g = l/16 with variable 16M + 4g + e.  Then:
//   * the B operands of four consecutive steps are one float4 of the
//     particle's row (chunk 4M + g), loaded, selected and written by the
//     lane that consumes it -- the select needs no shuffle;
//   * the A operands are one float4 per lane and row block; the host packs A
//     as [M][row block][lane][4] so that K-chunk M is one contiguous block
//     that the workgroup copies into LDS and each wave reads conflict-free.
// The two K-chunks of a step (one per half) are double-buffered in LDS and
// copied there by global-to-LDS loads (no registers in between); the next
// step's copy and the next select's row loads are issued before the current
// step's MFMAs, which read their A operands from LDS four row blocks at a
// time.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sso_device.hpp"

namespace sso {

typedef f4 floatx4;

constexpr int kDenseWaves = 8;
constexpr int kDenseBlock = 64 * kDenseWaves;

uint64_t dense_matrix_floats(uint32_t d)
{
    const uint64_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    return dp * dp;
}

// Host: a[k*d + j] (row-major d x d) -> packed[M][rb][lane][e] =
// A[16 rb + lane%16][16 M + 4 (lane/16) + e], zero outside d x d.
void dense_pack_matrix(const float *a, uint32_t d, float *out)
{
    const uint32_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    const uint32_t nb = dp / 16;
    size_t o = 0;
    for (uint32_t M = 0; M < nb; ++M)
        for (uint32_t rb = 0; rb < nb; ++rb)
            for (uint32_t lane = 0; lane < 64; ++lane)
                for (uint32_t e = 0; e < 4; ++e) {
                    const uint32_t k = 16 * rb + lane % 16;
                    const uint32_t j = 16 * M + 4 * (lane / 16) + e;
                    out[o++] = (k < d && j < d) ? a[(size_t)k * d + j] : 0.0f;
                }
}

// NB = dp / 16: row blocks of A, and K-chunks of 16 variables (NB is even).
// FULL_D: d = dp, so every chunk is whole and inside the row (no masks).
template <int NB, bool EQ21, bool INIT, bool FULL_D>
__global__ __launch_bounds__(kDenseBlock) void k_dense(SwarmDev S, uint32_t t)
{
    constexpr uint32_t HALF = NB / 2;                               // K-chunks per wave
    constexpr uint32_t CF4 = NB * 64u;                              // float4 per K-chunk
    constexpr uint32_t STEP_F4 = 2 * CF4;                           // both halves' chunks
    constexpr uint32_t PER = (STEP_F4 + kDenseBlock - 1) / kDenseBlock;
    constexpr bool FULL = STEP_F4 % kDenseBlock == 0;
    // Two step buffers, as two variables: the compiler then tells the LDS
    // reads of one from the copies in flight into the other, and does not
    // wait for those copies before the reads.  After the loop the buffers
    // carry the upper halves' partial accumulators (groups 0-1 in the first,
    // 2-3 in the second; NB x 64 lanes x 4 floats each).
    static_assert(STEP_F4 == 2 * NB * 64, "a buffer holds two groups' partial accumulators");
    __shared__ f4 lds0[STEP_F4];
    __shared__ f4 lds1[STEP_F4];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t grp4 = wave & 3u, half = wave >> 2;   // particle group, K half
    const uint32_t pcol = lane & 15u, lg = lane >> 4;
    const uint32_t i = blockIdx.x * 64u + grp4 * 16u + pcol;
    const bool valid = i < S.n;
    const f4 *a_pack = reinterpret_cast<const f4 *>(S.a);

    // The gBest key load goes out first (see generation_key_load).
    unsigned long long gkey = ~0ull;
    if constexpr (!INIT) gkey = generation_key_load(S, t);

    // The state word and pBest fitness; the state is decoded only after the
    // first row loads below have gone out, which do not depend on it.
    uint32_t st = ST_ALIAS;  // pBest in row 0, position aliased (generation 0)
    float fpi = 0.0f;
    if (!INIT && valid) {
        st = S.st[i];
        fpi = S.fp[i];
    }
    const size_t ioff = (size_t)(valid ? i : 0u) * S.stride;
    const f4 *s4 = reinterpret_cast<const f4 *>(S.s);

    // Step m stages K-chunk m (lower half) and K-chunk HALF + m (upper half).
    auto stage_addr = [&](uint32_t m, uint32_t q) -> size_t {
        return (size_t)(q < CF4 ? m : HALF + m) * CF4 + (q % CF4);
    };
    // Step m's two K-chunks straight from global memory into LDS buffer b:
    // each wave moves 64 consecutive float4 (no registers in between).
    auto stage_dma = [&](uint32_t m, uint32_t b) {
#pragma unroll
        for (uint32_t r = 0; r < PER; ++r) {
            const uint32_t q = tid + r * kDenseBlock;
            if (FULL || q < STEP_F4)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(a_pack + stage_addr(m, q)),
                    (__attribute__((address_space(3))) void *)(&(b ? lds1 : lds0)[r * kDenseBlock + wave * 64u]), 16, 0, 0);
        }
    };
    // Loads that do not depend on gBest go out before the start-of-generation
    // barrier: this lane's first pBest, position and shift.  The first A step
    // follows the gBest reduction (at generation 0 there is none): copies into
    // LDS still in flight would hold up its shuffles and barrier.
    if constexpr (INIT) stage_dma(0, 0);
    const uint32_t cbase = 4u * HALF * half;  // first chunk of this wave's half
    const f4 zero4 = f4{0.f, 0.f, 0.f, 0.f};
    f4 pv = zero4, xv = zero4, gv = zero4, sv = zero4;
    // The first chunk is read from both rows at once, without waiting for
    // the state word that says which row is the pBest (the same two loads).
    f4 row0 = zero4, row1 = zero4;
    if (valid && cbase + lg < S.chunks) {
        sv = s4[cbase + lg];
        if constexpr (!INIT) {
            row0 = reinterpret_cast<const f4 *>(S.rows + ioff)[cbase + lg];
            row1 = reinterpret_cast<const f4 *>(S.rows + S.buf + ioff)[cbase + lg];
        }
    }

    // The first step's random words while those loads are in flight (the
    // empty asm keeps them from being computed after the waits below).
    uint4 k_first = words4(S, cbase + lg, i, t);
    asm volatile("" : "+v"(k_first.x), "+v"(k_first.y), "+v"(k_first.z), "+v"(k_first.w));

    const uint32_t prow = st & ST_ROW;
    const bool alias = (st & ST_ALIAS) != 0u;
    const f4 *p4 = reinterpret_cast<const f4 *>(S.rows + prow * S.buf + ioff);
    f4 *x4 = reinterpret_cast<f4 *>(S.rows + (INIT ? 0u : (1u - prow)) * S.buf + ioff);
    // Where the position is read from: the pBest row itself when aliased.
    const f4 *xsrc = alias ? p4 : x4;
    pv = prow ? row1 : row0;
    xv = alias ? pv : (prow ? row0 : row1);

    const f4 *g4 = reinterpret_cast<const f4 *>(S.rows);
    if constexpr (!INIT) {
        const uint32_t glow = (uint32_t)generation_begin(S, t, blockIdx.x, gkey);
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        g4 = reinterpret_cast<const f4 *>(S.rows + (size_t)(glow & 1u) * S.buf + (size_t)gidx * S.stride);
        stage_dma(0, 0);
        if (valid && cbase + lg < S.chunks) gv = g4[cbase + lg];
    }
    auto prefetch = [&](uint32_t c) {
        if (valid && (FULL_D || c < S.chunks)) {
            sv = s4[c];
            if constexpr (!INIT) {
                pv = p4[c];
                xv = xsrc[c];
                gv = g4[c];
            }
        }
    };
    __builtin_amdgcn_s_waitcnt(0);  // this wave's DMA into buffer 0 has landed

    f4 acc[NB];
#pragma unroll
    for (uint32_t rb = 0; rb < NB; ++rb) acc[rb] = zero4;

    __syncthreads();

    // Per step: select from operands fetched one step earlier, then issue the
    // next step's row and A loads, then the MFMAs; the only wait on global
    // memory is before the staging write at the end of the step.
#pragma unroll
    for (uint32_t m = 0; m < HALF; ++m) {
        const uint32_t cur = m & 1u;
        const bool more = m + 1 < HALF;
        // Select this lane's chunk c of Eq. (2.1) and form d = x' - s.
        const uint32_t c = cbase + 4u * m + lg;
        f4 dv = zero4;
        if (valid && (FULL_D || c < S.chunks)) {
            const uint4 k = m == 0 ? k_first : words4(S, c, i, t);
            f4 xn;
            if constexpr (INIT)
                xn = init4(S, k);
            else
                xn = select4<EQ21>(S, k, gv, pv, xv);
            x4[c] = xn;
            if constexpr (FULL_D) {
                dv = xn - sv;
            } else {
                const uint32_t j0 = 4u * c;
                dv.x = (j0 + 0 < S.d) ? xn.x - sv.x : 0.f;
                dv.y = (j0 + 1 < S.d) ? xn.y - sv.y : 0.f;
                dv.z = (j0 + 2 < S.d) ? xn.z - sv.z : 0.f;
                dv.w = (j0 + 3 < S.d) ? xn.w - sv.w : 0.f;
            }
        }
        if (more) {
            prefetch(c + 4u);
            stage_dma(m + 1, cur ^ 1u);
        }
        // Keep the copies and loads above ahead of the MFMAs below, so that
        // their latency runs under the MFMAs rather than before the barrier.
        __builtin_amdgcn_sched_barrier(0);
        const f4 *la = (cur ? lds1 : lds0) + half * CF4;
#pragma unroll
        for (uint32_t r0 = 0; r0 < NB; r0 += 4) {
            f4 a4[4];
#pragma unroll
            for (uint32_t q = 0; q < 4 && r0 + q < NB; ++q) a4[q] = la[(r0 + q) * 64u + lane];
#pragma unroll
            for (uint32_t e = 0; e < 4; ++e)
#pragma unroll
                for (uint32_t q = 0; q < 4 && r0 + q < NB; ++q)
                    acc[r0 + q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[q][e], dv[e], acc[r0 + q], 0, 0, 0);
        }
        if (more) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's DMA for the next step has landed
        }
        __syncthreads();
    }

    // The upper half hands its partial Y^T to the lower half through LDS
    // (the staging buffers are free after the loop's last barrier).
    f4 *red = (grp4 < 2 ? lds0 : lds1) + (grp4 & 1u) * NB * 64u;
    if (half == 1) {
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb) red[rb * 64u + lane] = acc[rb];
    }
    __syncthreads();

    // f = sum_k y_k^2: this lane holds rows 4 lg + r of every row block.
    float f = 0.0f;
    if (half == 0) {
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb) {
            const f4 y = acc[rb] + red[rb * 64u + lane];
            f += y[0] * y[0];
            f += y[1] * y[1];
            f += y[2] * y[2];
            f += y[3] * y[3];
        }
    }
    f += __shfl_xor(f, 16, 64);
    f += __shfl_xor(f, 32, 64);

    const bool owner = half == 0 && valid;
    const bool improved = owner && (INIT || improves(f, fpi));
    uint32_t row = prow;
    float fnew = fpi;
    if (improved) {
        row = INIT ? 0u : 1u - prow;
        fnew = f;
    }
    if (owner && lg == 0) {
        S.st[i] = improved ? (row | ST_ALIAS) : row;
        if (improved) S.fp[i] = fnew;
    }
    // Only the lower halves hold keys; each commits on its own (no barrier).
    if (half == 0) {
        const unsigned long long key = owner ? gbest_key(fnew, i, row) : ~0ull;
        wave_commit(S, t, blockIdx.x * 4u + grp4, key, (improved && lg == 0) ? 1u : 0u);
    }
}

// ---------------------------------------------------------------------------
// Split contraction on bf16 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// An FP32 value v is the exact sum of three bf16 values v1 + v2 + v3: v1 is v
// rounded to 8 significant bits, v - v1 is exact in FP32 with at most 16, and
// so on.  Of the nine part products of a * d the kernel takes the six whose
// weight is 2^-16 or more relative to |a d| (a1 d1; a1 d2, a2 d1; a1 d3,
// a3 d1, a2 d2); each is exact in FP32 and the MFMA accumulates in FP32.  The
// three left out sum to less than 2^-23 |a d|.  The contraction then runs on
// the matrix cores at the bf16 rate, beside the select's VALU work, instead
// of on the FP32 path it shares with the VALU.
//
// Operand layout.  Step m covers variables [32 m, 32 m + 32).  In the
// 16x16x32 MFMA, lane l supplies A row l % 16 and B column l % 16, and inner
// elements 8 (l / 16) + j, j = 0..7, for both: B element j of lane l of a
// particle tile is variable 32 m + 8 (l / 16) + j of particle l % 16, i.e.
// chunks 8 m + 2 (l / 16) and 8 m + 2 (l / 16) + 1.  A is packed by the host
// as [m][row block][part][lane][8 bf16] (A element j of lane l in row block
// rb is A[16 rb + l % 16][32 m + 8 (l / 16) + j]), so step m is one
// contiguous 3 x NB KB block, double-buffered in LDS.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

uint64_t dense_split_halves(uint32_t d)
{
    return 3u * dense_matrix_floats(d);
}

namespace {

uint16_t bf16_nearest(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

}  // namespace

void dense_pack_split(const float *a, uint32_t d, uint16_t *out)
{
    const uint32_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    const uint32_t nb = dp / 16, steps = dp / 32;
    size_t o = 0;
    for (uint32_t m = 0; m < steps; ++m)
        for (uint32_t rb = 0; rb < nb; ++rb) {
            uint16_t part[3][64][8];
            for (uint32_t lane = 0; lane < 64; ++lane)
                for (uint32_t e = 0; e < 8; ++e) {
                    const uint32_t k = 16 * rb + lane % 16;
                    const uint32_t j = 32 * m + 8 * (lane / 16) + e;
                    const float v = (k < d && j < d) ? a[(size_t)k * d + j] : 0.0f;
                    const uint16_t h1 = bf16_nearest(v);
                    const float r1 = std::isfinite(v) ? v - bf16_value(h1) : 0.0f;
                    const uint16_t h2 = bf16_nearest(r1);
                    const uint16_t h3 = bf16_nearest(r1 - bf16_value(h2));
                    part[0][lane][e] = h1;
                    part[1][lane][e] = h2;
                    part[2][lane][e] = h3;
                }
            for (uint32_t p = 0; p < 3; ++p)
                for (uint32_t lane = 0; lane < 64; ++lane)
                    for (uint32_t e = 0; e < 8; ++e) out[o++] = part[p][lane][e];
        }
}

// Two-part fp16 split (contraction F16X2).  Row k of A is scaled by 2^e_k
// and the differences d = x - s by 2^e_d, powers of two that put the largest
// |a_kj| in [2^13, 2^14) and every |d_j| below 2^13 (from the box and the
// shift), well inside fp16's range; a scaled value v is split into
// h = fp16(v) and m = fp16((v - h) 2^11), each rounded to nearest.  The
// kernel takes the products h_a h_d, h_a m_d and m_a h_d (fp16 products are
// exact in FP32) and forms y_k = (sum h h + 2^-11 sum (h m + m h)) 2^-(e_k +
// e_d).  Layout: the parts as [step][row block][part][lane][8 halves]
// (2 dp^2 halves), then dp row factors 2^-(e_k + e_d), then 2^e_d (floats).
uint64_t dense_f16x2_halves(uint32_t d)
{
    const uint64_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    return 2u * dense_matrix_floats(d) + 2u * (dp + 4u);
}

namespace {

// e with 2^(e - 1) <= x < 2^e, for finite x > 0.
int exponent_above(double x)
{
    int e = 0;
    (void)std::frexp(x, &e);
    return e;
}

uint16_t f16_bits(float v)
{
    const _Float16 h = (_Float16)v;  // round to nearest even, subnormals included
    uint16_t u;
    memcpy(&u, &h, 2);
    return u;
}

float f16_value(uint16_t u)
{
    _Float16 h;
    memcpy(&h, &u, 2);
    return (float)h;
}

}  // namespace

bool dense_pack_f16x2(const float *a, uint32_t d, const float *s, float lo, float hi, uint16_t *out)
{
    const uint32_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    const uint32_t nb = dp / 16, steps = dp / 32;
    double dmax = 0.0;
    for (uint32_t j = 0; j < d; ++j) {
        if (!std::isfinite(s[j])) return false;
        dmax = std::max(dmax, std::max(std::fabs((double)lo - s[j]), std::fabs((double)hi - s[j])));
    }
    if (!std::isfinite(dmax)) return false;
    const int ed = dmax > 0.0 ? 13 - exponent_above(dmax) : 0;
    if (ed < -100 || ed > 100) return false;
    // Row exponents (checked without allocating; kept only when packing).
    auto row_exp = [&](uint32_t k, int *e) {
        double amax = 0.0;
        for (uint32_t j = 0; j < d; ++j) {
            const float v = a[(size_t)k * d + j];
            if (!std::isfinite(v)) return false;
            amax = std::max(amax, (double)std::fabs(v));
        }
        *e = amax > 0.0 ? 14 - exponent_above(amax) : 0;
        return *e >= -100 && *e <= 100 && *e + ed >= -120 && *e + ed <= 120;
    };
    for (uint32_t k = 0; k < d; ++k) {
        int e = 0;
        if (!row_exp(k, &e)) return false;
    }
    if (!out) return true;
    std::vector<int> er(dp, 0);
    for (uint32_t k = 0; k < d; ++k) (void)row_exp(k, &er[k]);
    size_t o = 0;
    for (uint32_t m = 0; m < steps; ++m)
        for (uint32_t rb = 0; rb < nb; ++rb) {
            uint16_t part[2][64][8];
            for (uint32_t lane = 0; lane < 64; ++lane)
                for (uint32_t e = 0; e < 8; ++e) {
                    const uint32_t k = 16 * rb + lane % 16;
                    const uint32_t j = 32 * m + 8 * (lane / 16) + e;
                    const float v = (k < d && j < d) ? (float)std::ldexp((double)a[(size_t)k * d + j], er[k])
                                                     : 0.0f;
                    const uint16_t h = f16_bits(v);
                    part[0][lane][e] = h;
                    part[1][lane][e] = f16_bits((v - f16_value(h)) * 2048.0f);
                }
            for (uint32_t p = 0; p < 2; ++p)
                for (uint32_t lane = 0; lane < 64; ++lane)
                    for (uint32_t e = 0; e < 8; ++e) out[o++] = part[p][lane][e];
        }
    float tail[4] = {(float)std::ldexp(1.0, ed), 0.f, 0.f, 0.f};
    std::vector<float> rf(dp);
    for (uint32_t k = 0; k < dp; ++k) rf[k] = (float)std::ldexp(1.0, -(er[k] + ed));
    memcpy(out + o, rf.data(), sizeof(float) * dp);
    memcpy(out + o + 2u * dp, tail, sizeof tail);
    return true;
}

// The generation kernel.  The 64 particles of a workgroup are spread over
// eight waves, two per SIMD, so that one wave's matrix-core work runs while
// the other selects or waits.
//   Select: thread (particle pl = tid / 8, q = tid % 8) selects chunk
//   8 m + q of its particle in step m (Eq. 2.1), writes it, and writes the
//   parts of d = x' - s (three bf16, or two scaled fp16) into LDS in the
//   B-operand layout: tile pl / 16, lane (pl % 16) + 16 (q / 2), elements
//   4 (q % 2) .. 4 (q % 2) + 3.
//   Contract: wave w owns row blocks 2 w and 2 w + 1 of A for all four tiles
//   of 16 particles: per step it takes its A operands (its row blocks, every
//   part) from global memory straight into registers -- no other wave uses
//   them, so they would only pass through LDS (8 % faster without) -- and
//   reads the B operands of all four tiles from LDS.
//   Fitness: each wave's partial sum of y_k^2 over its 32 rows per particle
//   meets the others' in LDS, added in wave order.
// One barrier per step: step m + 1's d parts are written during step m into
// the buffer not read in step m; step m + 1's A operands are requested at
// the start of step m into the register set not used in step m.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// The three bf16 parts of four FP32 values.
__device__ __forceinline__ void split3x4(f4 d, bf16x4 &h, bf16x4 &m, bf16x4 &l)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float v = d[j];
        const __bf16 v1 = (__bf16)v;
        const float r1 = v - (float)v1;
        const __bf16 v2 = (__bf16)r1;
        h[j] = v1;
        m[j] = v2;
        l[j] = (__bf16)(r1 - (float)v2);
    }
}

// The two fp16 parts of four scaled FP32 values (contraction F16X2).
__device__ __forceinline__ void split2x4(f4 v, half4 &h, half4 &m)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const _Float16 v1 = (_Float16)v[j];
        h[j] = v1;
        m[j] = (_Float16)((v[j] - (float)v1) * 2048.0f);
    }
}

// F16: the two-part fp16 split (three products, two accumulators) instead
// of the three-part bf16 one (six products).
template <int NB, bool EQ21, bool INIT, bool FULL_D, bool F16>
__global__ __launch_bounds__(512) void k_dense3(SwarmDev S, uint32_t t)
{
    constexpr uint32_t PARTS = F16 ? 2u : 3u;
    constexpr uint32_t STEPS = NB / 2;              // 32 variables per step
    constexpr uint32_t B_U = 4u * PARTS * 64u;      // 16-byte units of d parts per step
    __shared__ f4 ldb0[B_U];
    __shared__ f4 ldb1[B_U];
    __shared__ float fpart[8][64];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t pl = tid >> 3, q = tid & 7u;
    const uint32_t ip = blockIdx.x * 64u + pl;
    // A thread of a particle past the last one works as a copy of particle
    // n - 1 (same rows and words, the same values to the same addresses) and
    // its fitness is not used: the select has no branch.
    const uint32_t ie = ip < S.n ? ip : S.n - 1u;
    const uint32_t bsl = ((pl >> 4) * PARTS * 64u + (pl & 15u) + 16u * (q >> 1)) * 2u + (q & 1u);
    const f4 *a_pack = reinterpret_cast<const f4 *>(S.a3);
    // F16X2: row factors after the parts, then the scale of d.
    const float *rfac = reinterpret_cast<const float *>(S.a3 + 2u * NB * 16u * NB * 16u);
    const float dsc = F16 ? rfac[NB * 16u] : 1.0f;

    unsigned long long gkey = ~0ull;
    if constexpr (!INIT) gkey = generation_key_load(S, t);
    // The particle this thread decides for (wave 0): pBest fitness and state.
    const uint32_t idec = blockIdx.x * 64u + tid;
    const bool dvalid = tid < 64u && idec < S.n;
    uint32_t st = ST_ALIAS, std_ = ST_ALIAS;
    float fpi = 0.0f;
    if (!INIT) {
        st = S.st[ie];
        if (dvalid) {
            std_ = S.st[idec];
            fpi = S.fp[idec];
        }
    }
    const size_t ioff = (size_t)ie * S.stride;
    const f4 *s4 = reinterpret_cast<const f4 *>(S.s);

    const bool mine = NB >= 16 || 2u * wave < (uint32_t)NB;  // this wave owns row blocks
    // This wave's A operands of step m -- row blocks 2 wave and 2 wave + 1,
    // every part, 16 bytes per lane in the MFMA layout -- straight from
    // global memory (L2) into register set b: no other wave of the
    // workgroup reads them, so they take no LDS.
    f4 aop[2][2][PARTS];
    auto load_aop = [&](uint32_t m, uint32_t b) {
        if (mine) {
#pragma unroll
            for (uint32_t r = 0; r < 2; ++r)
#pragma unroll
                for (uint32_t p = 0; p < PARTS; ++p)
                    aop[b][r][p] = a_pack[(((size_t)m * NB + 2u * wave + r) * PARTS + p) * 64u + lane];
        }
    };
    // Step 0's operands do not depend on gBest: requested before the key
    // arrives.
    load_aop(0, 0);
    const f4 zero4 = f4{0.f, 0.f, 0.f, 0.f};
    // Operands of the select, two steps' worth: set m & 1 holds step m's
    // pBest, position, gBest and shift chunks.
    f4 pv[2], xv[2], gv[2], sv[2], row0 = zero4, row1 = zero4;
    pv[0] = pv[1] = xv[0] = xv[1] = gv[0] = gv[1] = sv[0] = sv[1] = zero4;
    if (FULL_D || q < S.chunks) {
        sv[0] = s4[q];
        if constexpr (!INIT) {
            row0 = reinterpret_cast<const f4 *>(S.rows + ioff)[q];
            row1 = reinterpret_cast<const f4 *>(S.rows + S.buf + ioff)[q];
        }
    }
    uint4 k_first = words4(S, q, ie, t);
    asm volatile("" : "+v"(k_first.x), "+v"(k_first.y), "+v"(k_first.z), "+v"(k_first.w));

    const uint32_t prow = st & ST_ROW;
    const bool alias = (st & ST_ALIAS) != 0u;
    const f4 *p4 = reinterpret_cast<const f4 *>(S.rows + prow * S.buf + ioff);
    f4 *x4 = reinterpret_cast<f4 *>(S.rows + (INIT ? 0u : (1u - prow)) * S.buf + ioff);
    const f4 *xsrc = alias ? p4 : x4;
    pv[0] = prow ? row1 : row0;
    xv[0] = alias ? pv[0] : (prow ? row0 : row1);

    const f4 *g4 = reinterpret_cast<const f4 *>(S.rows);
    // Step m's pBest, position and shift chunks into set b, and its gBest
    // chunk (known once the key of the previous generation is).
    auto prefetch_own = [&](uint32_t m, uint32_t b) {
        const uint32_t c = 8u * m + q;
        if (FULL_D || c < S.chunks) {
            sv[b] = s4[c];
            if constexpr (!INIT) {
                pv[b] = p4[c];
                xv[b] = xsrc[c];
            }
        }
    };
    auto prefetch_g = [&](uint32_t m, uint32_t b) {
        const uint32_t c = 8u * m + q;
        if constexpr (!INIT)
            if (FULL_D || c < S.chunks) gv[b] = g4[c];
    };
    if (STEPS > 1) prefetch_own(1, 1);
    if constexpr (!INIT) {
        const uint32_t glow = (uint32_t)generation_begin(S, t, blockIdx.x, gkey);
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        g4 = reinterpret_cast<const f4 *>(S.rows + (size_t)(glow & 1u) * S.buf + (size_t)gidx * S.stride);
        prefetch_g(0, 0);
        if (STEPS > 1) prefetch_g(1, 1);
    }

    // Select (Eq. 2.1) step m's chunk from set b and write the three bf16
    // parts of d = x' - s into d-part buffer `db`.
    auto select_step = [&](uint32_t m, uint32_t b, f4 *db) {
        const uint32_t c = 8u * m + q;
        f4 dv = zero4;
        if (FULL_D || c < S.chunks) {
            const uint4 k = m == 0 ? k_first : words4(S, c, ie, t);
            f4 xn;
            if constexpr (INIT)
                xn = init4(S, k);
            else
                xn = select4<EQ21>(S, k, gv[b], pv[b], xv[b]);
            x4[c] = xn;
            if constexpr (FULL_D) {
                dv = xn - sv[b];
            } else {
                const uint32_t j0 = 4u * c;
                dv.x = (j0 + 0 < S.d) ? xn.x - sv[b].x : 0.f;
                dv.y = (j0 + 1 < S.d) ? xn.y - sv[b].y : 0.f;
                dv.z = (j0 + 2 < S.d) ? xn.z - sv[b].z : 0.f;
                dv.w = (j0 + 3 < S.d) ? xn.w - sv[b].w : 0.f;
            }
        }
        if constexpr (F16) {
            half4 h, md;
            split2x4(dv * dsc, h, md);  // the scale is a power of two: exact
            half4 *dst = reinterpret_cast<half4 *>(db);
            dst[bsl] = h;
            dst[bsl + 128u] = md;
        } else {
            bf16x4 h, md, lo;
            split3x4(dv, h, md, lo);
            bf16x4 *dst = reinterpret_cast<bf16x4 *>(db);
            dst[bsl] = h;
            dst[bsl + 128u] = md;
            dst[bsl + 256u] = lo;
        }
    };

    select_step(0, 0, ldb0);

    f4 acc[2][4];
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r)
#pragma unroll
        for (uint32_t pt = 0; pt < 4; ++pt) acc[r][pt] = zero4;
    // F16X2: the cross products h m + m h, scaled by 2^-11 at the end.
    f4 acc2[2][4];
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r)
#pragma unroll
        for (uint32_t pt = 0; pt < 4; ++pt) acc2[r][pt] = zero4;

    __syncthreads();  // step 0's d parts are in LDS

#pragma unroll
    for (uint32_t m = 0; m < STEPS; ++m) {
        const uint32_t cur = m & 1u;
        const bool more = m + 1 < STEPS;
        if (more) load_aop(m + 1, cur ^ 1u);
        if (m + 2 < STEPS) {
            prefetch_own(m + 2, cur);
            prefetch_g(m + 2, cur);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (more) select_step(m + 1, cur ^ 1u, cur ? ldb0 : ldb1);
        if (mine) {
            const f4 *lb = cur ? ldb1 : ldb0;
            if constexpr (F16) {
                half8 bh[4], bm[4];
#pragma unroll
                for (uint32_t pt = 0; pt < 4; ++pt) {
                    bh[pt] = __builtin_bit_cast(half8, lb[(pt * 2u + 0u) * 64u + lane]);
                    bm[pt] = __builtin_bit_cast(half8, lb[(pt * 2u + 1u) * 64u + lane]);
                }
#pragma unroll
                for (uint32_t r = 0; r < 2; ++r) {
                    const half8 a1 = __builtin_bit_cast(half8, aop[cur][r][0]);
                    const half8 a2 = __builtin_bit_cast(half8, aop[cur][r][1]);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc2[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, bm[pt], acc2[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc2[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, bh[pt], acc2[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, bh[pt], acc[r][pt], 0, 0, 0);
                }
            } else {
                bf16x8 bh[4], bm[4], bl[4];
#pragma unroll
                for (uint32_t pt = 0; pt < 4; ++pt) {
                    bh[pt] = __builtin_bit_cast(bf16x8, lb[(pt * 3u + 0u) * 64u + lane]);
                    bm[pt] = __builtin_bit_cast(bf16x8, lb[(pt * 3u + 1u) * 64u + lane]);
                    bl[pt] = __builtin_bit_cast(bf16x8, lb[(pt * 3u + 2u) * 64u + lane]);
                }
#pragma unroll
                for (uint32_t r = 0; r < 2; ++r) {
                    const bf16x8 a1 = __builtin_bit_cast(bf16x8, aop[cur][r][0]);
                    const bf16x8 a2 = __builtin_bit_cast(bf16x8, aop[cur][r][1]);
                    const bf16x8 a3 = __builtin_bit_cast(bf16x8, aop[cur][r][PARTS - 1]);
                    // Smallest products first, four independent accumulators
                    // between two updates of the same one.
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bl[pt], acc[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, bh[pt], acc[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bm[pt], acc[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bm[pt], acc[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bh[pt], acc[r][pt], 0, 0, 0);
#pragma unroll
                    for (uint32_t pt = 0; pt < 4; ++pt)
                        acc[r][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bh[pt], acc[r][pt], 0, 0, 0);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // The LDS writes of this step (the next step's d parts) are visible
        // and this wave's LDS reads of the buffer the next step overwrites are
        // done before the barrier; loads of later steps stay in flight.
        // (lgkmcnt is bits 11:8; vmcnt 3:0 and 15:14, expcnt 6:4 at maxima.)
        __builtin_amdgcn_s_waitcnt(0xC07Fu);  // lgkmcnt(0)
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
    }

    // f = sum_k y_k^2: lane (column l % 16, group l / 16) holds rows
    // 4 (l / 16) + r of the wave's two row blocks for particle 16 pt + l % 16;
    // the four lane groups, then the eight waves, meet.
    if constexpr (F16) {
        // y = (sum h h + 2^-11 sum (h m + m h)) 2^-(e_k + e_d), row k of
        // element i of acc[r][pt] being 16 (2 wave + r) + 4 (lane / 16) + i.
        if (mine) {
#pragma unroll
            for (uint32_t r = 0; r < 2; ++r) {
                const f4 rf = reinterpret_cast<const f4 *>(rfac)[4u * (2u * wave + r) + (lane >> 4)];
#pragma unroll
                for (uint32_t pt = 0; pt < 4; ++pt)
                    acc[r][pt] = (acc[r][pt] + acc2[r][pt] * (1.0f / 2048.0f)) * rf;
            }
        }
    }
    float fw[4];
#pragma unroll
    for (uint32_t pt = 0; pt < 4; ++pt) {
        float f = 0.0f;
#pragma unroll
        for (uint32_t r = 0; r < 2; ++r) {
            f += acc[r][pt][0] * acc[r][pt][0];
            f += acc[r][pt][1] * acc[r][pt][1];
            f += acc[r][pt][2] * acc[r][pt][2];
            f += acc[r][pt][3] * acc[r][pt][3];
        }
        f += __shfl_xor(f, 16, 64);
        f += __shfl_xor(f, 32, 64);
        fw[pt] = f;
    }
    const uint32_t lgp = lane >> 4;
    const float mine_f = lgp == 0 ? fw[0] : lgp == 1 ? fw[1] : lgp == 2 ? fw[2] : fw[3];
    fpart[wave][16u * lgp + (lane & 15u)] = mine_f;
    __syncthreads();
    if (wave != 0) return;
    float f = 0.0f;
#pragma unroll
    for (uint32_t w = 0; w < 8; ++w) f += fpart[w][tid];

    const uint32_t prow_d = std_ & ST_ROW;
    const bool improved = dvalid && (INIT || improves(f, fpi));
    uint32_t row = prow_d;
    float fnew = fpi;
    if (improved) {
        row = INIT ? 0u : 1u - prow_d;
        fnew = f;
    }
    if (dvalid) {
        S.st[idec] = improved ? (row | ST_ALIAS) : row;
        if (improved) S.fp[idec] = fnew;
    }
    const unsigned long long key = dvalid ? gbest_key(fnew, idec, row) : ~0ull;
    wave_commit(S, t, blockIdx.x, key, improved ? 1u : 0u);
}

template <int NB, bool FULL_D, bool F16>
static void launch_split(const SwarmDev &S, uint32_t t, dim3 grid, hipStream_t st, bool eq21)
{
    const dim3 block(512);
    if (t == 0) {
        if (eq21)
            hipLaunchKernelGGL((k_dense3<NB, true, true, FULL_D, F16>), grid, block, 0, st, S, t);
        else
            hipLaunchKernelGGL((k_dense3<NB, false, true, FULL_D, F16>), grid, block, 0, st, S, t);
    } else {
        if (eq21)
            hipLaunchKernelGGL((k_dense3<NB, true, false, FULL_D, F16>), grid, block, 0, st, S, t);
        else
            hipLaunchKernelGGL((k_dense3<NB, false, false, FULL_D, F16>), grid, block, 0, st, S, t);
    }
}

template <int NB, bool FULL_D>
static void launch_nbf(const SwarmDev &S, uint32_t t, dim3 grid, hipStream_t st)
{
    const bool eq21 = S.order != 0;
    if (S.a3 && S.split == SPLIT_F16X2) {
        launch_split<NB, FULL_D, true>(S, t, grid, st, eq21);
        return;
    }
    if (S.a3) {
        launch_split<NB, FULL_D, false>(S, t, grid, st, eq21);
        return;
    }
    if (t == 0) {
        if (eq21)
            hipLaunchKernelGGL((k_dense<NB, true, true, FULL_D>), grid, dim3(kDenseBlock), 0, st, S, t);
        else
            hipLaunchKernelGGL((k_dense<NB, false, true, FULL_D>), grid, dim3(kDenseBlock), 0, st, S, t);
    } else {
        if (eq21)
            hipLaunchKernelGGL((k_dense<NB, true, false, FULL_D>), grid, dim3(kDenseBlock), 0, st, S, t);
        else
            hipLaunchKernelGGL((k_dense<NB, false, false, FULL_D>), grid, dim3(kDenseBlock), 0, st, S, t);
    }
}

template <int NB>
static void launch_nb(const SwarmDev &S, uint32_t t, dim3 grid, hipStream_t st)
{
    if (S.d == S.dp)
        launch_nbf<NB, true>(S, t, grid, st);
    else
        launch_nbf<NB, false>(S, t, grid, st);
}

int launch_dense_generation(const SwarmDev &S, uint32_t t, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((S.n + 63u) / 64u);
    switch (S.dp) {
    case 32: launch_nb<2>(S, t, grid, st); break;
    case 64: launch_nb<4>(S, t, grid, st); break;
    case 96: launch_nb<6>(S, t, grid, st); break;
    case 128: launch_nb<8>(S, t, grid, st); break;
    case 160: launch_nb<10>(S, t, grid, st); break;
    case 192: launch_nb<12>(S, t, grid, st); break;
    case 224: launch_nb<14>(S, t, grid, st); break;
    case 256: launch_nb<16>(S, t, grid, st); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace sso
