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
    const bool improved = owner && (INIT || f < fpi);
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

template <int NB, bool FULL_D>
static void launch_nbf(const SwarmDev &S, uint32_t t, dim3 grid, hipStream_t st)
{
    const bool eq21 = S.order != 0;
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
