// Dense objective f(x) = ||A (x - s)||^2 and its gradient 2 A^T A (x - s) on
// FP32 matrix cores (v_mfma_f32_16x16x4_f32), for given points (sso_eval)
// and for the gradient polish of a swarm's pBests (sso_polish).
//
// Work split as in gen_dense.hip: a workgroup of eight waves owns 64 points
// in four groups of 16; wave half h of a group holds the variables of
// K-chunks [h NB/2, (h+1) NB/2) of its 16 points (lane l: point l%16,
// float4 chunk 4M + l/16 of each of those K-chunks M).
//  1. Y^T = A D^T with D = X - s: each half contracts its K-chunks into a
//     partial Y^T (all NB row blocks), exactly as the generation kernel
//     does; the halves exchange partials through LDS so that both hold the
//     full Y^T, added in the generation kernel's order.
//  2. G^T = A^T Y^T: with A^T packed like A, element r of lane l's
//     accumulator for row block rb (Y^T row 16 rb + 4 (l/16) + r, point
//     l%16) is the B operand MFMA step (rb, r) needs, and output row block
//     jb comes back to the lanes holding chunk 4 jb + l/16 of each point.
//     Each half computes the output blocks of its own K-chunks, so a lane
//     receives the gradient of exactly the variables it holds and the
//     projected step happens in registers.
//  3. f = sum_k y_k^2 over the full Y^T, summed as the generation kernel
//     sums it.
// A and A^T (256 KB each at D=256) stay in L2 and reach the waves through
// LDS: a polish step is a sequence of stages of two K-chunks each (HALF
// stages of A for the residual, both halves' chunks at once; NB/2 stages of
// A^T, two row blocks each, for the gradient).  Every stage is copied into
// one of two LDS buffers by global-to-LDS loads while the waves contract the
// stage before it, so each operand crosses from L2 once per workgroup, not
// once per particle group.
#include "sso_device.hpp"

namespace sso {

namespace {

constexpr int kGradWaves = 8;
constexpr int kGradBlock = 64 * kGradWaves;
enum { MODE_EVAL = 0, MODE_GRAD = 1, MODE_POLISH = 2 };

template <int NB, int MODE, bool ALIGNED>
__global__ __launch_bounds__(kGradBlock) void k_dense_grad(SwarmDev S, GradArgs G, uint32_t steps,
                                                           float lr, uint32_t t)
{
    constexpr uint32_t HALF = NB / 2;
    constexpr uint32_t CF4 = NB * 64u;  // float4 per K-chunk of a packed matrix
    constexpr uint32_t STAGE_F4 = 2 * CF4;  // one stage: two K-chunks
    constexpr uint32_t PER = (STAGE_F4 + kGradBlock - 1) / kGradBlock;
    constexpr bool FULL = STAGE_F4 % kGradBlock == 0;
    __shared__ f4 red[4 * NB * 64];
    // Two stage buffers as two variables, so that the compiler tells the
    // reads of one from the copies in flight into the other.
    __shared__ f4 lds0[STAGE_F4];
    __shared__ f4 lds1[STAGE_F4];
    __shared__ f4 s_lds[NB * 4];  // the shift, dp / 4 chunks (zero past d)

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t grp4 = wave & 3u, half = wave >> 2;
    const uint32_t pcol = lane & 15u, lg = lane >> 4;
    const uint32_t i = blockIdx.x * 64u + grp4 * 16u + pcol;
    const uint32_t npts = MODE == MODE_POLISH ? S.n : G.m;
    const bool valid = i < npts;
    const f4 *a_pack = reinterpret_cast<const f4 *>(S.a);
    const f4 *at_pack = reinterpret_cast<const f4 *>(S.at);
    const f4 *s4 = reinterpret_cast<const f4 *>(S.s);
    const f4 zero4 = f4{0.f, 0.f, 0.f, 0.f};
    const uint32_t cbase = 4u * HALF * half;  // chunk of m = 0; chunk of m is cbase + 4 m + lg

    // Stage q < HALF: K-chunks q (lower half) and HALF + q (upper half) of A,
    // the residual's step q.  Stage q >= HALF: row blocks 2 (q - HALF) and
    // 2 (q - HALF) + 1 of A^T (each a whole packed K-chunk), the gradient's
    // step q - HALF.  Stage q goes to buffer q mod 2.
    auto stage_dma = [&](uint32_t q, uint32_t b) {
        // The copy addresses are the same at every polish step; opaque bases
        // keep the compiler from hoisting all of them out of the step loop
        // (they do not fit in registers).
        const f4 *ap = a_pack, *atp = at_pack;
        asm volatile("" : "+s"(ap), "+s"(atp));
#pragma unroll
        for (uint32_t r = 0; r < PER; ++r) {
            const uint32_t e = tid + r * kGradBlock;
            if (FULL || e < STAGE_F4) {
                const f4 *src = q < HALF ? ap + (size_t)(e < CF4 ? q : HALF + q) * CF4 + (e % CF4)
                                         : atp + (size_t)(2u * (q - HALF)) * CF4 + e;
                __builtin_amdgcn_global_load_lds(
                    (const void *)src,
                    (__attribute__((address_space(3))) void *)(&(b ? lds1 : lds0)[r * kGradBlock + wave * 64u]),
                    16, 0, 0);
            }
        }
    };
    stage_dma(0, 0);

    // The point, chunk by chunk (columns >= d are masked where used).
    f4 pc[HALF];
    uint32_t prow = 0;
    bool alias = true;
    float fpi = 0.0f;
    const float *rowp = S.rows;
    if constexpr (MODE == MODE_POLISH) {
        if (valid) {
            const uint32_t st = S.st[i];
            fpi = S.fp[i];
            prow = st & ST_ROW;
            alias = (st & ST_ALIAS) != 0u;
        }
        rowp = S.rows + prow * S.buf + (size_t)(valid ? i : 0u) * S.stride;
    }
#pragma unroll
    for (uint32_t m = 0; m < HALF; ++m) {
        const uint32_t c = cbase + 4u * m + lg;
        f4 v = zero4;
        if (valid && c < S.chunks) {
            if constexpr (MODE == MODE_POLISH) {
                v = reinterpret_cast<const f4 *>(rowp)[c];
            } else if constexpr (ALIGNED) {
                v = reinterpret_cast<const f4 *>(G.x + (size_t)i * G.ld)[c];
            } else {
                const float *xr = G.x + (size_t)i * G.ld;
                const uint32_t j0 = 4u * c;
                v.x = j0 + 0 < S.d ? xr[j0 + 0] : 0.f;
                v.y = j0 + 1 < S.d ? xr[j0 + 1] : 0.f;
                v.z = j0 + 2 < S.d ? xr[j0 + 2] : 0.f;
                v.w = j0 + 3 < S.d ? xr[j0 + 3] : 0.f;
            }
        }
        pc[m] = v;
    }

    // The shift into LDS: its reads then wait on the LDS counter only, not on
    // the copies in flight.
    for (uint32_t c = tid; c < NB * 4u; c += kGradBlock) s_lds[c] = c < S.chunks ? s4[c] : zero4;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copy of stage 0 has landed
    __syncthreads();

    f4 acc[NB];
    // acc = the full Y^T of the current point (both halves).  grad_next: a
    // gradient follows, so its first stage is copied during the last one here.
    auto residual = [&](bool grad_next) {
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb) acc[rb] = zero4;
#pragma unroll
        for (uint32_t m = 0; m < HALF; ++m) {
            const uint32_t cur = m & 1u;
            const uint32_t c = cbase + 4u * m + lg;
            f4 dv = zero4;
            if (valid && c < S.chunks) {
                const f4 sv = s_lds[c];
                const uint32_t j0 = 4u * c;
                dv.x = (j0 + 0 < S.d) ? pc[m].x - sv.x : 0.f;
                dv.y = (j0 + 1 < S.d) ? pc[m].y - sv.y : 0.f;
                dv.z = (j0 + 2 < S.d) ? pc[m].z - sv.z : 0.f;
                dv.w = (j0 + 3 < S.d) ? pc[m].w - sv.w : 0.f;
            }
            const bool copy = m + 1 < HALF || grad_next;
            if (copy) stage_dma(m + 1, cur ^ 1u);  // stage HALF is the gradient's first
            __builtin_amdgcn_sched_barrier(0);
            const f4 *la = (cur ? lds1 : lds0) + half * CF4 + lane;
            // Row blocks in groups of four: four independent accumulators
            // between dependent MFMAs, 16 registers of A operands.
#pragma unroll
            for (uint32_t r0 = 0; r0 < NB; r0 += 4) {
                f4 av[4];
#pragma unroll
                for (uint32_t q = 0; q < 4 && r0 + q < NB; ++q) av[q] = la[(r0 + q) * 64u];
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e)
#pragma unroll
                    for (uint32_t q = 0; q < 4 && r0 + q < NB; ++q)
                        acc[r0 + q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q][e], dv[e], acc[r0 + q], 0, 0, 0);
            }
            if (copy) __builtin_amdgcn_s_waitcnt(0);  // this wave's copy has landed
            __syncthreads();
        }
        f4 *r = red + (size_t)grp4 * NB * 64u + lane;
        if (half == 1) {
#pragma unroll
            for (uint32_t rb = 0; rb < NB; ++rb) r[rb * 64u] = acc[rb];
        }
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (uint32_t rb = 0; rb < NB; ++rb) {
                acc[rb] = acc[rb] + r[rb * 64u];
                r[rb * 64u] = acc[rb];
            }
        }
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (uint32_t rb = 0; rb < NB; ++rb) acc[rb] = r[rb * 64u];
        }
    };

    // gr[jj] = (A^T Y^T) for output block HALF * half + jj: half the gradient
    // of this lane's chunk jj.  res_next: a residual follows, so its first
    // stage is copied during the last one here.
    f4 gr[HALF];
    auto gradient = [&](bool res_next) {
#pragma unroll
        for (uint32_t jj = 0; jj < HALF; ++jj) gr[jj] = zero4;
#pragma unroll
        for (uint32_t g = 0; g < NB / 2; ++g) {
            const uint32_t cur = (HALF + g) & 1u;
            const bool copy = g + 1 < NB / 2 || res_next;
            if (copy) stage_dma(g + 1 < NB / 2 ? HALF + g + 1 : 0u, cur ^ 1u);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (uint32_t u = 0; u < 2; ++u) {
                const uint32_t rb = 2u * g + u;
                const f4 *la = (cur ? lds1 : lds0) + u * CF4 + (HALF * half) * 64u + lane;
                f4 av[HALF];
#pragma unroll
                for (uint32_t jj = 0; jj < HALF; ++jj) av[jj] = la[jj * 64u];
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e)
#pragma unroll
                    for (uint32_t jj = 0; jj < HALF; ++jj)
                        gr[jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[jj][e], acc[rb][e], gr[jj], 0, 0, 0);
            }
            if (copy) __builtin_amdgcn_s_waitcnt(0);  // this wave's copy has landed
            __syncthreads();
        }
    };

    auto fitness = [&]() -> float {
        float f = 0.0f;
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb) {
            const f4 y = acc[rb];
            f += y[0] * y[0];
            f += y[1] * y[1];
            f += y[2] * y[2];
            f += y[3] * y[3];
        }
        f += __shfl_xor(f, 16, 64);
        f += __shfl_xor(f, 32, 64);
        return f;
    };

    if constexpr (MODE == MODE_POLISH) {
        const float lo = S.lo, hi = S.lo + S.span;
        const float step = -2.0f * lr;  // p - lr * (2 A^T Y^T), one rounding
        // steps + 1 residuals: one per step, the last one scores the result.
        for (uint32_t k = 0;; ++k) {
            residual(k < steps);
            if (k == steps) break;
            gradient(true);
#pragma unroll
            for (uint32_t m = 0; m < HALF; ++m) {
                const uint32_t j0 = 4u * (cbase + 4u * m + lg);
                f4 v = pc[m];
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) {
                    const float u = fminf(fmaxf(__builtin_fmaf(step, gr[m][e], v[e]), lo), hi);
                    v[e] = (j0 + e < S.d) ? u : v[e];
                }
                pc[m] = v;
            }
        }
        const float f = fitness();
        // Algorithm 3's rule: a strict improvement replaces the pBest (NaN ordered last).
        const bool improved = valid && improves(f, fpi);
        const uint32_t nrow = alias ? 1u - prow : prow;
        if (improved) {
            // An aliased pBest is also the position: the polished point goes
            // to the other row, which becomes the pBest row, and the position
            // stays where it was.
            f4 *dst = reinterpret_cast<f4 *>(S.rows + nrow * S.buf + (size_t)i * S.stride);
#pragma unroll
            for (uint32_t m = 0; m < HALF; ++m) {
                const uint32_t c = cbase + 4u * m + lg;
                if (c < S.chunks) dst[c] = pc[m];
            }
        }
        if (half == 0) {
            if (improved && lg == 0) {
                S.st[i] = nrow;
                S.fp[i] = f;
            }
            const unsigned long long key = improved ? gbest_key(f, i, nrow) : ~0ull;
            wave_commit(S, t, blockIdx.x * 4u + grp4, key, 0u);
        }
    } else {
        residual(MODE == MODE_GRAD);
        if constexpr (MODE == MODE_GRAD) {
            gradient(false);
            if (valid) {
                const float scale = 2.0f * (G.gout ? G.gout[i] : 1.0f);
                float *gr_out = G.g + (size_t)i * G.ld;
#pragma unroll
                for (uint32_t m = 0; m < HALF; ++m) {
                    const uint32_t c = cbase + 4u * m + lg;
                    if (c >= S.chunks) continue;
                    const f4 v = gr[m] * scale;
                    if constexpr (ALIGNED) {
                        reinterpret_cast<f4 *>(gr_out)[c] = v;
                    } else {
                        const uint32_t j0 = 4u * c;
#pragma unroll
                        for (uint32_t e = 0; e < 4; ++e)
                            if (j0 + e < S.d) gr_out[j0 + e] = v[e];
                    }
                }
            }
        }
        const float f = fitness();
        if (G.f && valid && half == 0 && lg == 0) G.f[i] = f;
    }
}

template <int NB, int MODE>
int launch_mode(const SwarmDev &S, const GradArgs &G, uint32_t steps, float lr, uint32_t t,
                bool aligned, hipStream_t st)
{
    const uint32_t npts = MODE == MODE_POLISH ? S.n : G.m;
    const dim3 grid((npts + 63u) / 64u);
    if (aligned)
        hipLaunchKernelGGL((k_dense_grad<NB, MODE, true>), grid, dim3(kGradBlock), 0, st, S, G, steps, lr, t);
    else
        hipLaunchKernelGGL((k_dense_grad<NB, MODE, false>), grid, dim3(kGradBlock), 0, st, S, G, steps, lr, t);
    return (int)hipGetLastError();
}

template <int MODE>
int launch_dp(const SwarmDev &S, const GradArgs &G, uint32_t steps, float lr, uint32_t t, bool aligned,
              hipStream_t st)
{
    switch (S.dp) {
    case 32: return launch_mode<2, MODE>(S, G, steps, lr, t, aligned, st);
    case 64: return launch_mode<4, MODE>(S, G, steps, lr, t, aligned, st);
    case 96: return launch_mode<6, MODE>(S, G, steps, lr, t, aligned, st);
    case 128: return launch_mode<8, MODE>(S, G, steps, lr, t, aligned, st);
    case 160: return launch_mode<10, MODE>(S, G, steps, lr, t, aligned, st);
    case 192: return launch_mode<12, MODE>(S, G, steps, lr, t, aligned, st);
    case 224: return launch_mode<14, MODE>(S, G, steps, lr, t, aligned, st);
    case 256: return launch_mode<16, MODE>(S, G, steps, lr, t, aligned, st);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace

int launch_dense_eval(const SwarmDev &S, const GradArgs &G, void *stream)
{
    if (G.m == 0) return hipSuccess;
    // float4 access needs whole chunks and 16-byte aligned rows.
    const bool aligned = (S.d % 4u == 0) && (G.ld % 4u == 0) && ((uintptr_t)G.x % 16u == 0) &&
                         (!G.g || (uintptr_t)G.g % 16u == 0);
    if (G.g) return launch_dp<MODE_GRAD>(S, G, 0, 0.0f, 0, aligned, (hipStream_t)stream);
    return launch_dp<MODE_EVAL>(S, G, 0, 0.0f, 0, aligned, (hipStream_t)stream);
}

int launch_dense_polish(const SwarmDev &S, uint32_t steps, float lr, uint32_t t, void *stream)
{
    GradArgs G{};
    return launch_dp<MODE_POLISH>(S, G, steps, lr, t, true, (hipStream_t)stream);
}

}  // namespace sso
