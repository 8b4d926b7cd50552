// STREAM engine: one fused kernel per generation for the separable
// objectives (sphere, ripple) of one swarm; the body is in stream_body.hpp.
#include "stream_body.hpp"

namespace sso {

template <int KIND, int L, bool EQ21, bool INIT, bool RAGGED, bool STAGE, class Store>
__global__ __launch_bounds__(64 * kWaves) void k_stream(SwarmDev S, uint32_t t)
{
    stream_body<KIND, L, EQ21, INIT, RAGGED, STAGE, Store>(S, t, blockIdx.x, L ? (uint32_t)L : S.lanes);
}

template <int KIND, int L, bool EQ21, bool RAGGED, bool STAGE, class Store>
static int launch_kl(const SwarmDev &S, uint32_t t, hipStream_t st)
{
    constexpr int per_block = kWaves * (64 / L);
    const uint32_t blocks = (S.n + per_block - 1) / per_block;
    const size_t lds = STAGE ? stage_bytes<KIND, Store>(S) : 0;
    if (t == 0)
        hipLaunchKernelGGL((k_stream<KIND, L, EQ21, true, RAGGED, STAGE, Store>), dim3(blocks),
                           dim3(64 * kWaves), lds, st, S, t);
    else
        hipLaunchKernelGGL((k_stream<KIND, L, EQ21, false, RAGGED, STAGE, Store>), dim3(blocks),
                           dim3(64 * kWaves), lds, st, S, t);
    return (int)hipGetLastError();
}

template <int KIND, int L, bool EQ21, class Store>
static int launch_klr(const SwarmDev &S, uint32_t t, hipStream_t st)
{
    const bool ragged = (S.d & 3u) != 0u;
    if (S.chunks <= kStageMaxChunks)
        return ragged ? launch_kl<KIND, L, EQ21, true, true, Store>(S, t, st)
                      : launch_kl<KIND, L, EQ21, false, true, Store>(S, t, st);
    return ragged ? launch_kl<KIND, L, EQ21, true, false, Store>(S, t, st)
                  : launch_kl<KIND, L, EQ21, false, false, Store>(S, t, st);
}

template <int KIND, int L, bool EQ21>
static int launch_kls(const SwarmDev &S, uint32_t t, hipStream_t st)
{
    return S.storage == STORE_U24 ? launch_klr<KIND, L, EQ21, StoreU24>(S, t, st)
                                  : launch_klr<KIND, L, EQ21, StoreF32>(S, t, st);
}

template <int KIND, bool EQ21>
static int launch_k(const SwarmDev &S, uint32_t t, uint32_t lanes, hipStream_t st)
{
    switch (lanes) {
    case 8: return launch_kls<KIND, 8, EQ21>(S, t, st);
    case 16: return launch_kls<KIND, 16, EQ21>(S, t, st);
    case 32: return launch_kls<KIND, 32, EQ21>(S, t, st);
    case 64: return launch_kls<KIND, 64, EQ21>(S, t, st);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_stream_generation(const SwarmDev &S, uint32_t t, uint32_t lanes, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (is_paper_kind(S.kind)) return launch_stream_paper(S, t, st);
    const bool eq21 = S.order != 0;
    if (S.kind == OBJ_SPHERE)
        return eq21 ? launch_k<OBJ_SPHERE, true>(S, t, lanes, st)
                    : launch_k<OBJ_SPHERE, false>(S, t, lanes, st);
    if (S.kind == OBJ_RIPPLE)
        return eq21 ? launch_k<OBJ_RIPPLE, true>(S, t, lanes, st)
                    : launch_k<OBJ_RIPPLE, false>(S, t, lanes, st);
    return (int)hipErrorInvalidValue;
}

// Clears the trace ring (keys to "no gBest yet", counts to zero) and every
// sub-slot group.  A kernel rather than a memset so the clear can sit inside
// a captured graph.
__global__ void k_fill_trace(SwarmDev S)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < S.trace_cap) {
        S.keys[j] = ~0ull;
        S.cnt[j] = 0u;
    }
    if (j < kGroups * kSubSlots) {
        *sub_key(S, j / kSubSlots, j % kSubSlots) = ~0ull;
        *sub_cnt(S, j / kSubSlots, j % kSubSlots) = 0u;
    }
}

int launch_fill_trace(const SwarmDev &S, void *stream)
{
    const uint32_t items = S.trace_cap > kGroups * kSubSlots ? S.trace_cap : kGroups * kSubSlots;
    const uint32_t blocks = (items + 255u) / 256u;
    hipLaunchKernelGGL(k_fill_trace, dim3(blocks), dim3(256), 0, (hipStream_t)stream, S);
    return (int)hipGetLastError();
}

// The word of every (particle, variable) at generation t, as the kernels draw
// it.  Lane l of wave w in block (bx, by) owns chunk 64 bx + l of particles
// 4 by + w, 4 (by + gridDim.y) + w, ...; with vec (d a multiple of 4 and
// out 16-byte aligned) a chunk is one 16-byte store.
__global__ __launch_bounds__(256) void k_debug_rng(SwarmDev S, uint32_t t, uint32_t *out,
                                                   bool vec)
{
    const uint32_t c = blockIdx.x * 64u + (threadIdx.x & 63u);
    if (c >= S.chunks) return;
    for (uint32_t i = blockIdx.y * 4u + (threadIdx.x >> 6); i < S.n; i += gridDim.y * 4u) {
        const uint4 k = words4(S, c, i, t);
        uint32_t *row = out + (uint64_t)i * S.d;
        if (vec) {
            reinterpret_cast<uint4 *>(row)[c] = k;
        } else {
            const uint32_t v[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q)
                if (4u * c + q < S.d) row[4u * c + q] = v[q];
        }
    }
}

int launch_debug_rng(const SwarmDev &S, uint32_t t, uint32_t *out, void *stream)
{
    const dim3 grid((S.chunks + 63u) / 64u, std::min<uint32_t>((S.n + 3u) / 4u, 65535u));
    const bool vec = (S.d & 3u) == 0u && (reinterpret_cast<uintptr_t>(out) & 15u) == 0u;
    hipLaunchKernelGGL(k_debug_rng, grid, dim3(256), 0, (hipStream_t)stream, S, t, out, vec);
    return (int)hipGetLastError();
}

}  // namespace sso
