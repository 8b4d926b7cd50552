// STREAM engine for Table 3.2's functions: one fused kernel per generation,
// specialised per (function, order, storage) and, for the generations after
// the initialisation, per lane count LT = 8, 16, 32 or 64 (the counts a swarm
// can have); the initialisation takes S.lanes at run time.  Rows are staged
// (d <= 1024).  The body is in stream_body.hpp.
#include "stream_body.hpp"

namespace sso {

template <int KIND, bool EQ21, bool INIT, class Store, int LT>
__global__ __launch_bounds__(64 * kWaves) void k_stream_paper(SwarmDev S, uint32_t t)
{
    stream_body<KIND, LT, EQ21, INIT, true, true, Store>(S, t, blockIdx.x, LT ? (uint32_t)LT : S.lanes);
}

template <int KIND, bool EQ21, class Store>
static int launch_kind(const SwarmDev &S, uint32_t t, hipStream_t st)
{
    const uint32_t per_block = kWaves * (64u / S.lanes);
    const uint32_t blocks = (S.n + per_block - 1) / per_block;
    const size_t lds = stage_bytes<KIND, Store>(S);
    const dim3 grid(blocks), block(64 * kWaves);
    if (t == 0) {
        hipLaunchKernelGGL((k_stream_paper<KIND, EQ21, true, Store, 0>), grid, block, lds, st, S, t);
    } else {
        switch (S.lanes) {
        case 8: hipLaunchKernelGGL((k_stream_paper<KIND, EQ21, false, Store, 8>), grid, block, lds, st, S, t); break;
        case 16: hipLaunchKernelGGL((k_stream_paper<KIND, EQ21, false, Store, 16>), grid, block, lds, st, S, t); break;
        case 32: hipLaunchKernelGGL((k_stream_paper<KIND, EQ21, false, Store, 32>), grid, block, lds, st, S, t); break;
        case 64: hipLaunchKernelGGL((k_stream_paper<KIND, EQ21, false, Store, 64>), grid, block, lds, st, S, t); break;
        default: return (int)hipErrorInvalidValue;
        }
    }
    return (int)hipGetLastError();
}

template <bool EQ21, class Store>
static int launch_order_store(const SwarmDev &S, uint32_t t, hipStream_t st)
{
    switch (S.kind) {
    case OBJ_F1 + 0: return launch_kind<OBJ_F1 + 0, EQ21, Store>(S, t, st);
    case OBJ_F1 + 1: return launch_kind<OBJ_F1 + 1, EQ21, Store>(S, t, st);
    case OBJ_F1 + 2: return launch_kind<OBJ_F1 + 2, EQ21, Store>(S, t, st);
    case OBJ_F1 + 3: return launch_kind<OBJ_F1 + 3, EQ21, Store>(S, t, st);
    case OBJ_F1 + 4: return launch_kind<OBJ_F1 + 4, EQ21, Store>(S, t, st);
    case OBJ_F1 + 5: return launch_kind<OBJ_F1 + 5, EQ21, Store>(S, t, st);
    case OBJ_F1 + 6: return launch_kind<OBJ_F1 + 6, EQ21, Store>(S, t, st);
    case OBJ_F1 + 7: return launch_kind<OBJ_F1 + 7, EQ21, Store>(S, t, st);
    case OBJ_F1 + 8: return launch_kind<OBJ_F1 + 8, EQ21, Store>(S, t, st);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_stream_paper(const SwarmDev &S, uint32_t t, void *stream)
{
    static_assert(OBJ_F1 + 8 == OBJ_F9, "nine functions");
    hipStream_t st = (hipStream_t)stream;
    if (S.chunks > kStageMaxChunks || S.lanes == 0 || S.lanes > 64 || (S.lanes & (S.lanes - 1)))
        return (int)hipErrorInvalidValue;
    const bool eq21 = S.order != 0;
    if (S.storage == STORE_U24)
        return eq21 ? launch_order_store<true, StoreU24>(S, t, st) : launch_order_store<false, StoreU24>(S, t, st);
    return eq21 ? launch_order_store<true, StoreF32>(S, t, st) : launch_order_store<false, StoreF32>(S, t, st);
}

}  // namespace sso
