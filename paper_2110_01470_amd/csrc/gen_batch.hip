// BATCH engine: many independent swarms, each advanced one generation per
// launch by the STREAM body (stream_body.hpp).
//
// The swarms are separate problems (each its own objective instance, size,
// thresholds and Philox key), so the only thing they share is the launch:
// workgroup b reads its (swarm, block) pair from the tile table and the
// swarm's parameters from the swarm table -- both uniform, so they land in
// scalar registers -- and runs the same fused generation as the one-swarm
// kernel with the swarm's own lane width.  Workgroups of different swarms
// never communicate; those of one swarm meet only in that swarm's gBest
// sub-slots.  The host orders the tile table so that the longest workgroups
// start first.
#include "stream_body.hpp"

namespace sso {

template <int KIND, bool EQ21, bool INIT, class Store, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_batch(BatchDev B, uint32_t j)
{
    const uint32_t sw = B.tiles[2u * blockIdx.x];
    const uint32_t blk = B.tiles[2u * blockIdx.x + 1u];
    const SwarmDev S = B.table[sw];
    const uint32_t t = INIT ? 0u : *B.tbase + j;
    if (S.d & 3u)
        stream_body<KIND, 0, EQ21, INIT, true, true, Store, false, WAVES>(S, t, blk, S.lanes);
    else
        stream_body<KIND, 0, EQ21, INIT, false, true, Store, false, WAVES>(S, t, blk, S.lanes);
}

// Trace ring and sub-slot groups of swarm blockIdx.x to "nothing yet".
__global__ void k_batch_fill(BatchDev B)
{
    const SwarmDev &S = B.table[blockIdx.x];
    for (uint32_t q = threadIdx.x; q < S.trace_cap; q += blockDim.x) {
        S.keys[q] = ~0ull;
        S.cnt[q] = 0u;
    }
    for (uint32_t q = threadIdx.x; q < kGroups * kSubSlots; q += blockDim.x) {
        *sub_key(S, q / kSubSlots, q % kSubSlots) = ~0ull;
        *sub_cnt(S, q / kSubSlots, q % kSubSlots) = 0u;
    }
}

// *tbase = v (add == 0) or *tbase += v.
__global__ void k_batch_base(BatchDev B, uint32_t add, uint32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *B.tbase = add ? *B.tbase + v : v;
}

// Swarm blockIdx.x: gBest key and improved count of generation t from its
// sub-slot group (one wave).
__global__ void k_batch_collect(BatchDev B, uint32_t t)
{
    const SwarmDev &S = B.table[blockIdx.x];
    const uint32_t lane = threadIdx.x;
    const uint32_t g = t % kGroups;
    const bool used = lane < S.nsub;
    unsigned long long k = used ? *sub_key(S, g, lane) : ~0ull;
    uint32_t c = used ? *sub_cnt(S, g, lane) : 0u;
    k = wave_min_u64(k);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
    if (lane == 0) {
        B.results[2u * blockIdx.x] = k;
        B.results[2u * blockIdx.x + 1u] = c;
    }
}

namespace {

template <int KIND, bool EQ21, bool INIT, class Store>
const void *kernel_for_waves(uint32_t waves)
{
    if (waves == 4u) return reinterpret_cast<const void *>(&k_batch<KIND, EQ21, INIT, Store, 4>);
    if (waves == 8u) return reinterpret_cast<const void *>(&k_batch<KIND, EQ21, INIT, Store, 8>);
    return nullptr;
}

template <int KIND, bool EQ21, bool INIT>
const void *kernel_for_storage(const BatchDev &B)
{
    return B.storage == STORE_U24 ? kernel_for_waves<KIND, EQ21, INIT, StoreU24>(B.waves)
                                  : kernel_for_waves<KIND, EQ21, INIT, StoreF32>(B.waves);
}

template <int KIND, bool INIT>
const void *kernel_for_order(const BatchDev &B)
{
    return B.order ? kernel_for_storage<KIND, true, INIT>(B) : kernel_for_storage<KIND, false, INIT>(B);
}

template <bool INIT>
const void *batch_kernel(const BatchDev &B)
{
    if (B.kind == OBJ_SPHERE) return kernel_for_order<OBJ_SPHERE, INIT>(B);
    if (B.kind == OBJ_RIPPLE) return kernel_for_order<OBJ_RIPPLE, INIT>(B);
    return nullptr;
}

int launch_gen(const BatchDev &B, const void *fn, uint32_t j, hipStream_t st)
{
    if (!fn) return (int)hipErrorInvalidValue;
    BatchDev b = B;
    void *args[] = {&b, &j};
    return (int)hipLaunchKernel(fn, dim3(B.ntiles), dim3(64 * B.waves), args, B.lds, st);
}

}  // namespace

size_t batch_stage_bytes(int kind, int storage, uint32_t chunks)
{
    SwarmDev S{};
    S.chunks = chunks;
    if (kind == OBJ_RIPPLE)
        return storage == STORE_U24 ? stage_bytes<OBJ_RIPPLE, StoreU24>(S) : stage_bytes<OBJ_RIPPLE, StoreF32>(S);
    return storage == STORE_U24 ? stage_bytes<OBJ_SPHERE, StoreU24>(S) : stage_bytes<OBJ_SPHERE, StoreF32>(S);
}

int launch_batch_fill(const BatchDev &B, void *stream)
{
    hipLaunchKernelGGL(k_batch_fill, dim3(B.count), dim3(256), 0, (hipStream_t)stream, B);
    return (int)hipGetLastError();
}

int launch_batch_init(const BatchDev &B, void *stream)
{
    return launch_gen(B, batch_kernel<true>(B), 0u, (hipStream_t)stream);
}

int launch_batch_set_base(const BatchDev &B, uint32_t t, void *stream)
{
    hipLaunchKernelGGL(k_batch_base, dim3(1), dim3(64), 0, (hipStream_t)stream, B, 0u, t);
    return (int)hipGetLastError();
}

int launch_batch_generations(const BatchDev &B, uint32_t k, void *stream)
{
    const hipStream_t st = (hipStream_t)stream;
    const void *fn = batch_kernel<false>(B);
    for (uint32_t j = 1; j <= k; ++j) {
        const int e = launch_gen(B, fn, j, st);
        if (e) return e;
    }
    hipLaunchKernelGGL(k_batch_base, dim3(1), dim3(64), 0, st, B, 1u, k);
    return (int)hipGetLastError();
}

int batch_graph(const BatchDev &B, uint32_t k, void **graph_out)
{
    *graph_out = nullptr;
    const void *fn = batch_kernel<false>(B);
    if (!fn) return (int)hipErrorInvalidValue;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return (int)e;
    hipGraphNode_t prev = nullptr, node = nullptr;
    for (uint32_t j = 1; j <= k + 1 && e == hipSuccess; ++j) {
        BatchDev b = B;
        uint32_t jj = j, add = 1u, kk = k;
        void *gen_args[] = {&b, &jj};
        void *base_args[] = {&b, &add, &kk};
        hipKernelNodeParams p{};
        if (j <= k) {
            p.func = const_cast<void *>(fn);
            p.gridDim = dim3(B.ntiles);
            p.blockDim = dim3(64 * B.waves);
            p.sharedMemBytes = B.lds;
            p.kernelParams = gen_args;
        } else {
            p.func = reinterpret_cast<void *>(&k_batch_base);
            p.gridDim = dim3(1);
            p.blockDim = dim3(64);
            p.sharedMemBytes = 0;
            p.kernelParams = base_args;
        }
        p.extra = nullptr;
        e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        prev = node;
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return (int)e;
    }
    *graph_out = g;
    return hipSuccess;
}

int launch_batch_collect(const BatchDev &B, uint32_t t, void *stream)
{
    hipLaunchKernelGGL(k_batch_collect, dim3(B.count), dim3(64), 0, (hipStream_t)stream, B, t);
    return (int)hipGetLastError();
}

}  // namespace sso
