// STREAM engine: one fused kernel per generation for the separable
// objectives (sphere, ripple).
//
// One generation of Algorithm 2 in a single pass over the state: each group
// of L lanes owns one particle and walks its row in float4 chunks
// (chunk c, c + L, ...), so a wave's loads cover L * 16 contiguous bytes per
// row -- whole 128-byte lines for L >= 8.  Per chunk a lane draws one Philox
// block (four words, one per variable, Sec. 3.1), picks the four new values
// by Eq. (2.1), writes them, and accumulates the objective terms.  The L
// partial sums meet in a butterfly; every lane of the group then holds the
// same fitness, takes the pBest decision of Algorithm 3 (strict <), and the
// workgroup folds its (fitness, index) keys into the generation's gBest slot
// with one atomicMin (Algorithm 4).  Generation t reads gBest from slot t-1
// and clears slot t+1 for the next generation.
//
// With t == 0 the same kernel is the initialisation (kernel (I),
// Sec. 2.3.1): X^0 is drawn uniformly from the generation-0 words, written
// as the pBest row, and scored.
#include "sso_device.hpp"

namespace sso {

constexpr int kWaves = 4;

template <int KIND, int L, bool EQ21, bool INIT>
__global__ __launch_bounds__(64 * kWaves) void k_stream(SwarmDev S, uint32_t t)
{
    constexpr int G = 64 / L;  // particles per wave
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t ln = lane % L;
    const uint32_t i = (blockIdx.x * kWaves + wave) * G + lane / L;
    const bool valid = i < S.n;

    // gBest of the previous generation (unused at t == 0).
    const float *grow_ptr = nullptr;
    if constexpr (!INIT) {
        const unsigned long long gk = S.keys[(t - 1u) % S.trace_cap];
        const uint32_t glow = (uint32_t)gk;
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        grow_ptr = S.rows + (size_t)(glow & 1u) * S.buf + (size_t)gidx * S.dp;
    }

    uint32_t st = 0, prow = 0;
    bool alias = true;
    float fpi = 0.0f;
    if (!INIT && valid) {
        st = S.st[i];
        fpi = S.fp[i];
        prow = st & ST_ROW;
        alias = (st & ST_ALIAS) != 0u;
    }
    const size_t ioff = (size_t)i * S.dp;
    const float4 *prow_ptr = reinterpret_cast<const float4 *>(S.rows + prow * S.buf + ioff);
    // INIT writes the pBest row (row 0); a generation writes the other row.
    float4 *xrow_ptr = reinterpret_cast<float4 *>(S.rows + (INIT ? 0u : (1u - prow)) * S.buf + ioff);
    const float4 *g4 = reinterpret_cast<const float4 *>(grow_ptr);
    const float4 *s4 = reinterpret_cast<const float4 *>(S.s);
    const float4 *w4 = reinterpret_cast<const float4 *>(S.w);

    float acc = 0.0f;
    if (valid) {
        for (uint32_t c = ln; c < S.chunks; c += L) {
            const uint4 k = words4(S, c, i, t);
            float4 xn;
            if constexpr (INIT) {
                xn = make_float4(init_value(S, k.x), init_value(S, k.y), init_value(S, k.z),
                                 init_value(S, k.w));
            } else {
                const float4 p = prow_ptr[c];
                const float4 x = alias ? p : xrow_ptr[c];
                const float4 g = g4[c];
                xn = select4<EQ21>(S, k, g, p, x);
            }
            xrow_ptr[c] = xn;
            const float4 sv = s4[c];
            const float4 wv = (KIND == OBJ_RIPPLE) ? w4[c] : make_float4(0.f, 0.f, 0.f, 0.f);
            acc += terms4<KIND>(xn, sv, wv, 4u * c, S.d);
        }
    }
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);

    // Algorithm 3: replace the pBest on a strict improvement (NaN never does).
    const bool improved = valid && (INIT || acc < fpi);
    uint32_t row = prow;
    float fnew = fpi;
    if (improved) {
        row = INIT ? 0u : 1u - prow;
        fnew = acc;
    }
    if (valid && ln == 0) {
        S.st[i] = improved ? (row | ST_ALIAS) : row;
        if (improved) S.fp[i] = fnew;
    }
    const unsigned long long key = valid ? gbest_key(fnew, i, row) : ~0ull;

    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t nx = (t + 1u) % S.trace_cap;
        S.keys[nx] = ~0ull;
        S.cnt[nx] = 0u;
    }
    const uint32_t slot = t % S.trace_cap;
    workgroup_commit<kWaves>(key, (improved && ln == 0) ? 1u : 0u, S.keys + slot, S.cnt + slot);
}

template <int KIND, int L, bool EQ21>
static int launch_kl(const SwarmDev &S, uint32_t t, hipStream_t st)
{
    constexpr int per_block = kWaves * (64 / L);
    const uint32_t blocks = (S.n + per_block - 1) / per_block;
    if (t == 0)
        hipLaunchKernelGGL((k_stream<KIND, L, EQ21, true>), dim3(blocks), dim3(64 * kWaves), 0, st,
                           S, t);
    else
        hipLaunchKernelGGL((k_stream<KIND, L, EQ21, false>), dim3(blocks), dim3(64 * kWaves), 0,
                           st, S, t);
    return (int)hipGetLastError();
}

template <int KIND, bool EQ21>
static int launch_k(const SwarmDev &S, uint32_t t, uint32_t lanes, hipStream_t st)
{
    switch (lanes) {
    case 8: return launch_kl<KIND, 8, EQ21>(S, t, st);
    case 16: return launch_kl<KIND, 16, EQ21>(S, t, st);
    case 32: return launch_kl<KIND, 32, EQ21>(S, t, st);
    case 64: return launch_kl<KIND, 64, EQ21>(S, t, st);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_stream_generation(const SwarmDev &S, uint32_t t, uint32_t lanes, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const bool eq21 = S.order != 0;
    if (S.kind == OBJ_SPHERE)
        return eq21 ? launch_k<OBJ_SPHERE, true>(S, t, lanes, st)
                    : launch_k<OBJ_SPHERE, false>(S, t, lanes, st);
    if (S.kind == OBJ_RIPPLE)
        return eq21 ? launch_k<OBJ_RIPPLE, true>(S, t, lanes, st)
                    : launch_k<OBJ_RIPPLE, false>(S, t, lanes, st);
    return (int)hipErrorInvalidValue;
}

// Clears the whole trace ring: keys to "no gBest yet", counts to zero.  A
// kernel rather than a memset so the clear can sit inside a captured graph.
__global__ void k_fill_trace(unsigned long long *keys, uint32_t *cnt, uint32_t cap)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cap) {
        keys[j] = ~0ull;
        cnt[j] = 0u;
    }
}

int launch_fill_trace(const SwarmDev &S, void *stream)
{
    const uint32_t blocks = (S.trace_cap + 255u) / 256u;
    hipLaunchKernelGGL(k_fill_trace, dim3(blocks), dim3(256), 0, (hipStream_t)stream, S.keys,
                       S.cnt, S.trace_cap);
    return (int)hipGetLastError();
}

// The word of every (particle, variable) at generation t, as the kernels draw it.
__global__ void k_debug_rng(SwarmDev S, uint32_t t, uint32_t *out)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = (uint64_t)S.n * S.chunks;
    if (e >= total) return;
    const uint32_t i = (uint32_t)(e / S.chunks), c = (uint32_t)(e % S.chunks);
    const uint4 k = words4(S, c, i, t);
    const uint32_t v[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t j = 4u * c + q;
        if (j < S.d) out[(uint64_t)i * S.d + j] = v[q];
    }
}

int launch_debug_rng(const SwarmDev &S, uint32_t t, uint32_t *out, void *stream)
{
    const uint64_t total = (uint64_t)S.n * S.chunks;
    const uint64_t blocks = (total + 255u) / 256u;
    hipLaunchKernelGGL(k_debug_rng, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, S,
                       t, out);
    return (int)hipGetLastError();
}

}  // namespace sso
