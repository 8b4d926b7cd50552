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
constexpr int kInFlight = 4;  // chunks whose loads a lane issues before computing

template <int KIND, int L, bool EQ21, bool INIT>
__global__ __launch_bounds__(64 * kWaves) void k_stream(SwarmDev S, uint32_t t)
{
    constexpr int G = 64 / L;  // particles per wave
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t ln = lane % L;
    const uint32_t i = (blockIdx.x * kWaves + wave) * G + lane / L;
    const bool valid = i < S.n;

    uint32_t prow = 0;
    bool alias = true;
    float fpi = 0.0f;
    if (!INIT && valid) {
        const uint32_t st = S.st[i];
        fpi = S.fp[i];
        prow = st & ST_ROW;
        alias = (st & ST_ALIAS) != 0u;
    }
    const size_t ioff = (size_t)(valid ? i : 0u) * S.dp;
    const f4 *p4 = reinterpret_cast<const f4 *>(S.rows + prow * S.buf + ioff);
    // INIT writes the pBest row (row 0); a generation writes the other row.
    f4 *x4 = reinterpret_cast<f4 *>(S.rows + (INIT ? 0u : (1u - prow)) * S.buf + ioff);
    // The position is read from the pBest row itself when aliased.
    const f4 *xsrc = alias ? p4 : x4;
    const f4 *s4 = reinterpret_cast<const f4 *>(S.s);
    const f4 *w4 = reinterpret_cast<const f4 *>(S.w);
    const f4 zero = f4{0.f, 0.f, 0.f, 0.f};

    // The first batch of pBest / position loads does not depend on gBest:
    // issue it before the start-of-generation barrier.
    f4 pv[kInFlight], xv[kInFlight], gv[kInFlight];
    if (!INIT && valid) {
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const uint32_t c = ln + u * L;
            if (c < S.chunks) {
                pv[u] = p4[c];
                xv[u] = xsrc[c];
            }
        }
    }
    // gBest of the previous generation (unused at t == 0).
    const f4 *g4 = nullptr;
    if constexpr (!INIT) {
        const uint32_t glow = (uint32_t)generation_begin(S, t);
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        g4 = reinterpret_cast<const f4 *>(S.rows + (size_t)(glow & 1u) * S.buf + (size_t)gidx * S.dp);
    }

    float acc = 0.0f;
    if (valid) {
        for (uint32_t c0 = ln; c0 < S.chunks; c0 += kInFlight * L) {
            if constexpr (!INIT) {
#pragma unroll
                for (int u = 0; u < kInFlight; ++u) {
                    const uint32_t c = c0 + u * L;
                    if (c < S.chunks) {
                        if (c0 != ln) {  // later batches: rows not issued yet
                            pv[u] = p4[c];
                            xv[u] = xsrc[c];
                        }
                        gv[u] = g4[c];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) {
                const uint32_t c = c0 + u * L;
                if (c < S.chunks) {
                    const uint4 k = words4(S, c, i, t);
                    f4 xn;
                    if constexpr (INIT)
                        xn = init4(S, k);
                    else
                        xn = select4<EQ21>(S, k, gv[u], pv[u], xv[u]);
                    x4[c] = xn;
                    const f4 wv = (KIND == OBJ_RIPPLE) ? w4[c] : zero;
                    acc += terms4<KIND>(xn, s4[c], wv, 4u * c, S.d);
                }
            }
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

    generation_commit<kWaves>(S, t, key, (improved && ln == 0) ? 1u : 0u);
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
