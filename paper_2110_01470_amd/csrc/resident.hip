// RESIDENT engine: a swarm small enough for one workgroup's registers runs
// all requested generations in one launch.
//
// A generation of Algorithm 2 on a swarm like N=100, D=30 is 3,000 variable
// updates -- far too little to hide a kernel launch.  Here every lane owns
// one 4-float chunk of one particle (L lanes per particle, L = chunks rounded
// up to a power of two), keeps X and P of that chunk in registers, and only
// gBest and the argmin travel through LDS.  Per generation: Eq. (2.1) select
// and objective terms in registers, an L-lane butterfly for the fitness, the
// strict pBest test of Algorithm 3, a wave then workgroup minimum of the
// (fitness, index) key for Algorithm 4, and the winning particle's lanes copy
// its pBest into the LDS gBest row.  Two barriers per generation.
//
// Per lane the fitness is summed in the same order as the STREAM kernel with
// the same L (one chunk per lane, then the butterfly), so both engines take
// identical decisions.  On exit the state is written back with every pBest
// in row 0 and every position in row 1.
#include "sso_device.hpp"

namespace sso {

constexpr int kResidentMaxThreads = 1024;
constexpr int kResidentMaxWaves = kResidentMaxThreads / 64;

static uint32_t resident_lanes(uint32_t d)
{
    const uint32_t chunks = (d + 3) / 4;
    uint32_t L = 8;
    while (L < chunks) L <<= 1;
    return L;
}

bool resident_fits(uint32_t n, uint32_t d, int kind)
{
    if (kind != OBJ_SPHERE && kind != OBJ_RIPPLE) return false;
    const uint32_t L = resident_lanes(d);
    return L <= 64 && (uint64_t)n * L <= (uint64_t)kResidentMaxThreads;
}

template <int KIND, int L, bool EQ21>
__global__ __launch_bounds__(kResidentMaxThreads) void k_resident(SwarmDev S, uint32_t t_first,
                                                                 uint32_t generations)
{
    __shared__ f4 s_g[kDenseMaxD / 4];
    __shared__ unsigned long long s_key[kResidentMaxWaves];
    __shared__ uint32_t s_cnt[kResidentMaxWaves];

    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t nwaves = blockDim.x >> 6;
    const uint32_t c = threadIdx.x % L;          // this lane's chunk
    const uint32_t i = threadIdx.x / L;          // this lane's particle
    const bool valid = i < S.n;
    const bool owns = valid && c < S.chunks;     // lane holds real variables

    // Load the state of generation t_first - 1.
    f4 xv = f4{0.f, 0.f, 0.f, 0.f}, pv = xv, sv = xv, wv = xv;
    float fp = 0.0f;
    if (valid) {
        const uint32_t st = S.st[i];
        const uint32_t prow = st & ST_ROW;
        fp = S.fp[i];
        if (owns) {
            // An aliased position is the pBest row itself; selecting the row
            // pointer (not the loaded value) keeps both loads in registers.
            const size_t off = (size_t)i * S.stride;
            const float *prow_ptr = S.rows + prow * S.buf + off;
            const float *xrow_ptr = (st & ST_ALIAS) ? prow_ptr : S.rows + (1u - prow) * S.buf + off;
            pv = reinterpret_cast<const f4 *>(prow_ptr)[c];
            xv = reinterpret_cast<const f4 *>(xrow_ptr)[c];
        }
    }
    if (c < S.chunks) {
        sv = reinterpret_cast<const f4 *>(S.s)[c];
        if (KIND == OBJ_RIPPLE) wv = reinterpret_cast<const f4 *>(S.w)[c];
    }
    {
        // gBest of generation t_first - 1 from its sub-slot group; also
        // records that generation in the trace ring.
        __shared__ unsigned long long s_first;
        if (threadIdx.x < 64u) {
            const uint32_t g = (t_first - 1u) % kGroups;
            unsigned long long k = *sub_key(S, g, lane);
            uint32_t cc = *sub_cnt(S, g, lane);
            k = wave_min_u64(k);
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) cc += __shfl_xor(cc, m, 64);
            if (lane == 0) {
                s_first = k;
                S.keys[(t_first - 1u) % S.trace_cap] = k;
                S.cnt[(t_first - 1u) % S.trace_cap] = cc;
            }
        }
        __syncthreads();
        const unsigned long long gk = s_first;
        const uint32_t glow = (uint32_t)gk;
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        const f4 *grow = reinterpret_cast<const f4 *>(S.rows + (size_t)(glow & 1u) * S.buf +
                                                      (size_t)gidx * S.stride);
        for (uint32_t q = threadIdx.x; q < S.chunks; q += blockDim.x) s_g[q] = grow[q];
    }
    __syncthreads();

    for (uint32_t gen = 0; gen < generations; ++gen) {
        const uint32_t t = t_first + gen;
        float acc = 0.0f;
        if (owns) {
            const uint4 k = words4(S, c, i, t);
            xv = select4<EQ21>(S, k, s_g[c], pv, xv);
            acc += terms4<KIND>(xv, sv, wv, 4u * c, S.d);
        }
#pragma unroll
        for (int m = L / 2; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        const bool improved = valid && improves(acc, fp);
        if (improved) {
            pv = xv;
            fp = acc;
        }
        unsigned long long key = valid ? gbest_key(fp, i, 0u) : ~0ull;
        // Keys are equal within a particle's lanes, so the masks from L up
        // suffice; a few permutes are cheaper here than the full DPP minimum.
#pragma unroll
        for (int m = 32; m >= L; m >>= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)key, m, 64);
            const uint32_t hi = __shfl_xor((uint32_t)(key >> 32), m, 64);
            key = min_u64(key, ((unsigned long long)hi << 32) | lo);
        }
        const uint32_t cnt = (uint32_t)__popcll(__ballot(improved && c == 0));
        if (lane == 0) {
            s_key[wave] = key;
            s_cnt[wave] = cnt;
        }
        __syncthreads();
        unsigned long long best = s_key[0];
        for (uint32_t w = 1; w < nwaves; ++w) best = min_u64(best, s_key[w]);
        const uint32_t gidx = (uint32_t)best >> 1;
        if (owns && i == gidx) s_g[c] = pv;
        if (threadIdx.x == 0) {
            uint32_t total = 0;
            for (uint32_t w = 0; w < nwaves; ++w) total += s_cnt[w];
            const uint32_t slot = t % S.trace_cap;
            S.keys[slot] = best;
            S.cnt[slot] = total;
        }
        __syncthreads();
    }

    // Write back: pBest in row 0, position in row 1, no aliasing.
    if (valid) {
        const size_t off = (size_t)i * S.stride;
        if (owns) {
            reinterpret_cast<f4 *>(S.rows + off)[c] = pv;
            reinterpret_cast<f4 *>(S.rows + S.buf + off)[c] = xv;
        }
        if (c == 0) {
            S.st[i] = 0u;
            S.fp[i] = fp;
        }
    }
    // Leave the last generation's result where a following generation (and
    // the host) looks for it: sub-slot 0 of its group; clear the other groups.
    if (threadIdx.x < 64u) {
        const uint32_t tl = t_first + generations - 1u;
        const unsigned long long best = S.keys[tl % S.trace_cap];
        const uint32_t total = S.cnt[tl % S.trace_cap];
        for (uint32_t g = 0; g < kGroups; ++g) {
            const bool mine = g == tl % kGroups && lane == 0;
            *sub_key(S, g, lane) = mine ? best : ~0ull;
            *sub_cnt(S, g, lane) = mine ? total : 0u;
        }
    }
}

template <int KIND, bool EQ21>
static void launch_k(const SwarmDev &S, uint32_t t_first, uint32_t gens, dim3 block, hipStream_t st)
{
    switch (resident_lanes(S.d)) {
    case 8:
        hipLaunchKernelGGL((k_resident<KIND, 8, EQ21>), dim3(1), block, 0, st, S, t_first, gens);
        break;
    case 16:
        hipLaunchKernelGGL((k_resident<KIND, 16, EQ21>), dim3(1), block, 0, st, S, t_first, gens);
        break;
    case 32:
        hipLaunchKernelGGL((k_resident<KIND, 32, EQ21>), dim3(1), block, 0, st, S, t_first, gens);
        break;
    default:
        hipLaunchKernelGGL((k_resident<KIND, 64, EQ21>), dim3(1), block, 0, st, S, t_first, gens);
        break;
    }
}

int launch_resident(const SwarmDev &S, uint32_t t_first, uint32_t generations, void *stream)
{
    if (t_first == 0 || !resident_fits(S.n, S.d, S.kind)) return (int)hipErrorInvalidValue;
    const uint32_t threads = S.n * resident_lanes(S.d);
    const dim3 block((threads + 63u) / 64u * 64u);
    hipStream_t st = (hipStream_t)stream;
    const bool eq21 = S.order != 0;
    if (S.kind == OBJ_SPHERE) {
        if (eq21) launch_k<OBJ_SPHERE, true>(S, t_first, generations, block, st);
        else launch_k<OBJ_SPHERE, false>(S, t_first, generations, block, st);
    } else {
        if (eq21) launch_k<OBJ_RIPPLE, true>(S, t_first, generations, block, st);
        else launch_k<OBJ_RIPPLE, false>(S, t_first, generations, block, st);
    }
    return (int)hipGetLastError();
}

}  // namespace sso
