// RESIDENT engine: a swarm small enough for one workgroup's registers runs
// all requested generations in one launch.
//
// A generation of Algorithm 2 on a swarm like N=100, D=30 is 3,000 variable
// updates -- far too little to hide a kernel launch.  Here every lane owns
// one 4-float chunk of one particle (L lanes per particle, L = chunks rounded
// up to a power of two), keeps X and P of that chunk in registers, and only
// gBest and the argmin travel through LDS.  Per generation: Eq. (2.1) select
// and objective terms in registers, an L-lane butterfly for the fitness, the
// strict pBest test of Algorithm 3, a wave minimum of the (fitness, index)
// key whose particle posts its pBest row to LDS, one barrier, and the
// workgroup minimum over the posted keys for Algorithm 4, whose row is the
// next gBest.
//
// Per lane the fitness is summed in the same order as the STREAM kernel with
// the same L (one chunk per lane, then the butterfly), so both engines take
// identical decisions.  On exit the state is written back with every pBest
// in row 0 and every position in row 1.
#include "sso_device.hpp"
#include "sso_host.hpp"

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

// Table 3.2's functions: the STREAM engine's lanes per particle (its FP32
// rule), one chunk per lane, up to kPaperMaxSlots particles per thread (with
// more, the compiler no longer unrolls the loop over a thread's particles
// and their registers go to scratch memory; one workgroup would not beat a
// launch per generation there anyway).
constexpr uint32_t kPaperMaxSlots = 4;

namespace host {
uint32_t resident_paper_slots(uint32_t n, uint32_t d)
{
    const uint32_t L = stream_lanes(d, STORE_F32);
    const uint32_t chunks = (d + 3) / 4;
    if (chunks > L || n == 0) return 0;
    const uint32_t groups = kResidentMaxThreads / L;
    const uint32_t slots = (n + groups - 1) / groups;
    return slots <= kPaperMaxSlots ? slots : 0;
}
}  // namespace host

bool resident_fits(uint32_t n, uint32_t d, int kind)
{
    if (is_paper_kind(kind)) return host::resident_paper_slots(n, d) != 0;
    if (kind != OBJ_SPHERE && kind != OBJ_RIPPLE) return false;
    const uint32_t L = resident_lanes(d);
    return L <= 64 && (uint64_t)n * L <= (uint64_t)kResidentMaxThreads;
}

// x op x' where x' is x of the lane that the row-local DPP control CTRL names.
template <int CTRL>
__device__ __forceinline__ float dpp_partner(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// The L-lane butterfly of paper_finish (partners at lane distance xor m,
// m = L/2 down to 1; own value first) with the short distances as DPP moves
// instead of LDS permutes.  m = 8 is row_ror:8 (lane l + 8 mod 16 is l ^ 8);
// m = 4 is row_ror:4, whose source l + 4 mod 16 is l ^ 4 or (l ^ 4) ^ 8, and
// after the m = 8 step lanes l and l ^ 8 hold the same value; m = 2 and 1
// are quad permutes.  Every lane adds exactly the value the permute would
// have brought, so the sums are bit for bit those of paper_finish.
template <class Op>
__device__ __forceinline__ float lane_fold(float x, uint32_t L, Op op)
{
    if (L > 32u) x = op(x, __shfl_xor(x, 32, 64));
    if (L > 16u) x = op(x, __shfl_xor(x, 16, 64));
    if (L > 8u) x = op(x, dpp_partner<0x128>(x));  // row_ror:8
    if (L > 4u) x = L > 8u ? op(x, dpp_partner<0x124>(x))  // row_ror:4
                           : op(x, __shfl_xor(x, 4, 64));
    if (L > 2u) x = op(x, dpp_partner<0x4E>(x));    // quad_perm(2, 3, 0, 1)
    if (L > 1u) x = op(x, dpp_partner<0xB1>(x));    // quad_perm(1, 0, 3, 2)
    return x;
}

__device__ __forceinline__ float paper_fitness(PaperAcc q, uint32_t L, uint32_t d, int kind)
{
#pragma clang fp contract(off)
    q.a = lane_fold(q.a, L, [](float u, float v) { return u + v; });
    if (kind == OBJ_F1 + 5) q.b = lane_fold(q.b, L, [](float u, float v) { return u + v; });
    if (kind == OBJ_F1 + 6) q.p = lane_fold(q.p, L, [](float u, float v) { return u * v; });
    return paper_finish(q, 1u, d, kind);  // sums complete: only the function's last step
}

// Table 3.2's functions in one workgroup.  Lane ln of lane group g (L lanes,
// the STREAM engine's count for this d, so chunk ln of every particle the
// group holds) keeps chunk ln of particles g, g + G, ..., g + (P-1) G
// (G groups) in registers, and evaluates each particle exactly as the STREAM
// kernel does with the same L: paper_chunk on chunk ln, then paper_finish
// over the L lanes.  So the two engines sum every fitness in the same order
// and take the same decisions.
//
// One barrier per generation: before it, every wave posts its own best key
// and its best particle's pBest row in LDS and adds its improved count to
// the generation's counter; after it, every wave takes the minimum of the
// posted keys and reads the winning wave's row as gBest.  The posts and
// counters alternate between two buffers by generation, so a generation's
// posts never overwrite the ones the previous generation is still reading
// (every read of buffer b happens before the reader's next barrier, every
// later write of b after it).  The lane sums are those of paper_finish with
// the short distances as DPP moves (lane_fold).  The lane count LT (8, 16, 32
// or 64, the STREAM engine's for the swarm) is a template parameter, so the
// folds and lane masks are constants.
template <int KIND, bool EQ21, int P, int LT>
__global__ __launch_bounds__(kResidentMaxThreads) void k_resident_paper(SwarmDev S, uint32_t t_first,
                                                                       uint32_t generations)
{
    static_assert(LT >= 8 && LT <= 64 && (LT & (LT - 1)) == 0, "lane count");
    __shared__ f4 s_row[2][kResidentMaxWaves][64];
    __shared__ unsigned long long s_key[2][kResidentMaxWaves];
    __shared__ uint32_t s_cnt[2];  // improved pBests of the generation (LDS atomics)

    constexpr uint32_t L = LT;
    constexpr uint32_t lsh = (uint32_t)__builtin_ctz(L);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t nwaves = blockDim.x >> 6;
    const uint32_t ln = threadIdx.x & (L - 1u);
    const uint32_t g = threadIdx.x >> lsh;
    const uint32_t G = blockDim.x >> lsh;
    const bool has_chunk = ln < S.chunks;

    f4 xv[P], pv[P];
    float fp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        xv[p] = pv[p] = f4{0.f, 0.f, 0.f, 0.f};
        fp[p] = 0.0f;
        const uint32_t i = g + (uint32_t)p * G;
        if (i < S.n) {
            const uint32_t st = S.st[i];
            const uint32_t prow = st & ST_ROW;
            fp[p] = S.fp[i];
            if (has_chunk) {
                const size_t off = (size_t)i * S.stride;
                const float *prow_ptr = S.rows + prow * S.buf + off;
                const float *xrow_ptr = (st & ST_ALIAS) ? prow_ptr : S.rows + (1u - prow) * S.buf + off;
                pv[p] = reinterpret_cast<const f4 *>(prow_ptr)[ln];
                xv[p] = reinterpret_cast<const f4 *>(xrow_ptr)[ln];
            }
        }
    }
    // gBest of generation t_first - 1 from its sub-slot group (every wave
    // reduces the 64 sub-slots itself); wave 0 records that generation in the
    // trace ring.
    // The latest generation's key (wave-uniform) and improved count (thread
    // 0) stay in registers for the hand-off at the end.
    f4 gv = f4{0.f, 0.f, 0.f, 0.f};
    unsigned long long last_key;
    uint32_t last_cnt = 0;
    {
        const uint32_t gr = (t_first - 1u) % kGroups;
        const unsigned long long k0 = wave_min_u64(*sub_key(S, gr, lane));
        last_key = k0;
        if (threadIdx.x < 64u) {
            uint32_t cc = *sub_cnt(S, gr, lane);
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) cc += __shfl_xor(cc, m, 64);
            last_cnt = cc;
            if (lane == 0) {
                S.keys[(t_first - 1u) % S.trace_cap] = k0;
                S.cnt[(t_first - 1u) % S.trace_cap] = cc;
                s_cnt[0] = s_cnt[1] = 0u;
            }
        }
        const uint32_t glow = (uint32_t)k0;
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        if (has_chunk)
            gv = reinterpret_cast<const f4 *>(S.rows + (size_t)(glow & 1u) * S.buf +
                                             (size_t)gidx * S.stride)[ln];
    }
    __syncthreads();  // counters cleared

    uint32_t slot = t_first % S.trace_cap;  // trace ring slot of generation t (thread 0)
    for (uint32_t gen = 0; gen < generations; ++gen) {
        const uint32_t t = t_first + gen;
        const uint32_t b = gen & 1u;
        unsigned long long key = ~0ull, kp[P];
        uint32_t imp = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t i = g + (uint32_t)p * G;
            kp[p] = ~0ull;
            bool improved = false;
            if (i < S.n) {
                PaperAcc q;
                if (has_chunk) {
                    const uint4 k = words4(S, ln, i, t);
                    xv[p] = select4<EQ21>(S, k, gv, pv[p], xv[p]);
                    paper_chunk(q, xv[p], ln, S.d, L, ln, KIND);
                }
                const float f = paper_fitness(q, L, S.d, KIND);
                improved = improves(f, fp[p]);
                if (improved) {
                    pv[p] = xv[p];
                    fp[p] = f;
                }
                kp[p] = gbest_key(fp[p], i, 0u);
                key = min_u64(key, kp[p]);
            }
            imp += (uint32_t)__popcll(__ballot(improved && ln == 0u));
        }
        key = wave_min_u64(key);
        // The wave's best particle posts its pBest row (its key is unique).
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (has_chunk && kp[p] == key) s_row[b][wave][ln] = pv[p];
        if (lane == 0) {
            s_key[b][wave] = key;
            if (imp) atomicAdd(&s_cnt[b], imp);
        }
        __syncthreads();
        // At most 16 posted keys: lanes 0..15, one DPP row.
        static_assert(kResidentMaxWaves <= 16, "posted keys must fit one DPP row");
        const unsigned long long posted = lane < nwaves ? s_key[b][lane] : ~0ull;
        unsigned long long rmin = dpp_min_u64<0xB1>(posted);  // quad_perm(1, 0, 3, 2)
        rmin = dpp_min_u64<0x4E>(rmin);                       // quad_perm(2, 3, 0, 1)
        rmin = dpp_min_u64<0x141>(rmin);                      // row_half_mirror
        rmin = dpp_min_u64<0x140>(rmin);                      // row_mirror
        const unsigned long long best = readlane_u64(rmin, 0);
        const uint32_t bw = (uint32_t)__builtin_ctzll(__ballot(posted == best));
        if (has_chunk) gv = s_row[b][bw][ln];
        last_key = best;
        if (threadIdx.x == 0) {
            // Cleared for generation gen + 2, whose adds come after this
            // thread's next barrier.
            last_cnt = s_cnt[b];
            s_cnt[b] = 0u;
            S.keys[slot] = best;
            S.cnt[slot] = last_cnt;
            slot = slot + 1u == S.trace_cap ? 0u : slot + 1u;
        }
    }

    // Write back: pBest in row 0, position in row 1, no aliasing.
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t i = g + (uint32_t)p * G;
        if (i < S.n) {
            const size_t off = (size_t)i * S.stride;
            if (has_chunk) {
                reinterpret_cast<f4 *>(S.rows + off)[ln] = pv[p];
                reinterpret_cast<f4 *>(S.rows + S.buf + off)[ln] = xv[p];
            }
            if (ln == 0) {
                S.st[i] = 0u;
                S.fp[i] = fp[p];
            }
        }
    }
    // The last generation's result in sub-slot 0 of its group; the other
    // groups cleared.
    if (threadIdx.x < 64u) {
        const uint32_t tl = t_first + generations - 1u;
        for (uint32_t gr = 0; gr < kGroups; ++gr) {
            const bool mine = gr == tl % kGroups && lane == 0;
            *sub_key(S, gr, lane) = mine ? last_key : ~0ull;
            *sub_cnt(S, gr, lane) = mine ? last_cnt : 0u;
        }
    }
}

template <int KIND, bool EQ21, int LT>
static void launch_paper_lanes(const SwarmDev &S, uint32_t slots, uint32_t t_first, uint32_t gens,
                               dim3 block, hipStream_t st)
{
    switch (slots) {
    case 1: hipLaunchKernelGGL((k_resident_paper<KIND, EQ21, 1, LT>), dim3(1), block, 0, st, S, t_first, gens); break;
    case 2: hipLaunchKernelGGL((k_resident_paper<KIND, EQ21, 2, LT>), dim3(1), block, 0, st, S, t_first, gens); break;
    case 3: hipLaunchKernelGGL((k_resident_paper<KIND, EQ21, 3, LT>), dim3(1), block, 0, st, S, t_first, gens); break;
    default: hipLaunchKernelGGL((k_resident_paper<KIND, EQ21, 4, LT>), dim3(1), block, 0, st, S, t_first, gens); break;
    }
}

// S.lanes is the STREAM engine's FP32 lane count, a power of two in [8, 64]
// (checked by the caller).
template <int KIND, bool EQ21>
static void launch_paper_slots(const SwarmDev &S, uint32_t slots, uint32_t t_first, uint32_t gens,
                               dim3 block, hipStream_t st)
{
    switch (S.lanes) {
    case 8: launch_paper_lanes<KIND, EQ21, 8>(S, slots, t_first, gens, block, st); break;
    case 16: launch_paper_lanes<KIND, EQ21, 16>(S, slots, t_first, gens, block, st); break;
    case 32: launch_paper_lanes<KIND, EQ21, 32>(S, slots, t_first, gens, block, st); break;
    default: launch_paper_lanes<KIND, EQ21, 64>(S, slots, t_first, gens, block, st); break;
    }
}

// One kernel per function: with the function fixed at compile time its
// terms are straight-line code (16 % faster on Rosenbrock than one kernel
// switching on the kind at run time).
template <bool EQ21>
static void launch_paper_kind(const SwarmDev &S, uint32_t slots, uint32_t t_first, uint32_t gens,
                              dim3 block, hipStream_t st)
{
    switch (S.kind) {
    case OBJ_F1 + 0: launch_paper_slots<OBJ_F1 + 0, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 1: launch_paper_slots<OBJ_F1 + 1, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 2: launch_paper_slots<OBJ_F1 + 2, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 3: launch_paper_slots<OBJ_F1 + 3, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 4: launch_paper_slots<OBJ_F1 + 4, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 5: launch_paper_slots<OBJ_F1 + 5, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 6: launch_paper_slots<OBJ_F1 + 6, EQ21>(S, slots, t_first, gens, block, st); break;
    case OBJ_F1 + 7: launch_paper_slots<OBJ_F1 + 7, EQ21>(S, slots, t_first, gens, block, st); break;
    default: launch_paper_slots<OBJ_F1 + 8, EQ21>(S, slots, t_first, gens, block, st); break;
    }
}

template <int KIND, int L, bool EQ21>
__global__ __launch_bounds__(kResidentMaxThreads) void k_resident(SwarmDev S, uint32_t t_first,
                                                                 uint32_t generations)
{
    // Per generation parity b: each wave's minimum key and its best
    // particle's pBest row, and the generation's improved count (see
    // k_resident_paper for why two buffers make one barrier enough).
    __shared__ f4 s_row[2][kResidentMaxWaves][64];
    __shared__ unsigned long long s_key[2][kResidentMaxWaves];
    __shared__ uint32_t s_cnt[2];
    static_assert(L <= 64, "a particle's chunks must fit one wave");

    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t nwaves = blockDim.x >> 6;
    const uint32_t c = threadIdx.x % L;          // this lane's chunk
    const uint32_t i = threadIdx.x / L;          // this lane's particle
    const bool valid = i < S.n;
    const bool owns = valid && c < S.chunks;     // lane holds real variables

    // Load the state of generation t_first - 1.
    f4 xv = f4{0.f, 0.f, 0.f, 0.f}, pv = xv, sv = xv, wv = xv, gv = xv;
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
    // gBest of generation t_first - 1 from its sub-slot group (every wave
    // reduces the 64 sub-slots itself); wave 0 records that generation in the
    // trace ring.  The latest generation's key (wave-uniform) and improved
    // count (thread 0) stay in registers for the hand-off at the end.
    unsigned long long last_key;
    uint32_t last_cnt = 0;
    {
        const uint32_t gr = (t_first - 1u) % kGroups;
        const unsigned long long k0 = wave_min_u64(*sub_key(S, gr, lane));
        last_key = k0;
        if (threadIdx.x < 64u) {
            uint32_t cc = *sub_cnt(S, gr, lane);
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) cc += __shfl_xor(cc, m, 64);
            last_cnt = cc;
            if (lane == 0) {
                S.keys[(t_first - 1u) % S.trace_cap] = k0;
                S.cnt[(t_first - 1u) % S.trace_cap] = cc;
                s_cnt[0] = s_cnt[1] = 0u;
            }
        }
        const uint32_t glow = (uint32_t)k0;
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        if (c < S.chunks)
            gv = reinterpret_cast<const f4 *>(S.rows + (size_t)(glow & 1u) * S.buf +
                                             (size_t)gidx * S.stride)[c];
    }
    __syncthreads();  // counters cleared

    uint32_t slot = t_first % S.trace_cap;  // trace ring slot of generation t (thread 0)
    for (uint32_t gen = 0; gen < generations; ++gen) {
        const uint32_t b = gen & 1u;
        float acc = 0.0f;
        if (owns) {
            const uint4 k = words4(S, c, i, t_first + gen);
            xv = select4<EQ21>(S, k, gv, pv, xv);
            acc += terms4<KIND>(xv, sv, wv, 4u * c, S.d);
        }
        acc = lane_fold(acc, L, [](float u, float v) { return u + v; });
        const bool improved = valid && improves(acc, fp);
        if (improved) {
            pv = xv;
            fp = acc;
        }
        const unsigned long long mine = valid ? gbest_key(fp, i, 0u) : ~0ull;
        // Keys are equal within a particle's lanes, so the masks from L up
        // suffice; a few permutes are cheaper here than the full DPP minimum.
        unsigned long long key = mine;
#pragma unroll
        for (int m = 32; m >= L; m >>= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)key, m, 64);
            const uint32_t hi = __shfl_xor((uint32_t)(key >> 32), m, 64);
            key = min_u64(key, ((unsigned long long)hi << 32) | lo);
        }
        // The wave's best particle posts its pBest row (its key is unique).
        if (c < S.chunks && mine == key) s_row[b][wave][c] = pv;
        const uint32_t cnt = (uint32_t)__popcll(__ballot(improved && c == 0));
        if (lane == 0) {
            s_key[b][wave] = key;
            if (cnt) atomicAdd(&s_cnt[b], cnt);
        }
        __syncthreads();
        // At most 16 posted keys: lanes 0..15, one DPP row.
        const unsigned long long posted = lane < nwaves ? s_key[b][lane] : ~0ull;
        unsigned long long rmin = dpp_min_u64<0xB1>(posted);  // quad_perm(1, 0, 3, 2)
        rmin = dpp_min_u64<0x4E>(rmin);                       // quad_perm(2, 3, 0, 1)
        rmin = dpp_min_u64<0x141>(rmin);                      // row_half_mirror
        rmin = dpp_min_u64<0x140>(rmin);                      // row_mirror
        const unsigned long long best = readlane_u64(rmin, 0);
        const uint32_t bw = (uint32_t)__builtin_ctzll(__ballot(posted == best));
        if (c < S.chunks) gv = s_row[b][bw][c];
        last_key = best;
        if (threadIdx.x == 0) {
            // Cleared for generation gen + 2, whose adds come after this
            // thread's next barrier.
            last_cnt = s_cnt[b];
            s_cnt[b] = 0u;
            S.keys[slot] = best;
            S.cnt[slot] = last_cnt;
            slot = slot + 1u == S.trace_cap ? 0u : slot + 1u;
        }
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
        for (uint32_t g = 0; g < kGroups; ++g) {
            const bool own = g == tl % kGroups && lane == 0;
            *sub_key(S, g, lane) = own ? last_key : ~0ull;
            *sub_cnt(S, g, lane) = own ? last_cnt : 0u;
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
    // No launch for no generations: the kernels' hand-off at the end assumes
    // at least one generation's barrier lies between it and the first reads.
    if (generations == 0) return (int)hipSuccess;
    if (is_paper_kind(S.kind)) {
        // The lanes must be the STREAM engine's FP32 count (the context sets
        // them so); the gBest row is staged in 64 chunks of LDS at most.
        if (S.lanes != host::stream_lanes(S.d, STORE_F32) || S.storage != STORE_F32 || S.chunks > 64u ||
            (S.lanes != 8u && S.lanes != 16u && S.lanes != 32u && S.lanes != 64u))
            return (int)hipErrorInvalidValue;
        // One particle per group when they all fit; otherwise the full
        // workgroup, so that particle i sits in group i mod G of slot i / G:
        // the slots fill in order and the partly filled last one spreads its
        // waves over the SIMDs (waves w, w + 4, ... share one), which keeps
        // the busiest SIMD's share of particle slots near the mean.
        const uint32_t slots = host::resident_paper_slots(S.n, S.d);
        const dim3 block(slots == 1u ? (S.n * S.lanes + 63u) / 64u * 64u : (uint32_t)kResidentMaxThreads);
        hipStream_t st = (hipStream_t)stream;
        if (S.order != 0) launch_paper_kind<true>(S, slots, t_first, generations, block, st);
        else launch_paper_kind<false>(S, slots, t_first, generations, block, st);
        return (int)hipGetLastError();
    }
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
