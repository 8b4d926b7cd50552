// The fused generation body of the STREAM engine, shared by the one-swarm
// kernel (gen_stream.hip) and the batched kernel (gen_batch.hip).
//
// One generation of Algorithm 2 in a single pass over the state: each group
// of L lanes owns one particle and walks its row chunk by chunk (chunk c,
// c + L, ...; a chunk is 4 variables), so a wave's loads cover L contiguous
// chunks of a row.  Per chunk a lane draws one Philox block (four words, one
// per variable, Sec. 3.1), picks the four new values by Eq. (2.1), writes
// them, and accumulates the objective terms.  The L partial sums meet in a
// butterfly; every lane of the group then holds the same fitness, takes the
// pBest decision of Algorithm 3 (strict <), and the workgroup folds its
// (fitness, index) keys into the generation's gBest sub-slot (Algorithm 4).
//
// With t == 0 the same body is the initialisation (kernel (I), Sec. 2.3.1):
// X^0 is drawn uniformly from the generation-0 words, written as the pBest
// row, and scored.
#pragma once

#include "sso_device.hpp"

namespace sso {

constexpr int kWaves = (int)kStreamWaves;

// Words a chunk of 4 variables takes in a row.
template <class Store>
constexpr uint32_t chunk_words() { return sizeof(typename Store::T) == 16 && !Store::kPacked ? 4u : 3u; }

// Dynamic LDS of the staged kernels: shift, ripple weights, gBest row.
constexpr uint32_t kStageMaxChunks = 256;  // d <= 1024

// A guess at the low word (index << 1 | row) of generation t - 1's gBest key
// before that key is known: generation t - 2's, from the trace ring (written
// by workgroup 0 at the start of generation t - 1).  The gBest is usually
// the same particle in the same row from one generation to the next, and a
// pBest row is never written while a generation runs, so a kernel may load
// the guessed row early and keep it when the real key's low word is equal.
// Anything in the ring (even a cleared slot) names a row inside the
// workspace once the index is clamped to n - 1; cleared slots never match.
__device__ __forceinline__ uint32_t gbest_guess_low(const SwarmDev &S, uint32_t t)
{
    return t >= 2u ? (uint32_t)S.keys[(t - 2u) % S.trace_cap] : 0xFFFFFFFFu;
}

// Shift and weight arrays staged in LDS: ripple both, sphere the shift,
// Table 3.2's functions neither.
template <int KIND>
constexpr uint32_t staged_arrays() { return KIND == OBJ_RIPPLE ? 2u : is_paper_kind(KIND) ? 0u : 1u; }

template <int KIND, class Store>
inline size_t stage_bytes(const SwarmDev &S)
{
    return (size_t)S.chunks * 16u * staged_arrays<KIND>() + (size_t)S.chunks * chunk_words<Store>() * 4u;
}

// One generation t (the initialisation when INIT) for the particles of
// workgroup blk of swarm S, with L lanes per particle: the compile-time LT,
// or the power of two l when LT == 0 (the batched kernel, whose workgroups
// belong to swarms of different widths).
// RAGGED: d is not a multiple of 4, so the last chunk has padding columns.
// STAGE: the shift, the ripple weights and the gBest row are copied into LDS
// once per workgroup (dynamic LDS, see stage_bytes) and read from there, so
// the vector-memory path carries only the particle's own pBest and position.
// EARLY: the start of a generation is ordered for latency -- the gBest key
// is loaded before everything else, and a lane's first chunk is read from
// both rows without waiting for the state word (one dependent latency fewer;
// an aliased particle then reads one chunk more).  4 % faster on swarms
// small enough to be latency-bound (Table 3.2 functions, N <= 350, D = 50);
// the batched kernel, whose many short workgroups overlap one another, runs
// faster without it (567 vs 569-572 us per generation of the 512 swarms).
// With STAGE it also reads the guessed gBest row (gbest_guess_low) before
// the key arrives: another 3 % on those swarms (4.39 against 4.51 us at
// N = 350), none on ripple.
// WAVES: waves per workgroup (the batched kernel is built for 4 and 8).
template <int KIND, int LT, bool EQ21, bool INIT, bool RAGGED, bool STAGE, class Store,
          bool EARLY = true, int WAVES = kWaves>
__device__ __forceinline__ void stream_body(const SwarmDev &S, uint32_t t, uint32_t blk,
                                            uint32_t l)
{
    using T = typename Store::T;
    extern __shared__ f4 lds_dyn[];
    constexpr uint32_t CW = chunk_words<Store>();
    const uint32_t L = LT ? (uint32_t)LT : l;
    const uint32_t lsh = LT ? (uint32_t)__builtin_ctz((uint32_t)LT) : (uint32_t)__builtin_ctz(l);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t ln = lane & (L - 1u);
    // 64 / L particles per wave.
    const uint32_t i = ((blk * WAVES + wave) << (6u - lsh)) + (lane >> lsh);
    const bool valid = i < S.n;

    // With EARLY the gBest key load goes out first (see generation_key_load).
    unsigned long long gkey = ~0ull;
    if constexpr (!INIT && EARLY) gkey = generation_key_load(S, t);
    // The state word and pBest fitness; with EARLY the state is decoded only
    // after the first row loads below have gone out, which do not depend on it.
    uint32_t st = ST_ALIAS;  // pBest in row 0, position aliased (generation 0)
    float fpi = 0.0f;
    uint32_t prow = 0;
    bool alias = true;
    if (!INIT && valid) {
        st = S.st[i];
        fpi = S.fp[i];
        if constexpr (!EARLY) {
            prow = st & ST_ROW;
            alias = (st & ST_ALIAS) != 0u;
        }
    }
    uint32_t *rows = reinterpret_cast<uint32_t *>(S.rows);
    const size_t ioff = (size_t)(valid ? i : 0u) * S.stride;
    // This lane's first chunk of both rows, as stored (unpacked when the
    // chunk is computed): the same two loads as pBest and position, issued
    // without waiting for the state word that tells which is which.
    typename Store::R r0{}, r1{};
    if (EARLY && !INIT && valid && ln < S.chunks) {
        r0 = Store::load_raw(rows + ioff, ln);
        r1 = Store::load_raw(rows + S.buf + ioff, ln);
    }
    if constexpr (EARLY) {
        prow = st & ST_ROW;
        alias = (st & ST_ALIAS) != 0u;
    }
    const uint32_t *prow_ptr = rows + prow * S.buf + ioff;
    // INIT writes the pBest row (row 0); a generation writes the other row.
    uint32_t *xrow_ptr = rows + (INIT ? 0u : (1u - prow)) * S.buf + ioff;
    // The position is read from the pBest row itself when aliased.
    const uint32_t *xsrc = alias ? prow_ptr : xrow_ptr;
    const f4 *s4 = reinterpret_cast<const f4 *>(S.s);
    const f4 *w4 = reinterpret_cast<const f4 *>(S.w);
    const f4 zero = f4{0.f, 0.f, 0.f, 0.f};
    f4 *ls = lds_dyn;                                              // [chunks] shift
    f4 *lw = lds_dyn + S.chunks;                                   // [chunks] weights
    uint32_t *lg = reinterpret_cast<uint32_t *>(lds_dyn + staged_arrays<KIND>() * S.chunks);

    // Loads that do not depend on gBest go out before the start-of-generation
    // barrier: the shift and weights for staging.
    if constexpr (STAGE && !is_paper_kind(KIND)) {
        for (uint32_t q = tid; q < S.chunks; q += blockDim.x) {
            ls[q] = s4[q];
            if (KIND == OBJ_RIPPLE) lw[q] = w4[q];
        }
    }
    typename Store::R pr{}, xr{};
    if constexpr (EARLY) {
        pr = prow ? r1 : r0;
        xr = alias ? pr : (prow ? r0 : r1);
    } else if (!INIT && valid && ln < S.chunks) {
        pr = Store::load_raw(prow_ptr, ln);
        xr = Store::load_raw(xsrc, ln);
    }
    // gBest of the previous generation (unused at t == 0).
    const uint32_t *grow_ptr = nullptr;
    if constexpr (!INIT) {
        auto grow = [&](uint32_t low) {
            const uint32_t gidx = min(low >> 1, S.n - 1u);
            return rows + (size_t)(low & 1u) * S.buf + (size_t)gidx * S.stride;
        };
        // With EARLY the staged gBest row is first read from the guessed row
        // (gbest_guess_low) while the key is still on its way, and kept when
        // the key names the same row.
        constexpr uint32_t GQ = (kStageMaxChunks * 4u + 64u * WAVES - 1u) / (64u * WAVES);
        const uint32_t words = S.chunks * CW;
        uint32_t gpre[GQ];
        uint32_t guess = 0xFFFFFFFFu;
        if constexpr (EARLY && STAGE) {
            guess = gbest_guess_low(S, t);
            const uint32_t *gp = grow(guess);
#pragma unroll
            for (uint32_t k = 0; k < GQ; ++k) {
                const uint32_t q = tid + k * (64u * WAVES);
                gpre[k] = q < words ? gp[q] : 0u;
            }
        }
        const uint32_t glow = EARLY ? (uint32_t)generation_begin(S, t, blk, gkey)
                                    : (uint32_t)generation_begin(S, t, blk);
        grow_ptr = grow(glow);
        if constexpr (STAGE) {
            if (EARLY && glow == guess) {
#pragma unroll
                for (uint32_t k = 0; k < GQ; ++k) {
                    const uint32_t q = tid + k * (64u * WAVES);
                    if (q < words) lg[q] = gpre[k];
                }
            } else {
                for (uint32_t q = tid; q < words; q += blockDim.x) lg[q] = grow_ptr[q];
            }
        }
    }
    if constexpr (STAGE) __syncthreads();

    float acc = 0.0f;
    PaperAcc pacc;
    if (valid) {
        // Software pipeline: the next chunk's rows are requested before this
        // chunk is computed.
        for (uint32_t c = ln; c < S.chunks; c += L) {
            // The last iteration re-reads its own chunk (in bounds, unused),
            // so the load is unconditional and no register copies are needed.
            const uint32_t cn = (c + L < S.chunks) ? c + L : c;
            const T pc = Store::unpack(pr), xc = Store::unpack(xr);
            if (!INIT) {
                pr = Store::load_raw(prow_ptr, cn);
                xr = Store::load_raw(xsrc, cn);
            }
            const uint4 k = words4(S, c, i, t);
            T xn;
            if constexpr (INIT) {
                xn = Store::init(S, k);
            } else {
                const T g = STAGE ? Store::load(lg, c) : Store::load(grow_ptr, c);
                xn = Store::template select<EQ21>(S, k, g, pc, xc);
            }
            Store::store(xrow_ptr, c, xn);
            const f4 xf = Store::value(S, xn);
            if constexpr (is_paper_kind(KIND)) {
                paper_chunk(pacc, xf, c, S.d, L, ln, KIND);
            } else {
                const f4 sv = STAGE ? ls[c] : s4[c];
                const f4 wv = (KIND == OBJ_RIPPLE) ? (STAGE ? lw[c] : w4[c]) : zero;
                if constexpr (RAGGED)
                    acc += terms4<KIND>(xf, sv, wv, 4u * c, S.d);
                else
                    acc += terms4_full<KIND>(xf, sv, wv);
            }
        }
    }
    // Butterfly over the L lanes of the particle (the masks are immediates;
    // with a runtime width the steps above it are skipped uniformly).
    if constexpr (is_paper_kind(KIND)) {
        acc = paper_finish(pacc, L, S.d, KIND);
    } else {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1)
            if ((uint32_t)m < L) acc += __shfl_xor(acc, m, 64);
    }

    // Algorithm 3: replace the pBest on a strict improvement (NaN ordered last).
    const bool improved = valid && (INIT || improves(acc, fpi));
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

    generation_commit<WAVES>(S, t, blk, key, (improved && ln == 0) ? 1u : 0u);
}

}  // namespace sso
