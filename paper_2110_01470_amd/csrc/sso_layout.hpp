// State layout in device memory and the launchers each kernel file exports.
//
// Per particle i the workspace holds two rows of dp floats (dp = d rounded up
// to 32, so every row starts on a 128-byte line) and a state word:
//   bit 0 (ST_ROW)   which of the two rows holds the pBest,
//   bit 1 (ST_ALIAS) the current position equals the pBest (the other row is
//                    stale and is not read).
// A generation reads pBest (and, unless aliased, X) and writes the new
// position X' into the row that does NOT hold the pBest.  If X' improves on
// the pBest the two roles swap (ST_ROW flips, ST_ALIAS set); otherwise
// ST_ALIAS clears.  No pBest row is ever written in place during a
// generation, so gBest of the previous generation -- row (key & 1) of
// particle (key >> 1) -- stays valid while every particle reads it, and an
// improved particle costs no extra copy: 12 bytes per variable at most
// (read X, read P, write X'), 8 when aliased.
#pragma once

#include <stdint.h>

namespace sso {

enum { OBJ_SPHERE = 0, OBJ_RIPPLE = 1, OBJ_DENSE = 2 };
// Table 3.2's benchmark functions (values of sso_objective).
enum { OBJ_F1 = 11, OBJ_F9 = 19 };
constexpr bool is_paper_kind(int kind) { return kind >= OBJ_F1 && kind <= OBJ_F9; }

// Row storage.  F32: dp floats per row, a float4 per chunk of 4 variables.
// U24: every position is a point of the draw grid lo + u span 2^-24 with a
// 24-bit u (positions are only ever drawn that way or copied), so a row can
// hold the indices u: the 4 of a chunk packed into 3 32-bit words,
//   w0 = u0 | u1 << 24,  w1 = u1 >> 8 | u2 << 16,  w2 = u2 >> 16 | u3 << 8,
// which moves 9 bytes per variable and generation instead of 12.
enum { STORE_F32 = 0, STORE_U24 = 1 };
// The dense kernel's contraction when a split copy of A is held: three
// exact bf16 parts, or two scaled fp16 parts (gen_dense.hip).
enum { SPLIT_BF16X3 = 0, SPLIT_F16X2 = 1 };
enum : uint32_t { ST_ROW = 1u, ST_ALIAS = 2u };

constexpr uint32_t kRowAlign = 32;      // floats per row alignment unit (128 B)
// Waves per workgroup of the STREAM kernel and the batched kernel's default
// (measured on the ripple workload: 4, 8 and 16 waves run within 0.5 % of
// each other); the batched kernel is also built for 8 (the autotuner's pick).
#ifndef SSO_STREAM_WAVES
#define SSO_STREAM_WAVES 4
#endif
constexpr uint32_t kStreamWaves = SSO_STREAM_WAVES;
constexpr uint32_t kDenseMaxD = 256;    // dense kernel limit on d

// gBest hand-off between generations.  Every workgroup folds its (fitness,
// index) key and improvement count into one of kSubSlots sub-slots of the
// generation's group with device-scope atomics; sub-slots sit kSubStride
// 64-bit words (256 B) apart so the atomics of different workgroups do not
// serialise on one line.  Groups rotate over kGroups generations: generation
// t commits into group t % 3, reduces group (t - 1) % 3 to find gBest of the
// previous generation, and its workgroup 0 clears group (t + 1) % 3.  A swarm
// with few workgroups uses only the first nsub sub-slots of each group.
constexpr uint32_t kSubSlots = 64;
constexpr uint32_t kSubStride = 32;
constexpr uint32_t kGroups = 3;
constexpr uint32_t kSubWords = kGroups * kSubSlots * kSubStride;  // 64-bit words

struct SwarmDev {
    float *rows;                 // [2][n][stride] (floats, or packed 24-bit indices)
    float *fp;                   // [n] pBest fitness (FP32)
    uint32_t *st;                // [n] state word
    const float *s;              // [dp] shift, zero padded
    const float *w;              // [dp] ripple weights, zero padded (or null)
    const float *a;              // dense matrix, layout of the dense kernel (or null)
    const float *at;             // its transpose in the same layout (dense only)
    const uint16_t *a3;          // dense matrix split into bf16 or fp16 parts (split contraction), or null
    unsigned long long *keys;    // [trace_cap] gBest key per finished generation (ring)
    uint32_t *cnt;               // [trace_cap] improved pBests per finished generation (ring)
    unsigned long long *sub;     // [kGroups][kSubSlots][kSubStride]: key, then count
    uint64_t buf;                // 32-bit words from row buffer 0 to row buffer 1 (n * stride)
    uint32_t n, d, dp, chunks;   // dp = d rounded up to 32; chunks = ceil(d / 4)
    uint32_t stride;             // 32-bit words per row: dp (F32) or 3 chunks rounded up to 32 (U24)
    int32_t storage;             // STORE_F32 or STORE_U24
    uint32_t trace_cap;
    uint32_t th0, th1, th2, r;   // integer thresholds and fresh-draw rescale
    float lo, span, span24;      // span24 = span * 2^-24 (exact)
    uint32_t key0, key1, swarm;  // Philox key and fourth counter word
    int32_t kind, order;
    uint32_t nsub;               // sub-slots in use (a power of two <= kSubSlots)
    uint32_t lanes;              // lanes per particle (batched kernel; a power of two)
    int32_t split;               // SPLIT_BF16X3 or SPLIT_F16X2 (with a3)
};

// Batched engine: many independent separable swarms advance together, one
// launch per generation.  Workgroup b of a launch runs block tiles[2b+1] of
// swarm tiles[2b], whose parameters are table[tiles[2b]]; all swarms share
// the objective kind, the interval order and the row storage.  Generation
// launches read t = *tbase + j, so a captured block of launches (j = 1..K
// followed by a node that adds K to *tbase) can be replayed unchanged.
struct BatchDev {
    const SwarmDev *table;       // [count]
    const uint32_t *tiles;       // [ntiles][2]: swarm, block within the swarm
    uint32_t *tbase;             // generations completed before the current block
    unsigned long long *results; // [count][2]: gBest key, improved count (collect)
    uint32_t count, ntiles;
    uint32_t waves;              // waves per workgroup: 4 or 8
    uint32_t lds;                // dynamic LDS bytes per workgroup (largest swarm)
    int32_t kind, order, storage;
};

// Launchers (each returns hipSuccess or the launch error).
int launch_stream_generation(const SwarmDev &S, uint32_t t, uint32_t lanes, void *stream);
int launch_stream_paper(const SwarmDev &S, uint32_t t, void *stream);  // Table 3.2's functions
int launch_dense_generation(const SwarmDev &S, uint32_t t, void *stream);
int launch_fill_trace(const SwarmDev &S, void *stream);  // clears trace ring and sub-slot groups
int launch_debug_rng(const SwarmDev &S, uint32_t t, uint32_t *out, void *stream);
int launch_resident(const SwarmDev &S, uint32_t t_first, uint32_t generations, void *stream);
bool resident_fits(uint32_t n, uint32_t d, int kind);
uint64_t dense_matrix_floats(uint32_t d);
uint64_t dense_split_halves(uint32_t d);  // bf16 values of the split matrix
uint64_t dense_f16x2_halves(uint32_t d);  // 16-bit words of the fp16 split (parts and scales)

int launch_batch_fill(const BatchDev &B, void *stream);    // every swarm's trace ring and sub-slots
int launch_batch_init(const BatchDev &B, void *stream);    // generation 0 of every swarm
int launch_batch_set_base(const BatchDev &B, uint32_t t, void *stream);
// Generations *tbase + 1 .. *tbase + k, then *tbase += k.
int launch_batch_generations(const BatchDev &B, uint32_t k, void *stream);
// The same k launches and the base update as nodes of a new graph.
int batch_graph(const BatchDev &B, uint32_t k, void **graph_out);
// results[s] = gBest key and improved count of generation t, for every swarm.
int launch_batch_collect(const BatchDev &B, uint32_t t, void *stream);
size_t batch_stage_bytes(int kind, int storage, uint32_t chunks);
void dense_pack_matrix(const float *a, uint32_t d, float *out);
void dense_pack_split(const float *a, uint32_t d, uint16_t *out);
// The fp16 split of A with its scales for differences x - s within the box
// [lo, hi]; false (nothing written) if the instance does not fit the scaling
// (a non-finite value, or magnitudes beyond 2^+-100).  out may be null to
// check only.
bool dense_pack_f16x2(const float *a, uint32_t d, const float *s, float lo, float hi, uint16_t *out);

// Dense objective at given points and its gradient (grad_dense.hip).
struct GradArgs {
    const float *x;     // [m][ld] points (device)
    const float *gout;  // [m] factors of the gradients, or null (1)
    float *f;           // [m] f(x), or null
    float *g;           // [m][ld] gout * grad f(x), or null
    uint32_t m, ld;
};
// f and/or gradients at m points; S supplies s, a, at and d.
int launch_dense_eval(const SwarmDev &S, const GradArgs &G, void *stream);
// Gradient polish of every pBest of the swarm (steps projected steps of
// size lr, accept-if-better); new gBest keys go to generation t's group.
int launch_dense_polish(const SwarmDev &S, uint32_t steps, float lr, uint32_t t, void *stream);

}  // namespace sso
