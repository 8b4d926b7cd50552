/*
 * sso.h -- C ABI of the MI355X Simplified Swarm Optimization library
 * (libsso.so).  Method: Yeh, Liu, Tan, Huang, "Implementation of Parallel
 * Simplified Swarm Optimization in CUDA", arXiv 2110.01470.
 *
 * The library runs the synchronous SSO flow of Algorithm 2 on one GPU: an
 * initialisation (kernel (I), Sec. 2.3.1) followed by generations, each of
 * which sets every variable of every particle by Eq. (2.1), evaluates every
 * particle, replaces pBests that improved (Algorithm 3) and takes gBest as
 * the pBest of lowest fitness (Algorithm 4).  The problem statement follows
 * Sec. 3.3: f(X) over the box [L, U]^Nvar with Nsol particles; the variables
 * of Table 3.1 map onto sso_config below.
 *
 * Conventions for every call:
 *   - Plain C types only; no exceptions cross the boundary.
 *   - Host arrays belong to the caller and are read or written during the
 *     call only.  The device workspace belongs to the caller (any device
 *     allocation of at least sso_workspace_bytes() bytes, 256-byte aligned)
 *     and must outlive the context.  The context belongs to the library and
 *     is freed by sso_destroy().
 *   - sso_init/sso_step/sso_run/sso_debug_rng only enqueue work on the
 *     caller's HIP stream and return; sso_get_* and sso_set_state synchronise
 *     that stream.
 *   - One host thread at a time may drive a context.
 *   - Return value: SSO_OK or a negative SSO_E_* code; sso_last_error()
 *     gives the detail (including the HIP error string for SSO_E_HIP).
 */
#ifndef SSO_H
#define SSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSO_OK             0
#define SSO_E_INVAL       -1 /* bad argument or configuration                  */
#define SSO_E_NOMEM       -2 /* workspace smaller than sso_workspace_bytes()   */
#define SSO_E_HIP         -3 /* a HIP runtime call failed                      */
#define SSO_E_UNSUPPORTED -4 /* size beyond a kernel limit, or not a gfx950 GPU */
#define SSO_E_STATE       -5 /* call out of order (e.g. trace already dropped)  */

/* Objectives (all minimised).  SPHERE, RIPPLE and DENSE are shifted (optimum
 * 0 at x = s).  F1..F9 are the benchmark functions of Table 3.2, unshifted,
 * with P = d (s, w, a not used; the caller sets the box, e.g. the table's
 * feasible bounds); where the printed table is garbled the textbook form is
 * taken: F3 squares the running sums, F5 has the cosine, F6 has a = 20,
 * b = 0.2, c = 2 pi and + a + e, F8 sums Powell's four terms over the
 * floor(d/4) groups of four, F9 is meant for the box [-500, 500].  F1..F9
 * run on the STREAM engine with d <= 1024, and on the RESIDENT engine when
 * the swarm fits one workgroup (d <= 256, n at most 4 x 1024 / lanes per
 * particle); they are not available to batches. */
typedef enum {
    SSO_OBJ_SPHERE = 0, /* sum_j (x_j - s_j)^2                                  */
    SSO_OBJ_RIPPLE = 1, /* sum_j w_j (x_j - s_j)^2 + 0.5 sum_j sin^2(3(x_j - s_j)) */
    SSO_OBJ_DENSE  = 2, /* || A (x - s) ||^2, A is d x d                        */
    SSO_OBJ_F1_SPHERE = 11,     /* sum x_j^2                                      */
    SSO_OBJ_F2_ELLIPSOID = 12,  /* sum j x_j^2 (j from 1)                         */
    SSO_OBJ_F3_SCHWEFEL12 = 13, /* sum_i (sum_{j<=i} x_j)^2                       */
    SSO_OBJ_F4_ROSENBROCK = 14, /* sum_{j<d} 100 (x_{j+1} - x_j^2)^2 + (1 - x_j)^2 */
    SSO_OBJ_F5_RASTRIGIN = 15,  /* 10 d + sum x_j^2 - 10 cos(2 pi x_j)            */
    SSO_OBJ_F6_ACKLEY = 16,     /* -20 e^{-0.2 sqrt(mean x^2)} - e^{mean cos 2 pi x} + 20 + e */
    SSO_OBJ_F7_GRIEWANK = 17,   /* sum x_j^2 / 4000 - prod cos(x_j / sqrt j) + 1  */
    SSO_OBJ_F8_POWELL = 18,     /* sum over groups of (x1+10x2)^2 + 5(x3-x4)^2 + (x2-2x3)^4 + 10(x1-x4)^4 */
    SSO_OBJ_F9_SCHWEFEL226 = 19 /* 418.9829 d - sum x_j sin(sqrt|x_j|)            */
} sso_objective;

/* Order of the four intervals of Eq. (2.1).  A uniform word k in [0, 2^32)
 * stands for rand() = k 2^-32, and each threshold c becomes ceil(c 2^32).
 *   SSO_ORDER_GPS : gBest [0,cg), pBest [cg,cp), self [cp,cw), fresh [cw,1);
 *                   needs cg <= cp <= cw.
 *   SSO_ORDER_EQ21: self [0,cw), pBest [cw,cp), gBest [cp,cg), fresh [cg,1),
 *                   the order Eq. (2.1) prints; needs cw <= cp <= cg.
 * The fresh value is uniform on [lo, hi] (Table 3.1, "range for rand() > Cg"). */
typedef enum { SSO_ORDER_GPS = 0, SSO_ORDER_EQ21 = 1 } sso_order;

/* Engines.  AUTO picks RESIDENT when the whole swarm fits one workgroup's
 * registers (for Table 3.2's functions: while it is also faster, see
 * sso_get_mapping), else STREAM.  RESIDENT uses the STREAM engine's default
 * lanes per particle and ignores the config's `lanes`.  RESIDENT and STREAM
 * with the same lanes per
 * particle sum each fitness in the same order and give bit-identical runs;
 * another lanes setting sums in another order, so a pBest or gBest decision
 * between two fitness values a few FP32 ulps apart may go the other way. */
typedef enum {
    SSO_ENGINE_AUTO     = 0,
    SSO_ENGINE_STREAM   = 1, /* one fused kernel per generation                 */
    SSO_ENGINE_RESIDENT = 2  /* one workgroup keeps the swarm on chip and loops */
} sso_engine;

/* Row storage of positions and pBests.  Every position the method produces
 * is a point of the draw grid lo + u (hi - lo) 2^-24 with an integer
 * 0 <= u < 2^24 (values are only drawn that way, Eq. (2.1) and kernel (I), or
 * copied), so the STREAM engine can keep the 24-bit u instead of the FP32
 * value: 9 bytes move per variable and generation instead of 12, with
 * bit-identical positions.  AUTO picks U24 for the STREAM engine on the
 * separable objectives and F32 otherwise.  With U24, sso_set_state accepts
 * only positions on that grid. */
typedef enum { SSO_STORAGE_AUTO = 0, SSO_STORAGE_F32 = 1, SSO_STORAGE_U24 = 2 } sso_storage;

/* DENSE objective: how the generation kernel forms A (x - s).
 * F32: on FP32 matrix cores (v_mfma_f32_16x16x4_f32).
 * BF16X3: every FP32 operand is split exactly into three bf16 parts and the
 * six part products above 2^-24 relative weight go through bf16 matrix
 * cores with FP32 accumulation (the three omitted are below 2^-23 |a d|).
 * F16X2: each row of A, and the differences x - s, are scaled by powers of
 * two into fp16's range (from A, s and the box) and split into two fp16
 * parts; the three products of weight 2^-11 or more go through fp16 matrix
 * cores with FP32 accumulation (each exact in FP32; what is left out is
 * below 2^-20 |a d|, or below 2^-49 of the row's or the box's largest
 * magnitude for entries under 2^-27 of it).  Half the matrix-core work of
 * BF16X3.  Needs finite A and s with magnitudes within 2^+-100 of one
 * another (SSO_E_INVAL otherwise), and, in sso_set_state, positions inside
 * [lo, hi].  Both split forms hold a second copy of A (6 dp^2 bytes).
 * AUTO = F16X2 when the instance fits it, BF16X3 otherwise. */
typedef enum {
    SSO_CONTRACT_AUTO = 0,
    SSO_CONTRACT_F32 = 1,
    SSO_CONTRACT_BF16X3 = 2,
    SSO_CONTRACT_F16X2 = 3
} sso_contraction;

typedef struct {
    uint32_t n;          /* Nsol, particles, >= 1, < 2^31                         */
    uint32_t d;          /* Nvar, variables per particle, >= 1 (DENSE: <= 256)    */
    float    lo, hi;     /* [varMin, varMax]; finite, lo < hi, hi - lo finite     */
    double   cg, cp, cw; /* thresholds in [0,1], ordered as `order` requires, and
                            the fresh interval must hold more than 2^24 words
                            (1 - max threshold > 2^-8, checked in integer form)  */
    uint64_t seed;       /* Philox key: (seed mod 2^32, seed div 2^32)            */
    uint32_t swarm_id;   /* fourth Philox counter word                            */
    int32_t  kind;       /* sso_objective                                         */
    int32_t  order;      /* sso_order                                             */
    int32_t  engine;     /* sso_engine                                            */
    int32_t  storage;    /* sso_storage                                           */
    uint32_t lanes;      /* STREAM engine lanes per particle: 0 = auto, else a
                            power of two in [8, 64]                               */
    uint32_t trace_cap;  /* generations of (fG, gidx, improved) kept on device;
                            0 = 4096, else >= 4                                   */
    const float *s;      /* host [d]: shift (optimum); may be NULL for F1..F9      */
    const float *w;      /* host [d]: RIPPLE weights, else ignored (may be NULL)  */
    const float *a;      /* host [d*d] row-major: DENSE matrix, else ignored      */
    uint32_t polish_every; /* DENSE only: 0 = off; else after every generation t
                              with t mod polish_every == 0, sso_run applies
                              sso_polish(polish_steps, polish_lr)               */
    uint32_t polish_steps; /* gradient steps per polish (used when polish_every) */
    float    polish_lr;    /* step size; <= 0 means 0.05 / sigma_max(A)^2        */
    int32_t  contraction;  /* sso_contraction (DENSE only; ignored otherwise)    */
} sso_config;

typedef struct sso_ctx sso_ctx;

/* Bytes of device workspace the configuration needs; 0 if it is invalid. */
size_t sso_workspace_bytes(const sso_config *cfg);

/* Kernel function (I) of Sec. 2.3.1 and the initialisation that opens
 * Algorithm 2 (Sec. 3.3), its transfer of the problem to the device included.
 * Validates cfg, lays the state out in the workspace, uploads s, w, a
 * (synchronously), and enqueues the initialisation on `hip_stream`
 * (a hipStream_t; NULL = the null stream): X^0 uniform on [lo, hi] (Table
 * 3.1's range) from the Philox words of generation 0, P^0 = X^0,
 * fP^0 = f(X^0), gBest^0 = the lowest-index argmin (Algorithm 4).  *out
 * receives the context; on error *out is NULL. */
int sso_init(const sso_config *cfg, void *dev_workspace, size_t workspace_bytes,
             void *hip_stream, sso_ctx **out);

/* Enqueue one generation t -> t + 1: one pass of the loop body of
 * Algorithm 2 (Sec. 3.3), i.e. the search of kernel function (C) (Eq. 2.1
 * for every variable of every particle), the evaluation of kernel function
 * (E), and the update (U) of the pBests (Algorithm 3) and of gBest
 * (Algorithm 4), all reading only generation t's state. */
int sso_step(sso_ctx *ctx);

/* Enqueue `generations` generations: Algorithm 2's loop over iterations
 * (Sec. 3.3), with no host transfer between them. */
int sso_run(sso_ctx *ctx, uint32_t generations);

/* Algorithm 2's final step (Sec. 3.3), sending the result back to the host.
 * Synchronise, then copy gBest out: g_out host [d] (may be NULL), its FP32
 * fitness, its particle index, and the number of generations done. */
int sso_get_best(sso_ctx *ctx, float *g_out, float *f_out, uint32_t *idx_out,
                 uint64_t *gen_out);

/* Synchronise, then copy the state out into host arrays: x [n*d] current
 * positions, p [n*d] pBests, fp [n] pBest fitness (FP32), *t generations
 * done.  Any pointer may be NULL. */
int sso_get_state(sso_ctx *ctx, float *x, float *p, float *fp, uint64_t *t);

/* Replace the state with host arrays x, p [n*d], fp [n] and the generation
 * count t; gBest becomes the lowest-index argmin of fp.  Used for
 * checkpoint/resume and for parity checks from a given state.  Synchronises.
 * With U24 storage a value off the draw grid returns SSO_E_INVAL and leaves
 * the state unchanged. */
int sso_set_state(sso_ctx *ctx, const float *x, const float *p, const float *fp,
                  uint64_t t);

/* Synchronise, then copy the per-generation trace of generations
 * [first, first + count): fG (FP32 gBest fitness), gBest index, and the number
 * of pBests replaced in that generation (n for the initialisation).  The
 * device keeps the last trace_cap - 2 generations; asking for older or
 * future ones returns SSO_E_STATE.  Any output pointer may be NULL. */
int sso_get_trace(sso_ctx *ctx, uint64_t first, uint32_t count, float *fg,
                  uint32_t *gidx, uint32_t *improved);

/* Enqueue: write the Philox word of every (particle i, variable j) for
 * generation t to dev_words[i*d + j] (device memory, n*d uint32), with the
 * same generator and counter layout the kernels use. */
int sso_debug_rng(sso_ctx *ctx, uint64_t t, uint32_t *dev_words);

/* ------------------------------------------------------------------------
 * Differentiation (DENSE contexts; the objective is ||A (x - s)||^2, whose
 * gradient is 2 A^T A (x - s)).  Not part of the paper's method: an optional
 * gradient polish of the pBests beside plain SSO.
 * ------------------------------------------------------------------------ */

/* Enqueue, for m points x (device [m*d], row-major, FP32): f_out[i] = f(x_i)
 * (device [m], may be NULL) and grad_out[i*d + j] = gout[i] * df/dx_j at x_i
 * (device [m*d], may be NULL; gout device [m] or NULL for 1).  Uses the
 * context's s and A and its stream; the swarm state is not touched.
 * SSO_E_UNSUPPORTED for a non-DENSE context. */
int sso_eval(sso_ctx *ctx, const float *dev_x, uint32_t m, const float *dev_gout,
             float *f_out, float *grad_out);

/* Enqueue a gradient polish of every pBest: `steps` projected steps
 * p <- clip(p - lr * grad f(p), lo, hi) in FP32; a polished point replaces
 * the pBest iff its fitness is strictly lower (Algorithm 3's rule), the
 * current positions are unchanged, and gBest of the current generation is
 * re-derived.  lr <= 0 selects 0.05 / sigma_max(A)^2 (sigma_max from an FP64
 * power iteration on the host at sso_init); *lr_used (host, may be NULL)
 * receives the step size.  SSO_E_UNSUPPORTED for a non-DENSE context. */
int sso_polish(sso_ctx *ctx, uint32_t steps, float lr, float *lr_used);

/* Free the context (not the workspace).  NULL is allowed. */
void sso_destroy(sso_ctx *ctx);

/* ------------------------------------------------------------------------
 * Allocation-free run, for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * The same initialisation and generations as sso_init followed by
 * sso_run(generations) (same kernels, same results bit for bit), with the
 * swarm's state held in a device array the library owns instead of a caller
 * workspace and no context; then gBest after the last generation goes to
 * device memory: dev_g [d] FP32 position, *dev_f its FP32 fitness, *dev_idx
 * its particle index (each may be NULL).  Enqueued on `hip_stream` (NULL =
 * the null stream); returns without synchronising; the host arrays s and w
 * are read during the call.
 *
 * Limits: objectives SPHERE, RIPPLE and F1..F9 (DENSE returns
 * SSO_E_UNSUPPORTED); the state sso_workspace_bytes(cfg) reports must fit the
 * array, SSO_STATIC_SCRATCH_BYTES (64 MiB), else SSO_E_NOMEM and nothing is
 * enqueued.  Each GPU the library runs on holds its own array until the
 * process ends.  Every call on one GPU uses that GPU's array and leaves its
 * state there until the next call: calls that overlap on one GPU (from
 * other streams or host threads) race and give undefined results.  On its
 * success path the call allocates nothing, host or device; the error detail
 * is in sso_last_error(NULL).
 * ------------------------------------------------------------------------ */
#define SSO_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
int sso_run_static(const sso_config *cfg, uint32_t generations, void *hip_stream,
                   float *dev_g, float *dev_f, uint32_t *dev_idx);

/* What the context resolved its config to: *engine_out SSO_ENGINE_STREAM or
 * SSO_ENGINE_RESIDENT (AUTO takes RESIDENT for a separable swarm that fits
 * one workgroup, and for Table 3.2's functions while N times the lanes per
 * particle is at most 256 times 16 (f1, f2, f4, f8), 13 (f3), 11 (f5),
 * 9 (f6) or 10 (f7, f9); STREAM otherwise), *storage_out SSO_STORAGE_F32
 * or SSO_STORAGE_U24, *lanes_out the lanes per particle, *contraction_out
 * the dense kernel's SSO_CONTRACT_F32, _BF16X3 or _F16X2 (F32 for the other
 * objectives).  Any pointer may be NULL.  Host only; SSO_E_INVAL for a NULL
 * ctx. */
int sso_get_mapping(const sso_ctx *ctx, int *engine_out, int *storage_out, uint32_t *lanes_out,
                    int *contraction_out);

/* Static text for an SSO_* code. */
const char *sso_strerror(int code);

/* Detail of the last error on ctx, or of the calling thread's last failed
 * sso_init/sso_workspace_bytes when ctx is NULL.  Empty string if none. */
const char *sso_last_error(const sso_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batched swarms.  `count` independent swarms advance together, one fused
 * launch per generation for all of them, replayed from a HIP graph in
 * blocks of 50 generations.  Each swarm is described by its own sso_config
 * (size, box, thresholds, Philox key and swarm word, objective instance) and
 * evolves exactly as the one-swarm library would evolve it with the same
 * config and the same lanes per particle: the swarms share nothing but the
 * launches.  Every swarm of a batch must have the same separable kind
 * (SPHERE or RIPPLE), the same order and the same resolved storage; engine
 * must be AUTO or STREAM; d <= 1024.  The lanes per particle of each swarm
 * come from a mapping rule (a target number of 4-variable chunks per lane,
 * "cpl") unless its config fixes `lanes`; a generation launch runs
 * workgroups of 4 or 8 waves (4 until tuned); sso_batch_tune() picks the
 * rule and the workgroup size by timing.  Ownership, synchronisation and return codes are as for the
 * one-swarm calls; all swarms share the generation count.
 * ------------------------------------------------------------------------ */
typedef struct sso_batch sso_batch;

/* Bytes of device workspace for the batch; 0 if any config is invalid or
 * the batch constraints above do not hold (detail: sso_batch_last_error(NULL)). */
size_t sso_batch_workspace_bytes(const sso_config *cfgs, uint32_t count);

/* Validates, lays out, uploads every swarm's s (and w) synchronously, and
 * enqueues the initialisation of every swarm (as sso_init does for one). */
int sso_batch_init(const sso_config *cfgs, uint32_t count, void *dev_workspace,
                   size_t workspace_bytes, void *hip_stream, sso_batch **out);

/* Enqueue `generations` generations of every swarm. */
int sso_batch_run(sso_batch *b, uint32_t generations);

/* Autotuner.  Only right after sso_batch_init (no generations run yet):
 * for each candidate mapping -- rule cpl in {1, 2, 4, 8, 16} times
 * workgroups of 4 or 8 waves -- re-initialises the batch and times
 * `generations` generations with HIP events; keeps the fastest and
 * re-initialises under it, so the batch is again at generation 0.  The
 * mapping changes only the launch shape, never a swarm's results (a swarm's
 * lanes per particle come from the rule; its particles fall into workgroups
 * of 4 or 8 waves).  *cpl_out and *waves_out (may be NULL) receive the
 * choice, ms_out[10] (may be NULL) the milliseconds of candidate
 * 2 * r + w (r indexes the rules above in order, w = 0 for 4 waves, 1 for
 * 8).  Synchronises. */
int sso_batch_tune(sso_batch *b, uint32_t generations, uint32_t *cpl_out, uint32_t *waves_out,
                   float *ms_out);

/* Sets the mapping to rule cpl (1..64 chunks per lane) and workgroups of
 * `waves` waves (4 or 8) without timing, e.g. one an earlier
 * sso_batch_tune() chose; only at generation 0 (no generations run), and
 * re-initialises the batch (generation 0 again).  SSO_E_INVAL for another
 * rule or size, SSO_E_STATE after generations.  Enqueued on the batch's
 * stream. */
int sso_batch_set_mapping(sso_batch *b, uint32_t cpl, uint32_t waves);

/* The current mapping: *cpl_out the rule, *waves_out the waves per
 * workgroup, lanes_out[count] each swarm's lanes per particle, *tiles_out
 * the workgroups per generation launch.  Any pointer may be NULL. */
int sso_batch_mapping(sso_batch *b, uint32_t *cpl_out, uint32_t *waves_out, uint32_t *lanes_out,
                      uint32_t *tiles_out);

/* Synchronise, then for every swarm k: f_out[k] its gBest fitness (FP32),
 * idx_out[k] the gBest particle index, improved_out[k] the pBests replaced in
 * the last generation; *gen_out the generations done.  Any pointer may be NULL. */
int sso_batch_get_results(sso_batch *b, float *f_out, uint32_t *idx_out, uint32_t *improved_out,
                          uint64_t *gen_out);

/* Swarm k's gBest (as sso_get_best; g_out host [d_k]). */
int sso_batch_get_best(sso_batch *b, uint32_t k, float *g_out, float *f_out, uint32_t *idx_out);

/* Swarm k's state (as sso_get_state; x, p host [n_k * d_k], fp [n_k]). */
int sso_batch_get_state(sso_batch *b, uint32_t k, float *x, float *p, float *fp, uint64_t *t);

/* Replace swarm k's state (as sso_set_state).  t must equal the batch's
 * generation count, else SSO_E_STATE. */
int sso_batch_set_state(sso_batch *b, uint32_t k, const float *x, const float *p,
                        const float *fp, uint64_t t);

/* Swarm k's trace (as sso_get_trace). */
int sso_batch_get_trace(sso_batch *b, uint32_t k, uint64_t first, uint32_t count, float *fg,
                        uint32_t *gidx, uint32_t *improved);

/* Free the batch (not the workspace).  NULL is allowed. */
void sso_batch_destroy(sso_batch *b);

/* Detail of the last error on b, or of the calling thread's last failed
 * sso_batch_init/sso_batch_workspace_bytes when b is NULL. */
const char *sso_batch_last_error(const sso_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* SSO_H */
