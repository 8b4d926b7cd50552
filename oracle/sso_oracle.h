/*
 * CPU oracle for one synchronous Simplified Swarm Optimization (SSO) run.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the GPU library never does,
 * and the two share no code, headers or tables.
 *
 * What it computes (Yeh, Liu, Tan, Huang, "Implementation of Parallel
 * Simplified Swarm Optimization in CUDA", arXiv 2110.01470):
 *   - the SSO update rule of Eq. (2.1): each variable takes its value from
 *     gBest, its pBest, itself, or a fresh uniform draw on [varMin, varMax]
 *     (Table 3.1), chosen by which interval of [0,1) a uniform number lands in;
 *   - the synchronous flow of Algorithm 2: generation t reads only the state
 *     left by generation t-1, all particles search, then pBests (Algorithm 3)
 *     and gBest (Algorithm 4) are updated;
 *   - one random number per (generation, particle, variable), Sec. 3.1.
 *
 * Arithmetic: positions are FP32 values that are only ever drawn (one
 * correctly rounded fmaf) or copied, so they are exact.  Fitness is computed
 * in FP64 with a fixed pairwise summation and rounded once to FP32; pBest and
 * gBest decisions are taken on those FP32 values, the precision the GPU
 * library keeps its fitness in.  The FP64 values are kept beside them so that
 * tests can bound the GPU's FP32 fitness.
 */
#ifndef SSO_ORACLE_H
#define SSO_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SPHERE = 0, ORC_RIPPLE = 1, ORC_DENSE = 2 };

/* The benchmark functions of Table 3.2 (unshifted), P = d variables:
 *   F1 sphere         sum x_i^2
 *   F2 hyper-ellipsoid sum i x_i^2                       (i from 1)
 *   F3 Schwefel 1.2   sum_i (sum_{j<=i} x_j)^2
 *   F4 Rosenbrock     sum_{i<P} 100 (x_{i+1} - x_i^2)^2 + (1 - x_i)^2
 *   F5 Rastrigin      10 P + sum x_i^2 - 10 cos(2 pi x_i)
 *   F6 Ackley         -20 exp(-0.2 sqrt(sum x_i^2 / P)) - exp(sum cos(2 pi x_i) / P) + 20 + e
 *   F7 Griewank       sum x_i^2 / 4000 - prod cos(x_i / sqrt(i)) + 1
 *   F8 Powell         sum over the floor(P/4) groups g of four:
 *                     (x1 + 10 x2)^2 + 5 (x3 - x4)^2 + (x2 - 2 x3)^4 + 10 (x1 - x4)^4
 *   F9 Schwefel 2.26  418.9829 P - sum x_i sin(sqrt(|x_i|))
 * Where the printed table is garbled (F3, F5, F6, F8) these are the
 * textbook forms the table names; s, w and a are not used. */
enum { ORC_F1 = 11, ORC_F2, ORC_F3, ORC_F4, ORC_F5, ORC_F6, ORC_F7, ORC_F8, ORC_F9 };

/* Source of a variable in Eq. (2.1). */
enum { ORC_SRC_GBEST = 0, ORC_SRC_PBEST = 1, ORC_SRC_SELF = 2, ORC_SRC_FRESH = 3 };

/* Interval order of the four sources.  ORDER_GPS: gBest [0,cg), pBest
 * [cg,cp), self [cp,cw), fresh [cw,1) with cg <= cp <= cw.  ORDER_EQ21: the
 * order Eq. (2.1) prints, self [0,cw), pBest [cw,cp), gBest [cp,cg),
 * fresh [cg,1) with cw <= cp <= cg. */
enum { ORC_ORDER_GPS = 0, ORC_ORDER_EQ21 = 1 };

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): one block. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The random word of variable j of particle i at generation t:
 * word (j mod 4) of Philox4x32-10 with key (seed low, seed high) and
 * counter (j div 4, i, t, swarm).  out[i*d + j] for i < n, j < d. */
void orc_words(uint64_t seed, uint32_t swarm, uint32_t t, uint32_t n, uint32_t d,
               uint32_t *out);

/* Integer form of the thresholds and of the fresh draw. */
typedef struct {
    uint64_t th[3];  /* interval ends ceil(c * 2^32), non-decreasing          */
    int      src[3]; /* source of the first three intervals                   */
    uint32_t r;      /* floor(2^56 / (2^32 - th[2])): rescale to 24 bits      */
    float    lo, span;
} orc_rule;

/* Returns 0, or -1 if the parameters are invalid (see sso_oracle.c). */
int   orc_rule_make(double cg, double cp, double cw, int order, float lo, float hi,
                    orc_rule *out);
int   orc_source(const orc_rule *r, uint32_t word);
float orc_init_value(const orc_rule *r, uint32_t word);
float orc_fresh_value(const orc_rule *r, uint32_t word);

/* Objective in FP64 on FP32 inputs.  a is d*d row-major (DENSE only),
 * w is d (RIPPLE only). */
double orc_fitness(int kind, uint32_t d, const float *x, const float *s, const float *w,
                   const float *a);

/* Magnitude of the quantities a Table 3.2 function adds up at x (the same
 * sums with every term taken by absolute value and every difference as a sum
 * of magnitudes): the scale against which an FP32 evaluation's rounding
 * error is bounded.  Equals f for F1 and F2 (all terms non-negative).  NaN
 * for every other kind (s, w and a are not used). */
double orc_fitness_scale(int kind, uint32_t d, const float *x, const float *s, const float *w,
                         const float *a);

/* DENSE objective at an FP64 point: f = sum_k (sum_j A_kj (x_j - s_j))^2,
 * every sum pairwise (the same sums orc_fitness forms for FP32 points). */
double orc_dense_f64(uint32_t d, const double *x, const float *s, const float *a);

/* Its gradient at an FP64 point: g = 2 A^T y with y = A (x - s), every sum
 * pairwise.  out[d]. */
void orc_dense_grad(uint32_t d, const double *x, const float *s, const float *a, double *out);

/* One swarm. */
typedef struct {
    uint32_t n, d;
    int      kind;
    orc_rule rule;
    uint64_t seed;
    uint32_t swarm;
    float   *s, *w, *a;      /* owned copies of the objective parameters        */
    float   *x, *p;          /* [n*d] current positions and pBests               */
    float   *fp;             /* [n] pBest fitness, FP32 (decision precision)     */
    double  *fp64;           /* [n] pBest fitness, FP64                          */
    double  *fx64;           /* [n] FP64 fitness of the last generation's X      */
    uint8_t *improved;       /* [n] 1 if the last generation replaced the pBest  */
    float   *g;              /* [d] copy of P[gidx]                              */
    uint32_t gidx;
    uint64_t t;              /* generations done after initialisation            */
    uint32_t *words;         /* [n*d] scratch for generated words                */
} orc_swarm;

orc_swarm *orc_create(uint32_t n, uint32_t d, int kind, float lo, float hi, double cg,
                      double cp, double cw, int order, uint64_t seed, uint32_t swarm,
                      const float *s, const float *w, const float *a);
void orc_destroy(orc_swarm *sw);

/* Initialisation (kernel (I), Sec. 2.3.1) and one generation, with the
 * random words passed in; words[i*d + j]. */
void orc_init_with_words(orc_swarm *sw, const uint32_t *words);
void orc_generation_with_words(orc_swarm *sw, const uint32_t *words);

/* Same, with the words drawn from Philox at t = 0 and t = sw->t + 1. */
void orc_init(orc_swarm *sw);
void orc_step(orc_swarm *sw);
void orc_run(orc_swarm *sw, uint32_t generations);

/* Replace the state (positions, pBests and their fitness, generation count).
 * fp64 is recomputed from p; fp is taken as given; gBest is re-derived. */
void orc_set_state(orc_swarm *sw, const float *x, const float *p, const float *fp,
                   uint64_t t);

/* Gradient polish of every pBest of a DENSE swarm (an extension outside the
 * paper): `steps` times p <- fl32(clip(p - lr * grad f(p), lo, hi)), the
 * gradient taken in FP64 at the FP32 point and the box [lo, hi] the swarm's.
 * The polished point replaces the pBest iff its fitness, rounded to FP32, is
 * below the pBest's (the rule of Algorithm 3); positions X are unchanged.
 * gBest is re-derived.  improved[i] = 1 for each replaced pBest, fx64[i] the
 * FP64 fitness of particle i's polished point.  Returns -1 for a swarm whose
 * objective is not DENSE, else the number of replaced pBests. */
int orc_polish(orc_swarm *sw, uint32_t steps, double lr);

/* Index of the smallest fp (NaN above everything), lowest index on ties. */
uint32_t orc_argmin(uint32_t n, const float *fp);

/* Threads for the loops over particles (default 1; values below 1 mean 1).
 * The results are the same for any count.  orc_threads() reports the count
 * in use: always 1 in a build without OpenMP. */
void orc_set_threads(int n);
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
