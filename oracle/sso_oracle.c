/*
 * CPU oracle for Simplified Swarm Optimization (arXiv 2110.01470).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
 * code with the GPU path.  Plain loops, no blocking, no fusion: each function
 * follows one passage of the paper and says which.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fopenmp -fPIC -shared (no -march
 * flags, so no FMA contraction can creep into the FP64 fitness).  The loops
 * over particles may run on several threads (orc_set_threads; one by
 * default): every particle's work reads only the previous generation's state
 * and writes only its own row, and the argmin stays serial, so the results do
 * not depend on the thread count.
 */
#include "sso_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }

int orc_threads(void)
{
#ifdef _OPENMP
    return g_threads;
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11): ten rounds of the
 * Philox S-box on a 4x32-bit counter, with a 2x32-bit key bumped by the Weyl
 * constants between rounds.  Stands in for the cuRAND stream of Sec. 3.1.
 * ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += PHILOX_W0;
            k[1] += PHILOX_W1;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* One word per (generation, particle, variable), as Sec. 3.1 counts them:
 * variable j uses word j mod 4 of the block whose counter is
 * (j div 4, i, t, swarm). */
void orc_words(uint64_t seed, uint32_t swarm, uint32_t t, uint32_t n, uint32_t d,
               uint32_t *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (uint32_t i = 0; i < n; ++i) {
        for (uint32_t j = 0; j < d; ++j) {
            uint32_t ctr[4] = {j / 4u, i, t, swarm};
            uint32_t blk[4];
            orc_philox4x32_10(ctr, key, blk);
            out[(size_t)i * d + j] = blk[j % 4u];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Eq. (2.1) in integer form.  A word k in [0, 2^32) stands for rand() =
 * k * 2^-32.  rand() < c  <=>  k < ceil(c * 2^32), exactly, so the interval
 * test is an integer compare.  The fresh value is uniform on [varMin, varMax]
 * (Table 3.1); it reuses the word that chose the fresh interval: k - th[2] is
 * uniform on [0, W), W = 2^32 - th[2], and ((k - th[2]) * floor(2^56 / W)) >> 32
 * maps it to 24 bits.
 * ------------------------------------------------------------------------- */
static uint64_t threshold(double c) { return (uint64_t)ceil(c * 4294967296.0); }

int orc_rule_make(double cg, double cp, double cw, int order, float lo, float hi,
                  orc_rule *out)
{
    if (!out || !isfinite(lo) || !isfinite(hi) || !(lo < hi))
        return -1;
    if (!(cg >= 0.0 && cg <= 1.0 && cp >= 0.0 && cp <= 1.0 && cw >= 0.0 && cw <= 1.0))
        return -1;
    double c0, c1, c2;
    if (order == ORC_ORDER_GPS) {
        c0 = cg; c1 = cp; c2 = cw;
        out->src[0] = ORC_SRC_GBEST; out->src[1] = ORC_SRC_PBEST; out->src[2] = ORC_SRC_SELF;
    } else if (order == ORC_ORDER_EQ21) {
        c0 = cw; c1 = cp; c2 = cg;
        out->src[0] = ORC_SRC_SELF; out->src[1] = ORC_SRC_PBEST; out->src[2] = ORC_SRC_GBEST;
    } else {
        return -1;
    }
    if (!(c0 <= c1 && c1 <= c2))
        return -1;
    out->th[0] = threshold(c0);
    out->th[1] = threshold(c1);
    out->th[2] = threshold(c2);
    uint64_t w = 4294967296ull - out->th[2];
    if (w <= (1ull << 24)) /* the fresh interval must hold more than 2^24 words */
        return -1;
    out->r = (uint32_t)((1ull << 56) / w);
    out->lo = lo;
    out->span = hi - lo; /* FP32 subtraction, as the GPU library computes it */
    if (!isfinite(out->span) || !(out->span > 0.0f))
        return -1;
    return 0;
}

int orc_source(const orc_rule *r, uint32_t word)
{
    if (word < r->th[0]) return r->src[0];
    if (word < r->th[1]) return r->src[1];
    if (word < r->th[2]) return r->src[2];
    return ORC_SRC_FRESH;
}

static float draw(const orc_rule *r, uint32_t u24)
{
    /* u24 * 2^-24 is exact in FP32; fmaf rounds once. */
    return fmaf(ldexpf((float)u24, -24), r->span, r->lo);
}

float orc_init_value(const orc_rule *r, uint32_t word) { return draw(r, word >> 8); }

float orc_fresh_value(const orc_rule *r, uint32_t word)
{
    uint64_t q = (uint64_t)(word - (uint32_t)r->th[2]) * (uint64_t)r->r;
    return draw(r, (uint32_t)(q >> 32));
}

/* ---------------------------------------------------------------------------
 * Objectives, FP64 on FP32 inputs, summed pairwise:
 * S(v[0..n)) = S(v[0..h)) + S(v[h..n)), h = n/2, S of one element = element.
 * ------------------------------------------------------------------------- */
static double pairwise(const double *v, size_t n)
{
    if (n == 0) return 0.0;
    if (n == 1) return v[0];
    size_t h = n / 2;
    return pairwise(v, h) + pairwise(v + h, n - h);
}

/* Table 3.2.  With scale != 0 the same sums of magnitudes (see
 * orc_fitness_scale).  t and u are scratch arrays of d doubles. */
static double paper_function(int kind, uint32_t d, const float *x, double *t, double *u, int scale)
{
    const double pi = 3.14159265358979323846, e1 = 2.71828182845904523536;
    const double P = (double)d;
    double f = 0.0;
    switch (kind) {
    case ORC_F1:  /* sphere */
        for (uint32_t i = 0; i < d; ++i) t[i] = (double)x[i] * x[i];
        f = pairwise(t, d);
        break;
    case ORC_F2:  /* hyper-ellipsoid: the i-th square weighted by i (from 1) */
        for (uint32_t i = 0; i < d; ++i) t[i] = (double)(i + 1) * x[i] * x[i];
        f = pairwise(t, d);
        break;
    case ORC_F3: {  /* Schwefel 1.2: squares of the running sums */
        double run = 0.0;
        for (uint32_t i = 0; i < d; ++i) {
            run += scale ? fabs((double)x[i]) : (double)x[i];
            t[i] = run * run;
        }
        f = pairwise(t, d);
        break;
    }
    case ORC_F4: {  /* Rosenbrock: neighbouring pairs (x_i, x_{i+1}) */
        const uint32_t m = d ? d - 1 : 0;
        for (uint32_t i = 0; i < m; ++i) {
            const double xi = x[i], xn = x[i + 1];
            const double q = scale ? fabs(xn) + xi * xi : xn - xi * xi;
            const double r = scale ? 1.0 + fabs(xi) : 1.0 - xi;
            t[i] = 100.0 * q * q + r * r;
        }
        f = pairwise(t, m);
        break;
    }
    case ORC_F5:  /* Rastrigin */
        for (uint32_t i = 0; i < d; ++i) {
            const double c = cos(2.0 * pi * x[i]);
            t[i] = (double)x[i] * x[i] + (scale ? 10.0 * fabs(c) : -10.0 * c);
        }
        f = 10.0 * P + pairwise(t, d);
        break;
    case ORC_F6: {  /* Ackley, a = 20, b = 0.2, c = 2 pi */
        for (uint32_t i = 0; i < d; ++i) {
            t[i] = (double)x[i] * x[i];
            u[i] = cos(2.0 * pi * x[i]);
        }
        const double e_a = exp(-0.2 * sqrt(pairwise(t, d) / P));
        const double e_b = exp(pairwise(u, d) / P);
        f = scale ? 20.0 * e_a + e_b + 20.0 + e1 : -20.0 * e_a - e_b + 20.0 + e1;
        break;
    }
    case ORC_F7: {  /* Griewank */
        double prod = 1.0;
        for (uint32_t i = 0; i < d; ++i) {
            t[i] = (double)x[i] * x[i];
            prod *= cos((double)x[i] / sqrt((double)(i + 1)));
        }
        f = scale ? pairwise(t, d) / 4000.0 + fabs(prod) + 1.0 : pairwise(t, d) / 4000.0 - prod + 1.0;
        break;
    }
    case ORC_F8: {  /* Powell: groups (x1, x2, x3, x4) of four consecutive variables */
        const uint32_t g = d / 4;
        for (uint32_t k = 0; k < g; ++k) {
            const double x1 = x[4 * k], x2 = x[4 * k + 1], x3 = x[4 * k + 2], x4 = x[4 * k + 3];
            double a1, a2, a3, a4;
            if (scale) {
                a1 = fabs(x1) + 10.0 * fabs(x2);
                a2 = fabs(x3) + fabs(x4);
                a3 = fabs(x2) + 2.0 * fabs(x3);
                a4 = fabs(x1) + fabs(x4);
            } else {
                a1 = x1 + 10.0 * x2;
                a2 = x3 - x4;
                a3 = x2 - 2.0 * x3;
                a4 = x1 - x4;
            }
            t[k] = a1 * a1 + 5.0 * a2 * a2 + a3 * a3 * a3 * a3 + 10.0 * a4 * a4 * a4 * a4;
        }
        f = pairwise(t, g);
        break;
    }
    case ORC_F9:  /* Schwefel 2.26 */
        for (uint32_t i = 0; i < d; ++i) {
            const double v = (double)x[i] * sin(sqrt(fabs((double)x[i])));
            t[i] = scale ? fabs(v) : v;
        }
        f = scale ? 418.9829 * P + pairwise(t, d) : 418.9829 * P - pairwise(t, d);
        break;
    default:
        f = NAN;
    }
    return f;
}

double orc_fitness(int kind, uint32_t d, const float *x, const float *s, const float *w,
                   const float *a)
{
    double *t = (double *)malloc(sizeof(double) * (d ? d : 1));
    double *u = (double *)malloc(sizeof(double) * (d ? d : 1));
    double f = 0.0;
    if (kind == ORC_SPHERE) {
        /* sum_j (x_j - s_j)^2 */
        for (uint32_t j = 0; j < d; ++j) {
            double dj = (double)x[j] - (double)s[j];
            t[j] = dj * dj;
        }
        f = pairwise(t, d);
    } else if (kind == ORC_RIPPLE) {
        /* sum_j w_j (x_j - s_j)^2  +  0.5 * sum_j sin^2(3 (x_j - s_j)) */
        for (uint32_t j = 0; j < d; ++j) {
            double dj = (double)x[j] - (double)s[j];
            double sn = sin(3.0 * dj);
            t[j] = (double)w[j] * dj * dj;
            u[j] = sn * sn;
        }
        f = pairwise(t, d) + 0.5 * pairwise(u, d);
    } else if (kind == ORC_DENSE) {
        for (uint32_t j = 0; j < d; ++j) t[j] = (double)x[j];
        f = orc_dense_f64(d, t, s, a);
    } else if (kind >= ORC_F1 && kind <= ORC_F9) {
        f = paper_function(kind, d, x, t, u, 0);
    } else {
        f = NAN;
    }
    free(t);
    free(u);
    return f;
}

double orc_fitness_scale(int kind, uint32_t d, const float *x, const float *s, const float *w,
                         const float *a)
{
    (void)s; (void)w; (void)a;
    /* Defined for Table 3.2's functions only (their FP32 error bound); the
     * shifted objectives have none here. */
    if (kind < ORC_F1 || kind > ORC_F9) return NAN;
    double *t = (double *)malloc(sizeof(double) * (d ? d : 1));
    double *u = (double *)malloc(sizeof(double) * (d ? d : 1));
    const double f = paper_function(kind, d, x, t, u, 1);
    free(t);
    free(u);
    return f;
}

/* ---------------------------------------------------------------------------
 * Swarm.
 * ------------------------------------------------------------------------- */
/* y = A (x - s), y_k summed pairwise over j. */
static void dense_residual(uint32_t d, const double *x, const float *s, const float *a, double *y)
{
    double *t = (double *)malloc(sizeof(double) * (d ? d : 1));
    for (uint32_t k = 0; k < d; ++k) {
        for (uint32_t j = 0; j < d; ++j)
            t[j] = (double)a[(size_t)k * d + j] * (x[j] - (double)s[j]);
        y[k] = pairwise(t, d);
    }
    free(t);
}

double orc_dense_f64(uint32_t d, const double *x, const float *s, const float *a)
{
    /* y_k = sum_j A_kj (x_j - s_j);  f = sum_k y_k^2 */
    double *y = (double *)malloc(sizeof(double) * (d ? d : 1));
    dense_residual(d, x, s, a, y);
    for (uint32_t k = 0; k < d; ++k) y[k] = y[k] * y[k];
    const double f = pairwise(y, d);
    free(y);
    return f;
}

void orc_dense_grad(uint32_t d, const double *x, const float *s, const float *a, double *out)
{
    /* df/dx_j = 2 sum_k A_kj y_k */
    double *y = (double *)malloc(sizeof(double) * (d ? d : 1));
    double *t = (double *)malloc(sizeof(double) * (d ? d : 1));
    dense_residual(d, x, s, a, y);
    for (uint32_t j = 0; j < d; ++j) {
        for (uint32_t k = 0; k < d; ++k) t[k] = (double)a[(size_t)k * d + j] * y[k];
        out[j] = 2.0 * pairwise(t, d);
    }
    free(t);
    free(y);
}

static float *dup_floats(const float *src, size_t n)
{
    if (!src) return NULL;
    float *p = (float *)malloc(sizeof(float) * (n ? n : 1));
    memcpy(p, src, sizeof(float) * n);
    return p;
}

orc_swarm *orc_create(uint32_t n, uint32_t d, int kind, float lo, float hi, double cg,
                      double cp, double cw, int order, uint64_t seed, uint32_t swarm,
                      const float *s, const float *w, const float *a)
{
    const int paper = kind >= ORC_F1 && kind <= ORC_F9;
    if (n == 0 || d == 0 || (!s && !paper)) return NULL;
    if (kind == ORC_RIPPLE && !w) return NULL;
    if (kind == ORC_DENSE && !a) return NULL;
    if (kind != ORC_SPHERE && kind != ORC_RIPPLE && kind != ORC_DENSE && !paper) return NULL;
    orc_swarm *sw = (orc_swarm *)calloc(1, sizeof *sw);
    if (orc_rule_make(cg, cp, cw, order, lo, hi, &sw->rule) != 0) {
        free(sw);
        return NULL;
    }
    size_t nd = (size_t)n * d;
    sw->n = n; sw->d = d; sw->kind = kind; sw->seed = seed; sw->swarm = swarm;
    sw->s = dup_floats(s, d);
    sw->w = kind == ORC_RIPPLE ? dup_floats(w, d) : NULL;
    sw->a = kind == ORC_DENSE ? dup_floats(a, (size_t)d * d) : NULL;
    sw->x = (float *)calloc(nd, sizeof(float));
    sw->p = (float *)calloc(nd, sizeof(float));
    sw->fp = (float *)calloc(n, sizeof(float));
    sw->fp64 = (double *)calloc(n, sizeof(double));
    sw->fx64 = (double *)calloc(n, sizeof(double));
    sw->improved = (uint8_t *)calloc(n, 1);
    sw->g = (float *)calloc(d, sizeof(float));
    sw->words = (uint32_t *)calloc(nd, sizeof(uint32_t));
    return sw;
}

void orc_destroy(orc_swarm *sw)
{
    if (!sw) return;
    free(sw->s); free(sw->w); free(sw->a);
    free(sw->x); free(sw->p); free(sw->fp); free(sw->fp64); free(sw->fx64);
    free(sw->improved); free(sw->g); free(sw->words);
    free(sw);
}

static int less_f32(float a, float b)
{
    /* NaN orders above everything, so it never becomes gBest over a number. */
    if (isnan(a)) return 0;
    if (isnan(b)) return 1;
    return a < b;
}

uint32_t orc_argmin(uint32_t n, const float *fp)
{
    uint32_t best = 0;
    for (uint32_t i = 1; i < n; ++i)
        if (less_f32(fp[i], fp[best])) best = i;
    return best;
}

static double fitness_of(const orc_swarm *sw, const float *row)
{
    return orc_fitness(sw->kind, sw->d, row, sw->s, sw->w, sw->a);
}

/* gBest: Algorithm 4, read as the lowest-index argmin of the pBest fitness,
 * copied out of the pBest array so the next generation reads a stable vector. */
static void update_gbest(orc_swarm *sw)
{
    sw->gidx = orc_argmin(sw->n, sw->fp);
    memcpy(sw->g, sw->p + (size_t)sw->gidx * sw->d, sizeof(float) * sw->d);
}

/* Kernel (I), Sec. 2.3.1: uniform population; the first pBests are the
 * initial positions. */
void orc_init_with_words(orc_swarm *sw, const uint32_t *words)
{
    size_t nd = (size_t)sw->n * sw->d;
    for (size_t e = 0; e < nd; ++e)
        sw->x[e] = orc_init_value(&sw->rule, words[e]);
    memcpy(sw->p, sw->x, sizeof(float) * nd);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (uint32_t i = 0; i < sw->n; ++i) {
        double f = fitness_of(sw, sw->x + (size_t)i * sw->d);
        sw->fx64[i] = f;
        sw->fp64[i] = f;
        sw->fp[i] = (float)f;
        sw->improved[i] = 1;
    }
    update_gbest(sw);
    sw->t = 0;
}

/* One generation of Algorithm 2. */
void orc_generation_with_words(orc_swarm *sw, const uint32_t *words)
{
    const uint32_t n = sw->n, d = sw->d;
    /* Search, Eq. (2.1), from the state of the previous generation.  Element
     * (i, j) reads only x_ij, p_ij and g_j, none of which this loop changes
     * for another element, so updating x in place is the same as reading a
     * frozen copy. */
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (uint32_t i = 0; i < n; ++i) {
        for (uint32_t j = 0; j < d; ++j) {
            size_t e = (size_t)i * d + j;
            uint32_t k = words[e];
            switch (orc_source(&sw->rule, k)) {
            case ORC_SRC_GBEST: sw->x[e] = sw->g[j]; break;
            case ORC_SRC_PBEST: sw->x[e] = sw->p[e]; break;
            case ORC_SRC_SELF:  /* keeps x[e] */ break;
            default:            sw->x[e] = orc_fresh_value(&sw->rule, k); break;
            }
        }
    }
    /* Evaluate, then Algorithm 3: replace the pBest on a strict improvement. */
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (uint32_t i = 0; i < n; ++i) {
        const float *xi = sw->x + (size_t)i * d;
        double f = fitness_of(sw, xi);
        float f32 = (float)f;
        sw->fx64[i] = f;
        sw->improved[i] = 0;
        if (less_f32(f32, sw->fp[i])) {
            memcpy(sw->p + (size_t)i * d, xi, sizeof(float) * d);
            sw->fp[i] = f32;
            sw->fp64[i] = f;
            sw->improved[i] = 1;
        }
    }
    /* Algorithm 4. */
    update_gbest(sw);
    sw->t += 1;
}

void orc_init(orc_swarm *sw)
{
    orc_words(sw->seed, sw->swarm, 0u, sw->n, sw->d, sw->words);
    orc_init_with_words(sw, sw->words);
}

void orc_step(orc_swarm *sw)
{
    orc_words(sw->seed, sw->swarm, (uint32_t)(sw->t + 1), sw->n, sw->d, sw->words);
    orc_generation_with_words(sw, sw->words);
}

void orc_run(orc_swarm *sw, uint32_t generations)
{
    for (uint32_t g = 0; g < generations; ++g)
        orc_step(sw);
}

void orc_set_state(orc_swarm *sw, const float *x, const float *p, const float *fp,
                   uint64_t t)
{
    size_t nd = (size_t)sw->n * sw->d;
    memcpy(sw->x, x, sizeof(float) * nd);
    memcpy(sw->p, p, sizeof(float) * nd);
    memcpy(sw->fp, fp, sizeof(float) * sw->n);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (uint32_t i = 0; i < sw->n; ++i) {
        sw->fp64[i] = fitness_of(sw, sw->p + (size_t)i * sw->d);
        sw->fx64[i] = fitness_of(sw, sw->x + (size_t)i * sw->d);
        sw->improved[i] = 0;
    }
    update_gbest(sw);
    sw->t = t;
}

int orc_polish(orc_swarm *sw, uint32_t steps, double lr)
{
    if (sw->kind != ORC_DENSE) return -1;
    const uint32_t d = sw->d;
    const double lo = sw->rule.lo, hi = (double)(sw->rule.lo + sw->rule.span);
    int replaced = 0;
    /* Each pBest is polished on its own (scratch per particle), so the loop
     * may run on several threads. */
#pragma omp parallel for num_threads(g_threads) schedule(static) reduction(+ : replaced)
    for (uint32_t i = 0; i < sw->n; ++i) {
        double *p = (double *)malloc(sizeof(double) * d);
        double *g = (double *)malloc(sizeof(double) * d);
        float *q = (float *)malloc(sizeof(float) * d);
        float *pi = sw->p + (size_t)i * d;
        for (uint32_t j = 0; j < d; ++j) q[j] = pi[j];
        for (uint32_t k = 0; k < steps; ++k) {
            for (uint32_t j = 0; j < d; ++j) p[j] = (double)q[j];
            orc_dense_grad(d, p, sw->s, sw->a, g);
            for (uint32_t j = 0; j < d; ++j) {
                double v = p[j] - lr * g[j];
                if (v < lo) v = lo;
                if (v > hi) v = hi;
                q[j] = (float)v;
            }
        }
        const double f64 = orc_fitness(ORC_DENSE, d, q, sw->s, sw->w, sw->a);
        const float f32 = (float)f64;
        sw->fx64[i] = f64;
        sw->improved[i] = 0;
        const int better = less_f32(f32, sw->fp[i]);
        if (better) {
            for (uint32_t j = 0; j < d; ++j) pi[j] = q[j];
            sw->fp[i] = f32;
            sw->fp64[i] = f64;
            sw->improved[i] = 1;
            ++replaced;
        }
        free(q);
        free(g);
        free(p);
    }
    update_gbest(sw);
    return replaced;
}
