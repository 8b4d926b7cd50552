// Host side of the C ABI declared in include/sso.h.
//
// Validation, workspace layout, uploads, kernel dispatch and state
// import/export.  No arithmetic of the method runs here except the integer
// thresholds (Eq. 2.1 in integer form) and, in sso_set_state, the
// lowest-index argmin that defines gBest for an imported state (Algorithm 4).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sso.h"
#include "sso_layout.hpp"

using namespace sso;

struct sso_ctx {
    SwarmDev S;
    hipStream_t stream;
    int engine;        // resolved engine
    int storage;       // resolved row storage (STORE_F32 / STORE_U24)
    uint32_t lanes;    // STREAM lanes per particle
    uint64_t t;        // generations done
    uint64_t trace_base;
    std::string err;
};

namespace {

thread_local std::string g_err;

constexpr uint32_t kDefaultTraceCap = 4096;
constexpr uint32_t kMaxD = 1u << 20;

size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

struct Layout {
    size_t rows, fp, st, s, w, a, keys, cnt, sub, total;
    uint32_t dp, stride, trace_cap;
    int engine, storage;
};

// Engine and storage a valid configuration resolves to.
void resolve(const sso_config &c, int *engine, int *storage);

Layout make_layout(const sso_config &c)
{
    Layout L{};
    resolve(c, &L.engine, &L.storage);
    L.dp = round_up(c.d, kRowAlign);
    L.stride = L.storage == STORE_U24 ? round_up(3 * ((c.d + 3) / 4), kRowAlign) : L.dp;
    L.trace_cap = c.trace_cap ? c.trace_cap : kDefaultTraceCap;
    size_t off = 0;
    L.rows = off; off += align256((size_t)2 * c.n * L.stride * sizeof(uint32_t));
    L.fp = off;   off += align256((size_t)c.n * sizeof(float));
    L.st = off;   off += align256((size_t)c.n * sizeof(uint32_t));
    L.s = off;    off += align256((size_t)L.dp * sizeof(float));
    L.w = off;    off += c.kind == SSO_OBJ_RIPPLE ? align256((size_t)L.dp * sizeof(float)) : 0;
    L.a = off;    off += c.kind == SSO_OBJ_DENSE ? align256(dense_matrix_floats(c.d) * sizeof(float)) : 0;
    L.keys = off; off += align256((size_t)L.trace_cap * sizeof(unsigned long long));
    L.cnt = off;  off += align256((size_t)L.trace_cap * sizeof(uint32_t));
    L.sub = off;  off += align256((size_t)kSubWords * sizeof(unsigned long long));
    L.total = off;
    return L;
}

uint64_t threshold(double c) { return (uint64_t)std::ceil(c * 4294967296.0); }

bool resident_possible(const sso_config &c) { return resident_fits(c.n, c.d, c.kind); }

void resolve(const sso_config &c, int *engine, int *storage)
{
    int e = c.engine;
    if (c.kind == SSO_OBJ_DENSE) e = SSO_ENGINE_STREAM;
    if (e == SSO_ENGINE_AUTO) e = resident_possible(c) ? SSO_ENGINE_RESIDENT : SSO_ENGINE_STREAM;
    *engine = e;
    const bool packable = e == SSO_ENGINE_STREAM && c.kind != SSO_OBJ_DENSE;
    *storage = (c.storage == SSO_STORAGE_F32 || !packable) ? STORE_F32 : STORE_U24;
}

// Lanes per particle for the STREAM engine: the chunk count rounded up to a
// power of two, at least 8, at most 32 with 24-bit rows and 64 with FP32 rows
// (measured on the ripple workload with D=1000: U24 131.9 us at 32 lanes vs
// 135.1 at 64; F32 160.2 us at 64 vs 172.1 at 32).
uint32_t stream_lanes(uint32_t d, int storage)
{
    const uint32_t chunks = (d + 3) / 4;
    const uint32_t cap = storage == STORE_U24 ? 32u : 64u;
    uint32_t L = 8;
    while (L < chunks && L < cap) L <<= 1;
    return L;
}

// Returns SSO_OK or an error code, with the reason in *why.
int validate(const sso_config *c, std::string *why)
{
    auto bad = [&](int code, const char *msg) {
        *why = msg;
        return code;
    };
    if (!c) return bad(SSO_E_INVAL, "cfg is NULL");
    if (c->n == 0 || c->n >= (1u << 31)) return bad(SSO_E_INVAL, "n must be in [1, 2^31)");
    if (c->d == 0) return bad(SSO_E_INVAL, "d must be >= 1");
    if (c->d > kMaxD) return bad(SSO_E_UNSUPPORTED, "d exceeds 2^20");
    if (c->kind < SSO_OBJ_SPHERE || c->kind > SSO_OBJ_DENSE) return bad(SSO_E_INVAL, "unknown objective kind");
    if (c->kind == SSO_OBJ_DENSE && c->d > kDenseMaxD) return bad(SSO_E_UNSUPPORTED, "dense objective supports d <= 256");
    if (c->order != SSO_ORDER_GPS && c->order != SSO_ORDER_EQ21) return bad(SSO_E_INVAL, "unknown interval order");
    if (c->engine < SSO_ENGINE_AUTO || c->engine > SSO_ENGINE_RESIDENT) return bad(SSO_E_INVAL, "unknown engine");
    if (c->lanes != 0 && (c->lanes < 8 || c->lanes > 64 || (c->lanes & (c->lanes - 1))))
        return bad(SSO_E_INVAL, "lanes must be 0 or a power of two in [8, 64]");
    if (c->trace_cap != 0 && c->trace_cap < 4) return bad(SSO_E_INVAL, "trace_cap must be 0 or >= 4");
    if (!c->s) return bad(SSO_E_INVAL, "s is NULL");
    if (c->kind == SSO_OBJ_RIPPLE && !c->w) return bad(SSO_E_INVAL, "ripple objective needs w");
    if (c->kind == SSO_OBJ_DENSE && !c->a) return bad(SSO_E_INVAL, "dense objective needs a");
    if (!std::isfinite(c->lo) || !std::isfinite(c->hi) || !(c->lo < c->hi))
        return bad(SSO_E_INVAL, "need finite lo < hi");
    const float span = c->hi - c->lo;
    if (!std::isfinite(span)) return bad(SSO_E_INVAL, "hi - lo overflows FP32");
    const double cs[3] = {c->cg, c->cp, c->cw};
    for (double v : cs)
        if (!(v >= 0.0 && v <= 1.0)) return bad(SSO_E_INVAL, "thresholds must be in [0, 1]");
    const double t0 = c->order == SSO_ORDER_GPS ? c->cg : c->cw;
    const double t2 = c->order == SSO_ORDER_GPS ? c->cw : c->cg;
    if (!(t0 <= c->cp && c->cp <= t2)) return bad(SSO_E_INVAL, "thresholds out of order for this interval order");
    if ((1ull << 32) - threshold(t2) <= (1ull << 24))
        return bad(SSO_E_INVAL, "fresh interval must hold more than 2^24 words (1 - last threshold > 2^-8)");
    if (c->engine == SSO_ENGINE_RESIDENT && !resident_fits(c->n, c->d, c->kind))
        return bad(SSO_E_UNSUPPORTED, "swarm does not fit the resident engine (one workgroup, separable objective)");
    if (c->storage < SSO_STORAGE_AUTO || c->storage > SSO_STORAGE_U24) return bad(SSO_E_INVAL, "unknown storage");
    if (c->storage == SSO_STORAGE_U24) {
        int e, st;
        resolve(*c, &e, &st);
        if (st != STORE_U24)
            return bad(SSO_E_UNSUPPORTED, "24-bit storage needs the STREAM engine and a separable objective");
    }
    return SSO_OK;
}

int hip_fail(std::string *err, hipError_t e, const char *what)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    *err = buf;
    return SSO_E_HIP;
}

#define HIP_TRY(err, call)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(err, e_, #call); \
    } while (0)

uint32_t orderable_host(float f)
{
    uint32_t b;
    std::memcpy(&b, &f, 4);
    if (f != f) return 0xFFFFFFFFu;
    if (f == 0.0f) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

float from_orderable(uint32_t o)
{
    const uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

// Row conversion between FP32 values and the storage format.  A U24 row holds
// the grid index u of every value, value = fma(u, span 2^-24, lo) rounded
// once to FP32, four indices per three 32-bit words (sso_layout.hpp).
float grid_value(const SwarmDev &S, uint32_t u) { return std::fmaf((float)(int32_t)u, S.span24, S.lo); }

void row_to_values(const SwarmDev &S, const uint32_t *row, float *out)
{
    if (S.storage == STORE_F32) {
        std::memcpy(out, row, sizeof(float) * S.d);
        return;
    }
    for (uint32_t j = 0; j < S.d; ++j) {
        const uint32_t *w = row + 3 * (j / 4);
        uint32_t u = 0;
        switch (j % 4) {
        case 0: u = w[0] & 0xFFFFFFu; break;
        case 1: u = (w[0] >> 24) | ((w[1] & 0xFFFFu) << 8); break;
        case 2: u = (w[1] >> 16) | ((w[2] & 0xFFu) << 16); break;
        default: u = w[2] >> 8; break;
        }
        out[j] = grid_value(S, u);
    }
}

bool same_bits(float a, float b) { return std::memcmp(&a, &b, sizeof a) == 0; }

// Grid index of x, or false when x is not a grid point.
bool grid_index(const SwarmDev &S, float x, uint32_t *u)
{
    if (!std::isfinite(x)) return false;
    const double guess = std::nearbyint(((double)x - (double)S.lo) / (double)S.span24);
    for (double cand : {guess, guess - 1.0, guess + 1.0}) {
        if (cand < 0.0 || cand >= 16777216.0) continue;
        if (same_bits(grid_value(S, (uint32_t)cand), x)) {
            *u = (uint32_t)cand;
            return true;
        }
    }
    return false;
}

bool values_to_row(const SwarmDev &S, const float *in, uint32_t *row)
{
    if (S.storage == STORE_F32) {
        std::memcpy(row, in, sizeof(float) * S.d);
        return true;
    }
    for (uint32_t c = 0; c < S.chunks; ++c) {
        uint32_t u[4] = {0, 0, 0, 0};
        for (uint32_t e = 0; e < 4; ++e) {
            const uint32_t j = 4 * c + e;
            if (j < S.d && !grid_index(S, in[j], &u[e])) return false;
        }
        row[3 * c + 0] = u[0] | (u[1] << 24);
        row[3 * c + 1] = (u[1] >> 8) | (u[2] << 16);
        row[3 * c + 2] = (u[2] >> 16) | (u[3] << 8);
    }
    return true;
}

// gBest key and improvement count of generation t, from its sub-slot group
// (the trace ring holds a generation only once the next one has run).
int current_result(sso_ctx *ctx, unsigned long long *key, uint32_t *count)
{
    const SwarmDev &S = ctx->S;
    std::vector<unsigned long long> grp((size_t)kSubSlots * kSubStride);
    const unsigned long long *src = S.sub + (size_t)(ctx->t % kGroups) * kSubSlots * kSubStride;
    HIP_TRY(&ctx->err, hipMemcpy(grp.data(), src, sizeof(unsigned long long) * grp.size(), hipMemcpyDeviceToHost));
    unsigned long long k = ~0ull;
    uint32_t c = 0;
    for (uint32_t j = 0; j < kSubSlots; ++j) {
        const unsigned long long kj = grp[(size_t)j * kSubStride];
        uint32_t cj;
        std::memcpy(&cj, &grp[(size_t)j * kSubStride + 1], sizeof cj);
        if (kj < k) k = kj;
        c += cj;
    }
    *key = k;
    *count = c;
    return SSO_OK;
}

int launch_generations(sso_ctx *ctx, uint64_t t_first, uint32_t count)
{
    const SwarmDev &S = ctx->S;
    if (ctx->engine == SSO_ENGINE_RESIDENT) {
        const int e = launch_resident(S, (uint32_t)t_first, count, ctx->stream);
        if (e) return hip_fail(&ctx->err, (hipError_t)e, "resident kernel launch");
        return SSO_OK;
    }
    for (uint32_t k = 0; k < count; ++k) {
        const uint32_t t = (uint32_t)(t_first + k);
        const int e = S.kind == SSO_OBJ_DENSE ? launch_dense_generation(S, t, ctx->stream)
                                              : launch_stream_generation(S, t, ctx->lanes, ctx->stream);
        if (e) return hip_fail(&ctx->err, (hipError_t)e, "generation kernel launch");
    }
    return SSO_OK;
}

int launch_init(sso_ctx *ctx)
{
    const SwarmDev &S = ctx->S;
    int e = launch_fill_trace(S, ctx->stream);
    if (e) return hip_fail(&ctx->err, (hipError_t)e, "trace fill launch");
    e = S.kind == SSO_OBJ_DENSE ? launch_dense_generation(S, 0, ctx->stream)
                                : launch_stream_generation(S, 0, ctx->lanes, ctx->stream);
    if (e) return hip_fail(&ctx->err, (hipError_t)e, "init kernel launch");
    return SSO_OK;
}

}  // namespace

extern "C" {

size_t sso_workspace_bytes(const sso_config *cfg)
{
    std::string why;
    if (validate(cfg, &why) != SSO_OK) {
        g_err = why;
        return 0;
    }
    return make_layout(*cfg).total;
}

int sso_init(const sso_config *cfg, void *ws, size_t ws_bytes, void *stream, sso_ctx **out)
{
    if (!out) {
        g_err = "out is NULL";
        return SSO_E_INVAL;
    }
    *out = nullptr;
    std::string why;
    int rc = validate(cfg, &why);
    if (rc != SSO_OK) {
        g_err = why;
        return rc;
    }
    const Layout L = make_layout(*cfg);
    if (!ws || ((uintptr_t)ws & 255u)) {
        g_err = "workspace must be a non-NULL, 256-byte aligned device pointer";
        return SSO_E_INVAL;
    }
    if (ws_bytes < L.total) {
        g_err = "workspace smaller than sso_workspace_bytes()";
        return SSO_E_NOMEM;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        g_err = "no HIP device";
        return SSO_E_HIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_err = std::string("library is built for gfx950, device is ") + prop.gcnArchName;
        return SSO_E_UNSUPPORTED;
    }

    sso_ctx *ctx = new sso_ctx();
    ctx->stream = (hipStream_t)stream;
    ctx->t = 0;
    ctx->trace_base = 0;
    const int engine = L.engine;
    ctx->engine = engine;
    ctx->storage = L.storage;
    ctx->lanes = (engine == SSO_ENGINE_STREAM && cfg->lanes) ? cfg->lanes : stream_lanes(cfg->d, L.storage);

    char *base = (char *)ws;
    SwarmDev &S = ctx->S;
    S.rows = (float *)(base + L.rows);
    S.fp = (float *)(base + L.fp);
    S.st = (uint32_t *)(base + L.st);
    S.s = (const float *)(base + L.s);
    S.w = cfg->kind == SSO_OBJ_RIPPLE ? (const float *)(base + L.w) : nullptr;
    S.a = cfg->kind == SSO_OBJ_DENSE ? (const float *)(base + L.a) : nullptr;
    S.keys = (unsigned long long *)(base + L.keys);
    S.cnt = (uint32_t *)(base + L.cnt);
    S.sub = (unsigned long long *)(base + L.sub);
    S.buf = (uint64_t)cfg->n * L.stride;
    S.n = cfg->n;
    S.d = cfg->d;
    S.dp = L.dp;
    S.stride = L.stride;
    S.storage = L.storage;
    S.chunks = (cfg->d + 3) / 4;
    S.trace_cap = L.trace_cap;
    const bool gps = cfg->order == SSO_ORDER_GPS;
    const uint64_t th0 = threshold(gps ? cfg->cg : cfg->cw);
    const uint64_t th1 = threshold(cfg->cp);
    const uint64_t th2 = threshold(gps ? cfg->cw : cfg->cg);
    S.th0 = (uint32_t)th0;
    S.th1 = (uint32_t)th1;
    S.th2 = (uint32_t)th2;
    S.r = (uint32_t)((1ull << 56) / ((1ull << 32) - th2));
    S.lo = cfg->lo;
    S.span = cfg->hi - cfg->lo;
    S.span24 = std::ldexp(S.span, -24);
    S.key0 = (uint32_t)cfg->seed;
    S.key1 = (uint32_t)(cfg->seed >> 32);
    S.swarm = cfg->swarm_id;
    S.kind = cfg->kind;
    S.order = cfg->order;
    S.nsub = kSubSlots;
    S.lanes = ctx->lanes;

    std::vector<float> pad(L.dp, 0.0f);
    std::memcpy(pad.data(), cfg->s, sizeof(float) * cfg->d);
    std::string *err = &g_err;
    auto fail = [&](int code) {
        delete ctx;
        return code;
    };
    hipError_t e = hipMemcpyAsync((void *)S.s, pad.data(), sizeof(float) * L.dp, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return fail(hip_fail(err, e, "upload s"));
    std::vector<float> wpad, apack;
    if (cfg->kind == SSO_OBJ_RIPPLE) {
        wpad.assign(L.dp, 0.0f);
        std::memcpy(wpad.data(), cfg->w, sizeof(float) * cfg->d);
        e = hipMemcpyAsync((void *)S.w, wpad.data(), sizeof(float) * L.dp, hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) return fail(hip_fail(err, e, "upload w"));
    }
    if (cfg->kind == SSO_OBJ_DENSE) {
        apack.assign(dense_matrix_floats(cfg->d), 0.0f);
        dense_pack_matrix(cfg->a, cfg->d, apack.data());
        e = hipMemcpyAsync((void *)S.a, apack.data(), sizeof(float) * apack.size(), hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) return fail(hip_fail(err, e, "upload a"));
    }
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(hip_fail(err, e, "synchronise uploads"));
    rc = launch_init(ctx);
    if (rc != SSO_OK) {
        g_err = ctx->err;
        return fail(rc);
    }
    *out = ctx;
    return SSO_OK;
}

int sso_run(sso_ctx *ctx, uint32_t generations)
{
    if (!ctx) return SSO_E_INVAL;
    if (generations == 0) return SSO_OK;
    if (ctx->t + generations >= (1ull << 32)) {
        ctx->err = "generation counter would exceed 2^32 - 1";
        return SSO_E_UNSUPPORTED;
    }
    const int rc = launch_generations(ctx, ctx->t + 1, generations);
    if (rc == SSO_OK) ctx->t += generations;
    return rc;
}

int sso_step(sso_ctx *ctx) { return sso_run(ctx, 1); }

int sso_get_best(sso_ctx *ctx, float *g_out, float *f_out, uint32_t *idx_out, uint64_t *gen_out)
{
    if (!ctx) return SSO_E_INVAL;
    const SwarmDev &S = ctx->S;
    HIP_TRY(&ctx->err, hipStreamSynchronize(ctx->stream));
    unsigned long long key = 0;
    uint32_t count = 0;
    const int rc = current_result(ctx, &key, &count);
    if (rc != SSO_OK) return rc;
    const uint32_t low = (uint32_t)key;
    const uint32_t gidx = low >> 1, row = low & 1u;
    if (gidx >= S.n) {
        ctx->err = "no gBest recorded for the current generation";
        return SSO_E_STATE;
    }
    if (g_out) {
        std::vector<uint32_t> words(S.stride);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(S.rows) + row * S.buf + (size_t)gidx * S.stride;
        HIP_TRY(&ctx->err, hipMemcpy(words.data(), src, sizeof(uint32_t) * S.stride, hipMemcpyDeviceToHost));
        row_to_values(S, words.data(), g_out);
    }
    if (f_out) *f_out = from_orderable((uint32_t)(key >> 32));
    if (idx_out) *idx_out = gidx;
    if (gen_out) *gen_out = ctx->t;
    return SSO_OK;
}

int sso_get_state(sso_ctx *ctx, float *x, float *p, float *fp, uint64_t *t)
{
    if (!ctx) return SSO_E_INVAL;
    const SwarmDev &S = ctx->S;
    HIP_TRY(&ctx->err, hipStreamSynchronize(ctx->stream));
    if (x || p) {
        std::vector<uint32_t> rows((size_t)2 * S.buf);
        std::vector<uint32_t> st(S.n);
        HIP_TRY(&ctx->err, hipMemcpy(rows.data(), S.rows, sizeof(uint32_t) * rows.size(), hipMemcpyDeviceToHost));
        HIP_TRY(&ctx->err, hipMemcpy(st.data(), S.st, sizeof(uint32_t) * S.n, hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < S.n; ++i) {
            const uint32_t prow = st[i] & ST_ROW;
            const uint32_t *pr = rows.data() + prow * S.buf + (size_t)i * S.stride;
            const uint32_t *xr = (st[i] & ST_ALIAS) ? pr : rows.data() + (1u - prow) * S.buf + (size_t)i * S.stride;
            if (p) row_to_values(S, pr, p + (size_t)i * S.d);
            if (x) row_to_values(S, xr, x + (size_t)i * S.d);
        }
    }
    if (fp) HIP_TRY(&ctx->err, hipMemcpy(fp, S.fp, sizeof(float) * S.n, hipMemcpyDeviceToHost));
    if (t) *t = ctx->t;
    return SSO_OK;
}

int sso_set_state(sso_ctx *ctx, const float *x, const float *p, const float *fp, uint64_t t)
{
    if (!ctx) return SSO_E_INVAL;
    if (!x || !p || !fp) {
        ctx->err = "x, p and fp are required";
        return SSO_E_INVAL;
    }
    if (t >= (1ull << 32) - 1) {
        ctx->err = "generation counter must be below 2^32 - 1";
        return SSO_E_UNSUPPORTED;
    }
    const SwarmDev &S = ctx->S;
    std::vector<uint32_t> rows((size_t)2 * S.buf, 0u);
    for (uint32_t i = 0; i < S.n; ++i) {
        if (!values_to_row(S, p + (size_t)i * S.d, rows.data() + (size_t)i * S.stride) ||
            !values_to_row(S, x + (size_t)i * S.d, rows.data() + S.buf + (size_t)i * S.stride)) {
            ctx->err = "a position is not on the 24-bit draw grid of [lo, hi] (use F32 storage)";
            return SSO_E_INVAL;
        }
    }
    std::vector<uint32_t> st(S.n, 0u);
    // gBest of the imported state: lowest-index argmin (pBests sit in row 0).
    unsigned long long best = ~0ull;
    for (uint32_t i = 0; i < S.n; ++i) {
        const unsigned long long k = ((unsigned long long)orderable_host(fp[i]) << 32) |
                                     ((unsigned long long)i << 1);
        if (k < best) best = k;
    }
    const uint32_t zero = 0;
    HIP_TRY(&ctx->err, hipStreamSynchronize(ctx->stream));
    HIP_TRY(&ctx->err, hipMemcpy(S.rows, rows.data(), sizeof(uint32_t) * rows.size(), hipMemcpyHostToDevice));
    HIP_TRY(&ctx->err, hipMemcpy(S.st, st.data(), sizeof(uint32_t) * S.n, hipMemcpyHostToDevice));
    HIP_TRY(&ctx->err, hipMemcpy(S.fp, fp, sizeof(float) * S.n, hipMemcpyHostToDevice));
    const int e = launch_fill_trace(S, ctx->stream);
    if (e) return hip_fail(&ctx->err, (hipError_t)e, "trace fill launch");
    HIP_TRY(&ctx->err, hipStreamSynchronize(ctx->stream));
    HIP_TRY(&ctx->err, hipMemcpy(S.keys + t % S.trace_cap, &best, sizeof best, hipMemcpyHostToDevice));
    HIP_TRY(&ctx->err, hipMemcpy(S.cnt + t % S.trace_cap, &zero, sizeof zero, hipMemcpyHostToDevice));
    // The next generation finds gBest in sub-slot 0 of generation t's group.
    unsigned long long *slot0 = S.sub + (size_t)(t % kGroups) * kSubSlots * kSubStride;
    HIP_TRY(&ctx->err, hipMemcpy(slot0, &best, sizeof best, hipMemcpyHostToDevice));
    ctx->t = t;
    ctx->trace_base = t;
    return SSO_OK;
}

int sso_get_trace(sso_ctx *ctx, uint64_t first, uint32_t count, float *fg, uint32_t *gidx, uint32_t *improved)
{
    if (!ctx) return SSO_E_INVAL;
    const SwarmDev &S = ctx->S;
    if (count == 0) return SSO_OK;
    const uint64_t last = first + count - 1;
    const uint64_t oldest_kept = ctx->t + 3 > S.trace_cap ? ctx->t + 3 - S.trace_cap : 0;
    if (first < ctx->trace_base || first < oldest_kept || last > ctx->t) {
        ctx->err = "requested generations are not in the trace window";
        return SSO_E_STATE;
    }
    HIP_TRY(&ctx->err, hipStreamSynchronize(ctx->stream));
    std::vector<unsigned long long> keys(S.trace_cap);
    std::vector<uint32_t> cnt(S.trace_cap);
    HIP_TRY(&ctx->err, hipMemcpy(keys.data(), S.keys, sizeof(unsigned long long) * S.trace_cap, hipMemcpyDeviceToHost));
    HIP_TRY(&ctx->err, hipMemcpy(cnt.data(), S.cnt, sizeof(uint32_t) * S.trace_cap, hipMemcpyDeviceToHost));
    if (last == ctx->t) {
        unsigned long long key = 0;
        uint32_t c = 0;
        const int rc = current_result(ctx, &key, &c);
        if (rc != SSO_OK) return rc;
        keys[ctx->t % S.trace_cap] = key;
        cnt[ctx->t % S.trace_cap] = c;
    }
    for (uint32_t k = 0; k < count; ++k) {
        const uint32_t slot = (uint32_t)((first + k) % S.trace_cap);
        if (fg) fg[k] = from_orderable((uint32_t)(keys[slot] >> 32));
        if (gidx) gidx[k] = (uint32_t)keys[slot] >> 1;
        if (improved) improved[k] = cnt[slot];
    }
    return SSO_OK;
}

int sso_debug_rng(sso_ctx *ctx, uint64_t t, uint32_t *dev_words)
{
    if (!ctx || !dev_words) return SSO_E_INVAL;
    if (t >= (1ull << 32)) {
        ctx->err = "t must be below 2^32";
        return SSO_E_INVAL;
    }
    const int e = launch_debug_rng(ctx->S, (uint32_t)t, dev_words, ctx->stream);
    if (e) return hip_fail(&ctx->err, (hipError_t)e, "debug rng launch");
    return SSO_OK;
}

void sso_destroy(sso_ctx *ctx) { delete ctx; }

const char *sso_strerror(int code)
{
    switch (code) {
    case SSO_OK: return "ok";
    case SSO_E_INVAL: return "invalid argument";
    case SSO_E_NOMEM: return "workspace too small";
    case SSO_E_HIP: return "HIP runtime error";
    case SSO_E_UNSUPPORTED: return "unsupported size or device";
    case SSO_E_STATE: return "call out of order";
    default: return "unknown error";
    }
}

const char *sso_last_error(const sso_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

}  // extern "C"
