// Host side of the one-swarm C ABI declared in include/sso.h: workspace
// layout, uploads and kernel dispatch (checks and state import/export are in
// host_swarm.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sso.h"
#include "sso_device.hpp"
#include "sso_host.hpp"
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
    // DENSE: the matrix (host, row-major) for sigma_max, and the polish schedule.
    std::vector<float> a_host;
    double sigma_max = 0.0;  // 0 until first needed
    uint32_t polish_every = 0, polish_steps = 0;
    float polish_lr = 0.0f;
    std::string err;
};

namespace {

using namespace sso::host;

// Detail of the calling thread's last failed context-less call, kept in a
// fixed buffer so that setting it allocates nothing.
struct ErrText {
    char buf[512];
    ErrText &operator=(const char *m)
    {
        std::snprintf(buf, sizeof buf, "%s", m);
        return *this;
    }
    ErrText &operator=(const std::string &m) { return *this = m.c_str(); }
    const char *c_str() const { return buf; }
};
thread_local ErrText g_err;

struct Layout {
    size_t rows, fp, st, s, w, a, at, a3, keys, cnt, sub, total;
    uint32_t dp, stride, trace_cap;
    int engine, storage;
};

// The DENSE generation kernel takes a split contraction (bf16 or fp16
// parts of A in the workspace; the bf16 form is the larger) unless the FP32
// one is asked for.
bool split_contraction(const sso_config &c)
{
    return c.kind == SSO_OBJ_DENSE && c.contraction != SSO_CONTRACT_F32;
}
static_assert(kRowAlign >= 32, "the fp16 split and its scales fit the bf16 split's region when dp >= 32");

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
    L.at = off;   off += c.kind == SSO_OBJ_DENSE ? align256(dense_matrix_floats(c.d) * sizeof(float)) : 0;
    L.a3 = off;   off += split_contraction(c) ? align256(dense_split_halves(c.d) * sizeof(uint16_t)) : 0;
    L.keys = off; off += align256((size_t)L.trace_cap * sizeof(unsigned long long));
    L.cnt = off;  off += align256((size_t)L.trace_cap * sizeof(uint32_t));
    L.sub = off;  off += align256((size_t)kSubWords * sizeof(unsigned long long));
    L.total = off;
    return L;
}

// Largest singular value of the DENSE matrix: power iteration on A^T A in
// FP64 from the all-ones vector; the Rayleigh quotient ||A v||^2 converges
// monotonically from below.  Run once, when a default step size is needed.
double sigma_max(sso_ctx *ctx)
{
    if (ctx->sigma_max > 0.0) return ctx->sigma_max;
    const uint32_t d = ctx->S.d;
    const std::vector<float> &a = ctx->a_host;
    std::vector<double> v(d, 1.0 / std::sqrt((double)d)), y(d), w(d);
    double lam = 0.0;
    for (int it = 0; it < 5000; ++it) {
        for (uint32_t k = 0; k < d; ++k) {
            double acc = 0.0;
            for (uint32_t j = 0; j < d; ++j) acc += (double)a[(size_t)k * d + j] * v[j];
            y[k] = acc;
        }
        double ny = 0.0;
        for (uint32_t k = 0; k < d; ++k) ny += y[k] * y[k];
        for (uint32_t j = 0; j < d; ++j) {
            double acc = 0.0;
            for (uint32_t k = 0; k < d; ++k) acc += (double)a[(size_t)k * d + j] * y[k];
            w[j] = acc;
        }
        double nw = 0.0;
        for (uint32_t j = 0; j < d; ++j) nw += w[j] * w[j];
        nw = std::sqrt(nw);
        const double prev = lam;
        lam = ny;  // v has unit norm: v^T A^T A v
        if (nw == 0.0) break;
        for (uint32_t j = 0; j < d; ++j) v[j] = w[j] / nw;
        if (it > 0 && std::fabs(lam - prev) <= 1e-15 * lam) break;
    }
    ctx->sigma_max = std::sqrt(lam);
    return ctx->sigma_max;
}

// The polish step size: lr, or 0.05 / sigma_max^2 when lr <= 0.
float polish_step_size(sso_ctx *ctx, float lr)
{
    if (lr > 0.0f) return lr;
    const double s = sigma_max(ctx);
    return s > 0.0 ? (float)(0.05 / (s * s)) : 0.0f;
}

// Lanes per particle of a STREAM swarm: the configured count, else the
// default rule.
uint32_t swarm_lanes(const sso_config &c, const Layout &L)
{
    return (L.engine == SSO_ENGINE_STREAM && c.lanes) ? c.lanes : stream_lanes(c.d, L.storage);
}

// Points the swarm's device arrays at their regions of the workspace `base`
// and fills in the sizes and the method's parameters.
void bind_layout(const sso_config &c, const Layout &L, char *base, uint32_t lanes, SwarmDev &S)
{
    S.rows = (float *)(base + L.rows);
    S.fp = (float *)(base + L.fp);
    S.st = (uint32_t *)(base + L.st);
    S.s = (const float *)(base + L.s);
    S.w = c.kind == SSO_OBJ_RIPPLE ? (const float *)(base + L.w) : nullptr;
    S.a = c.kind == SSO_OBJ_DENSE ? (const float *)(base + L.a) : nullptr;
    S.at = c.kind == SSO_OBJ_DENSE ? (const float *)(base + L.at) : nullptr;
    S.a3 = split_contraction(c) ? (const uint16_t *)(base + L.a3) : nullptr;
    S.split = resolve_contraction(c) == SSO_CONTRACT_F16X2 ? SPLIT_F16X2 : SPLIT_BF16X3;
    S.keys = (unsigned long long *)(base + L.keys);
    S.cnt = (uint32_t *)(base + L.cnt);
    S.sub = (unsigned long long *)(base + L.sub);
    S.buf = (uint64_t)c.n * L.stride;
    S.n = c.n;
    S.d = c.d;
    S.dp = L.dp;
    S.stride = L.stride;
    S.storage = L.storage;
    S.chunks = (c.d + 3) / 4;
    S.trace_cap = L.trace_cap;
    set_params(c, S);
    S.nsub = kSubSlots;
    S.lanes = lanes;
}

// Enqueues generations t_first .. t_first + count - 1 of a swarm with no
// polish schedule (one launch per generation, or one RESIDENT launch for all).
hipError_t enqueue_generations(const SwarmDev &S, int engine, uint32_t lanes, uint64_t t_first,
                               uint32_t count, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    if (engine == SSO_ENGINE_RESIDENT) return (hipError_t)launch_resident(S, (uint32_t)t_first, count, stream);
    for (uint32_t k = 0; k < count; ++k) {
        const uint32_t t = (uint32_t)(t_first + k);
        const int e = S.kind == SSO_OBJ_DENSE ? launch_dense_generation(S, t, stream)
                                              : launch_stream_generation(S, t, lanes, stream);
        if (e) return (hipError_t)e;
    }
    return hipSuccess;
}

int launch_generations(sso_ctx *ctx, uint64_t t_first, uint32_t count)
{
    const SwarmDev &S = ctx->S;
    if (!ctx->polish_every) {
        const hipError_t e = enqueue_generations(S, ctx->engine, ctx->lanes, t_first, count, ctx->stream);
        if (e != hipSuccess) return hip_fail(&ctx->err, e, "generation kernel launch");
        return SSO_OK;
    }
    const float lr = ctx->polish_every ? polish_step_size(ctx, ctx->polish_lr) : 0.0f;
    for (uint32_t k = 0; k < count; ++k) {
        const uint32_t t = (uint32_t)(t_first + k);
        int e = S.kind == SSO_OBJ_DENSE ? launch_dense_generation(S, t, ctx->stream)
                                        : launch_stream_generation(S, t, ctx->lanes, ctx->stream);
        if (e) return hip_fail(&ctx->err, (hipError_t)e, "generation kernel launch");
        if (ctx->polish_every && t % ctx->polish_every == 0) {
            e = launch_dense_polish(S, ctx->polish_steps, lr, t, ctx->stream);
            if (e) return hip_fail(&ctx->err, (hipError_t)e, "polish kernel launch");
        }
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

// ---------------------------------------------------------------------------
// Allocation-free run (sso_run_static).  The swarm's state lives in one
// library-owned device array per GPU instead of a caller workspace.  In host
// code `scratch` names a host-side stand-in, not the device memory: host code
// uses only the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr size_t kStaticBytes = (size_t)SSO_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];  // device address of `scratch` per device, once set up

// The array's address on device `dev` (current), looked up on the first call
// for that device; *why is set on failure.
void *static_scratch(int dev, const char **why)
{
    if (dev < 0 || dev >= kMaxDevices) {
        *why = "device ordinal beyond the allocation-free run's device table (64)";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr || ((uintptr_t)ptr & 255u)) {
            *why = "hipGetSymbolAddress of the static state array failed";
            return nullptr;
        }
        g_static_ptr[dev] = ptr;
    }
    return g_static_ptr[dev];
}

// Zero padding of s and w beyond d (the whole of s when there is no shift):
// the kernels read whole chunks of the staged arrays.  A kernel rather than a
// memset, like the trace fill.
__global__ void k_static_pad(float *s, float *w, uint32_t from_s, uint32_t d, uint32_t dp)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < dp && j >= from_s) s[j] = 0.0f;
    if (w && j < dp && j >= d) w[j] = 0.0f;
}

// gBest of generation t into device memory: the lowest key over the 64
// sub-slots of generation t's group (Algorithm 4's argmin, as the next
// generation would take it), its FP32 fitness, particle index and position.
__global__ __launch_bounds__(256) void k_best_out(SwarmDev S, uint32_t t, float *g, float *f,
                                                  uint32_t *idx)
{
    __shared__ unsigned long long best;
    if (threadIdx.x < 64u) {
        const unsigned long long k = wave_min_u64(*sub_key(S, t % kGroups, threadIdx.x));
        if (threadIdx.x == 0) best = k;
    }
    __syncthreads();
    const unsigned long long key = best;
    const uint32_t i = (uint32_t)key >> 1, row = (uint32_t)key & 1u;
    const bool found = i < S.n;
    if (threadIdx.x == 0) {
        const uint32_t o = (uint32_t)(key >> 32);
        const uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
        if (f) *f = found ? __uint_as_float(b) : __uint_as_float(0x7FC00000u);
        if (idx) *idx = found ? i : 0xFFFFFFFFu;
    }
    if (!g || !found) return;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(S.rows) + row * S.buf + (size_t)i * S.stride;
    for (uint32_t j = threadIdx.x; j < S.d; j += blockDim.x) {
        float v;
        if (S.storage == STORE_U24) {
            const f4 q = StoreU24::value(S, StoreU24::load(src, j >> 2));
            v = q[j & 3u];
        } else {
            v = __uint_as_float(src[j]);
        }
        g[j] = v;
    }
}

}  // namespace

extern "C" {

int sso_run_static(const sso_config *cfg, uint32_t generations, void *stream, float *dev_g,
                   float *dev_f, uint32_t *dev_idx)
{
    const char *why = "";
    const int rc = validate_msg(cfg, &why);
    if (rc != SSO_OK) {
        g_err = why;
        return rc;
    }
    if (cfg->kind == SSO_OBJ_DENSE) {
        g_err = "the allocation-free run takes SPHERE, RIPPLE and F1..F9, not DENSE";
        return SSO_E_UNSUPPORTED;
    }
    if (generations >= 0xFFFFFFFFu) {
        g_err = "generations must be below 2^32 - 1";
        return SSO_E_UNSUPPORTED;
    }
    const Layout L = make_layout(*cfg);
    if (L.total > kStaticBytes) {
        std::snprintf(g_err.buf, sizeof g_err.buf,
                      "the swarm needs %zu bytes of device state; the allocation-free run's static "
                      "array holds %zu (SSO_STATIC_SCRATCH_BYTES)",
                      L.total, kStaticBytes);
        return SSO_E_NOMEM;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        g_err = "no HIP device";
        return SSO_E_HIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_err = "library is built for gfx950";
        return SSO_E_UNSUPPORTED;
    }
    char *base = (char *)static_scratch(dev, &why);
    if (!base) {
        g_err = why;
        return SSO_E_HIP;
    }
    hipStream_t st = (hipStream_t)stream;
    SwarmDev S{};
    const uint32_t lanes = swarm_lanes(*cfg, L);
    bind_layout(*cfg, L, base, lanes, S);
    auto hip_err = [&](hipError_t e, const char *what) {
        std::snprintf(g_err.buf, sizeof g_err.buf, "%s: %s", what, hipGetErrorString(e));
        return SSO_E_HIP;
    };
    hipError_t e = hipSuccess;
    if (cfg->s)
        e = hipMemcpyAsync((void *)S.s, cfg->s, sizeof(float) * cfg->d, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && cfg->kind == SSO_OBJ_RIPPLE)
        e = hipMemcpyAsync((void *)S.w, cfg->w, sizeof(float) * cfg->d, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_err(e, "upload s, w");
    hipLaunchKernelGGL(k_static_pad, dim3((L.dp + 255u) / 256u), dim3(256), 0, st, (float *)S.s,
                       (float *)S.w, cfg->s ? cfg->d : 0u, cfg->d, L.dp);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "padding kernel launch");
    int k = launch_fill_trace(S, st);
    if (!k) k = launch_stream_generation(S, 0, lanes, st);
    if (k) return hip_err((hipError_t)k, "initialisation launch");
    e = enqueue_generations(S, L.engine, lanes, 1, generations, st);
    if (e != hipSuccess) return hip_err(e, "generation kernel launch");
    hipLaunchKernelGGL(k_best_out, dim3(1), dim3(256), 0, st, S, generations, dev_g, dev_f, dev_idx);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "gBest copy launch");
    return SSO_OK;
}

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
    ctx->lanes = swarm_lanes(*cfg, L);

    SwarmDev &S = ctx->S;
    bind_layout(*cfg, L, (char *)ws, ctx->lanes, S);

    std::string err_text;
    std::string *err = &err_text;
    auto fail = [&](int code) {
        g_err = err_text;
        delete ctx;
        return code;
    };
    rc = upload_separable(*cfg, S, ctx->stream, err);
    if (rc != SSO_OK) return fail(rc);
    std::vector<float> apack, atpack;
    std::vector<uint16_t> a3pack;
    if (cfg->kind == SSO_OBJ_DENSE) {
        const uint32_t d = cfg->d;
        ctx->a_host.assign(cfg->a, cfg->a + (size_t)d * d);
        std::vector<float> at((size_t)d * d);
        for (uint32_t k = 0; k < d; ++k)
            for (uint32_t j = 0; j < d; ++j) at[(size_t)j * d + k] = cfg->a[(size_t)k * d + j];
        apack.assign(dense_matrix_floats(d), 0.0f);
        atpack.assign(dense_matrix_floats(d), 0.0f);
        dense_pack_matrix(cfg->a, d, apack.data());
        dense_pack_matrix(at.data(), d, atpack.data());
        hipError_t e = hipMemcpyAsync((void *)S.a, apack.data(), sizeof(float) * apack.size(),
                                      hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)S.at, atpack.data(), sizeof(float) * atpack.size(),
                               hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess && S.a3) {
            a3pack.assign(dense_split_halves(d), 0);
            if (S.split == SPLIT_F16X2)
                (void)dense_pack_f16x2(cfg->a, d, cfg->s, cfg->lo, cfg->hi, a3pack.data());  // fits: resolved so
            else
                dense_pack_split(cfg->a, d, a3pack.data());
            e = hipMemcpyAsync((void *)S.a3, a3pack.data(), sizeof(uint16_t) * a3pack.size(),
                               hipMemcpyHostToDevice, ctx->stream);
        }
        if (e != hipSuccess) return fail(hip_fail(err, e, "upload a"));
        ctx->polish_every = cfg->polish_every;
        ctx->polish_steps = cfg->polish_steps;
        ctx->polish_lr = cfg->polish_lr;
    }
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(hip_fail(err, e, "synchronise uploads"));
    rc = launch_init(ctx);
    if (rc != SSO_OK) {
        err_text = ctx->err;
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
    const int rc = get_best(ctx->S, ctx->stream, ctx->t, &ctx->err, g_out, f_out, idx_out);
    if (rc == SSO_OK && gen_out) *gen_out = ctx->t;
    return rc;
}

int sso_get_state(sso_ctx *ctx, float *x, float *p, float *fp, uint64_t *t)
{
    if (!ctx) return SSO_E_INVAL;
    const int rc = get_state(ctx->S, ctx->stream, &ctx->err, x, p, fp);
    if (rc == SSO_OK && t) *t = ctx->t;
    return rc;
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
    const int rc = set_state(ctx->S, ctx->stream, t, &ctx->err, x, p, fp);
    if (rc != SSO_OK) return rc;
    ctx->t = t;
    ctx->trace_base = t;
    return SSO_OK;
}

int sso_get_trace(sso_ctx *ctx, uint64_t first, uint32_t count, float *fg, uint32_t *gidx, uint32_t *improved)
{
    if (!ctx) return SSO_E_INVAL;
    return get_trace(ctx->S, ctx->stream, ctx->t, ctx->trace_base, &ctx->err, first, count, fg, gidx,
                     improved);
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

int sso_eval(sso_ctx *ctx, const float *dev_x, uint32_t m, const float *dev_gout, float *f_out,
             float *grad_out)
{
    if (!ctx) return SSO_E_INVAL;
    if (ctx->S.kind != SSO_OBJ_DENSE) {
        ctx->err = "sso_eval needs the dense objective";
        return SSO_E_UNSUPPORTED;
    }
    if (m && !dev_x) {
        ctx->err = "x is NULL";
        return SSO_E_INVAL;
    }
    if (m >= (1u << 31)) {
        ctx->err = "m must be below 2^31";
        return SSO_E_UNSUPPORTED;
    }
    GradArgs G{};
    G.x = dev_x;
    G.gout = dev_gout;
    G.f = f_out;
    G.g = grad_out;
    G.m = m;
    G.ld = ctx->S.d;
    const int e = launch_dense_eval(ctx->S, G, ctx->stream);
    if (e) return hip_fail(&ctx->err, (hipError_t)e, "dense eval launch");
    return SSO_OK;
}

int sso_polish(sso_ctx *ctx, uint32_t steps, float lr, float *lr_used)
{
    if (!ctx) return SSO_E_INVAL;
    if (ctx->S.kind != SSO_OBJ_DENSE) {
        ctx->err = "sso_polish needs the dense objective";
        return SSO_E_UNSUPPORTED;
    }
    if (!(lr == lr) || std::isinf(lr)) {
        ctx->err = "lr must be finite";
        return SSO_E_INVAL;
    }
    const float step = polish_step_size(ctx, lr);
    const int e = launch_dense_polish(ctx->S, steps, step, (uint32_t)ctx->t, ctx->stream);
    if (e) return hip_fail(&ctx->err, (hipError_t)e, "polish kernel launch");
    if (lr_used) *lr_used = step;
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

int sso_get_mapping(const sso_ctx *ctx, int *engine_out, int *storage_out, uint32_t *lanes_out,
                    int *contraction_out)
{
    if (!ctx) return SSO_E_INVAL;
    if (engine_out) *engine_out = ctx->engine;
    if (storage_out) *storage_out = ctx->storage == STORE_U24 ? SSO_STORAGE_U24 : SSO_STORAGE_F32;
    if (lanes_out) *lanes_out = ctx->S.lanes;
    if (contraction_out)
        *contraction_out = !ctx->S.a3 ? SSO_CONTRACT_F32
                                      : ctx->S.split == SPLIT_F16X2 ? SSO_CONTRACT_F16X2 : SSO_CONTRACT_BF16X3;
    return SSO_OK;
}

}  // extern "C"
