// Host helpers of sso_host.hpp.  No arithmetic of the method runs here
// except the integer thresholds (Eq. 2.1 in integer form) and, when a state
// is imported, the lowest-index argmin that defines its gBest (Algorithm 4).
#include "sso_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

namespace sso {
namespace host {

namespace {

constexpr uint32_t kMaxD = 1u << 20;

#define HIP_TRY(err, call)                                     \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(err, e_, #call); \
    } while (0)

bool same_bits(float a, float b) { return std::memcmp(&a, &b, sizeof a) == 0; }

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

bool resident_possible(const sso_config &c)
{
    if (!resident_fits(c.n, c.d, c.kind)) return false;
    // Table 3.2's functions: one workgroup's time grows with the waves of
    // particles each SIMD walks (N L / 256), by 0.2-0.5 us per wave (more for
    // the functions with transcendentals), while a launch per generation
    // costs 4.3-5.1 us whatever N; the limits are where the two meet,
    // measured at D = 50 and N = 100, 200, 256.
    if (!is_paper_kind(c.kind)) return true;
    const uint64_t waves = ((uint64_t)c.n * stream_lanes(c.d, STORE_F32) + 255u) / 256u;
    return waves <= kResidentPaperAutoWaves[c.kind - SSO_OBJ_F1_SPHERE];
}

}  // namespace

size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

uint32_t stream_lanes(uint32_t d, int storage)
{
    const uint32_t chunks = (d + 3) / 4;
    const uint32_t cap = storage == STORE_U24 ? 32u : 64u;
    uint32_t L = 8;
    while (L < chunks && L < cap) L <<= 1;
    return L;
}

uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

uint64_t threshold(double c) { return (uint64_t)std::ceil(c * 4294967296.0); }

void resolve(const sso_config &c, int *engine, int *storage)
{
    int e = c.engine;
    if (c.kind == SSO_OBJ_DENSE) e = SSO_ENGINE_STREAM;
    if (e == SSO_ENGINE_AUTO) e = resident_possible(c) ? SSO_ENGINE_RESIDENT : SSO_ENGINE_STREAM;
    *engine = e;
    const bool packable = e == SSO_ENGINE_STREAM && c.kind != SSO_OBJ_DENSE;
    *storage = (c.storage == SSO_STORAGE_F32 || !packable) ? STORE_F32 : STORE_U24;
}

int resolve_contraction(const sso_config &c)
{
    if (c.kind != SSO_OBJ_DENSE || c.contraction == SSO_CONTRACT_F32) return SSO_CONTRACT_F32;
    if (c.contraction == SSO_CONTRACT_BF16X3) return SSO_CONTRACT_BF16X3;
    if (c.contraction == SSO_CONTRACT_F16X2) return SSO_CONTRACT_F16X2;
    return dense_pack_f16x2(c.a, c.d, c.s, c.lo, c.hi, nullptr) ? SSO_CONTRACT_F16X2 : SSO_CONTRACT_BF16X3;
}

int validate(const sso_config *c, std::string *why)
{
    const char *msg = "";
    const int rc = validate_msg(c, &msg);
    if (rc != SSO_OK) *why = msg;
    return rc;
}

int validate_msg(const sso_config *c, const char **why)
{
    auto bad = [&](int code, const char *msg) {
        *why = msg;
        return code;
    };
    if (!c) return bad(SSO_E_INVAL, "cfg is NULL");
    if (c->n == 0 || c->n >= (1u << 31)) return bad(SSO_E_INVAL, "n must be in [1, 2^31)");
    if (c->d == 0) return bad(SSO_E_INVAL, "d must be >= 1");
    if (c->d > kMaxD) return bad(SSO_E_UNSUPPORTED, "d exceeds 2^20");
    const bool paper = is_paper_kind(c->kind);
    if ((c->kind < SSO_OBJ_SPHERE || c->kind > SSO_OBJ_DENSE) && !paper)
        return bad(SSO_E_INVAL, "unknown objective kind");
    if (paper && c->d > 1024) return bad(SSO_E_UNSUPPORTED, "the Table 3.2 functions support d <= 1024");
    if (c->kind == SSO_OBJ_DENSE && c->d > kDenseMaxD) return bad(SSO_E_UNSUPPORTED, "dense objective supports d <= 256");
    if (c->order != SSO_ORDER_GPS && c->order != SSO_ORDER_EQ21) return bad(SSO_E_INVAL, "unknown interval order");
    if (c->engine < SSO_ENGINE_AUTO || c->engine > SSO_ENGINE_RESIDENT) return bad(SSO_E_INVAL, "unknown engine");
    if (c->lanes != 0 && (c->lanes < 8 || c->lanes > 64 || (c->lanes & (c->lanes - 1))))
        return bad(SSO_E_INVAL, "lanes must be 0 or a power of two in [8, 64]");
    if (c->trace_cap != 0 && c->trace_cap < 4) return bad(SSO_E_INVAL, "trace_cap must be 0 or >= 4");
    if (!c->s && !paper) return bad(SSO_E_INVAL, "s is NULL");
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
        return bad(SSO_E_UNSUPPORTED, "swarm does not fit the resident engine (one workgroup; separable objective or Table 3.2 function)");
    if (c->polish_every != 0 && c->kind != SSO_OBJ_DENSE)
        return bad(SSO_E_UNSUPPORTED, "the gradient polish needs the dense objective");
    if (!(c->polish_lr == c->polish_lr) || std::isinf(c->polish_lr)) return bad(SSO_E_INVAL, "polish_lr must be finite");
    if (c->storage < SSO_STORAGE_AUTO || c->storage > SSO_STORAGE_U24) return bad(SSO_E_INVAL, "unknown storage");
    if (c->contraction < SSO_CONTRACT_AUTO || c->contraction > SSO_CONTRACT_F16X2) return bad(SSO_E_INVAL, "unknown contraction");
    if (c->kind == SSO_OBJ_DENSE && c->contraction == SSO_CONTRACT_F16X2 &&
        !dense_pack_f16x2(c->a, c->d, c->s, c->lo, c->hi, nullptr))
        return bad(SSO_E_INVAL, "the f16x2 contraction needs finite A and s with magnitudes within 2^+-100");
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

void set_params(const sso_config &c, SwarmDev &S)
{
    const bool gps = c.order == SSO_ORDER_GPS;
    const uint64_t th0 = threshold(gps ? c.cg : c.cw);
    const uint64_t th1 = threshold(c.cp);
    const uint64_t th2 = threshold(gps ? c.cw : c.cg);
    S.th0 = (uint32_t)th0;
    S.th1 = (uint32_t)th1;
    S.th2 = (uint32_t)th2;
    S.r = (uint32_t)((1ull << 56) / ((1ull << 32) - th2));
    S.lo = c.lo;
    S.span = c.hi - c.lo;
    S.span24 = std::ldexp(S.span, -24);
    S.key0 = (uint32_t)c.seed;
    S.key1 = (uint32_t)(c.seed >> 32);
    S.swarm = c.swarm_id;
    S.kind = c.kind;
    S.order = c.order;
}

int upload_separable(const sso_config &c, const SwarmDev &S, hipStream_t st, std::string *err)
{
    std::vector<float> pad(S.dp, 0.0f);
    if (c.s) std::memcpy(pad.data(), c.s, sizeof(float) * c.d);  // Table 3.2's functions have none
    HIP_TRY(err, hipMemcpyAsync((void *)S.s, pad.data(), sizeof(float) * S.dp, hipMemcpyHostToDevice, st));
    HIP_TRY(err, hipStreamSynchronize(st));
    if (c.kind == SSO_OBJ_RIPPLE) {
        std::fill(pad.begin(), pad.end(), 0.0f);
        std::memcpy(pad.data(), c.w, sizeof(float) * c.d);
        HIP_TRY(err, hipMemcpyAsync((void *)S.w, pad.data(), sizeof(float) * S.dp, hipMemcpyHostToDevice, st));
        HIP_TRY(err, hipStreamSynchronize(st));
    }
    return SSO_OK;
}

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

int current_result(const SwarmDev &S, uint64_t t, std::string *err, unsigned long long *key,
                   uint32_t *count)
{
    std::vector<unsigned long long> grp((size_t)kSubSlots * kSubStride);
    const unsigned long long *src = S.sub + (size_t)(t % kGroups) * kSubSlots * kSubStride;
    HIP_TRY(err, hipMemcpy(grp.data(), src, sizeof(unsigned long long) * grp.size(), hipMemcpyDeviceToHost));
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

int get_best(const SwarmDev &S, hipStream_t st, uint64_t t, std::string *err, float *g_out,
             float *f_out, uint32_t *idx_out)
{
    HIP_TRY(err, hipStreamSynchronize(st));
    unsigned long long key = 0;
    uint32_t count = 0;
    const int rc = current_result(S, t, err, &key, &count);
    if (rc != SSO_OK) return rc;
    const uint32_t low = (uint32_t)key;
    const uint32_t gidx = low >> 1, row = low & 1u;
    if (gidx >= S.n) {
        *err = "no gBest recorded for the current generation";
        return SSO_E_STATE;
    }
    if (g_out) {
        std::vector<uint32_t> words(S.stride);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(S.rows) + row * S.buf + (size_t)gidx * S.stride;
        HIP_TRY(err, hipMemcpy(words.data(), src, sizeof(uint32_t) * S.stride, hipMemcpyDeviceToHost));
        row_to_values(S, words.data(), g_out);
    }
    if (f_out) *f_out = from_orderable((uint32_t)(key >> 32));
    if (idx_out) *idx_out = gidx;
    return SSO_OK;
}

int get_state(const SwarmDev &S, hipStream_t st, std::string *err, float *x, float *p, float *fp)
{
    HIP_TRY(err, hipStreamSynchronize(st));
    if (x || p) {
        std::vector<uint32_t> rows((size_t)2 * S.buf);
        std::vector<uint32_t> stw(S.n);
        HIP_TRY(err, hipMemcpy(rows.data(), S.rows, sizeof(uint32_t) * rows.size(), hipMemcpyDeviceToHost));
        HIP_TRY(err, hipMemcpy(stw.data(), S.st, sizeof(uint32_t) * S.n, hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < S.n; ++i) {
            const uint32_t prow = stw[i] & ST_ROW;
            const uint32_t *pr = rows.data() + prow * S.buf + (size_t)i * S.stride;
            const uint32_t *xr = (stw[i] & ST_ALIAS) ? pr : rows.data() + (1u - prow) * S.buf + (size_t)i * S.stride;
            if (p) row_to_values(S, pr, p + (size_t)i * S.d);
            if (x) row_to_values(S, xr, x + (size_t)i * S.d);
        }
    }
    if (fp) HIP_TRY(err, hipMemcpy(fp, S.fp, sizeof(float) * S.n, hipMemcpyDeviceToHost));
    return SSO_OK;
}

int set_state(const SwarmDev &S, hipStream_t st, uint64_t t, std::string *err, const float *x,
              const float *p, const float *fp)
{
    if (S.a3 && S.split == SPLIT_F16X2) {
        // The fp16 split's scaling holds for differences x - s of positions
        // inside the box.
        const float hi = S.lo + S.span;
        for (size_t k = 0; k < (size_t)S.n * S.d; ++k)
            if (!(x[k] >= S.lo && x[k] <= hi && p[k] >= S.lo && p[k] <= hi)) {
                *err = "with the f16x2 contraction every position must lie in [lo, hi]";
                return SSO_E_INVAL;
            }
    }
    std::vector<uint32_t> rows((size_t)2 * S.buf, 0u);
    for (uint32_t i = 0; i < S.n; ++i) {
        if (!values_to_row(S, p + (size_t)i * S.d, rows.data() + (size_t)i * S.stride) ||
            !values_to_row(S, x + (size_t)i * S.d, rows.data() + S.buf + (size_t)i * S.stride)) {
            *err = "a position is not on the 24-bit draw grid of [lo, hi] (use F32 storage)";
            return SSO_E_INVAL;
        }
    }
    std::vector<uint32_t> stw(S.n, 0u);
    // gBest of the imported state: lowest-index argmin (pBests sit in row 0).
    unsigned long long best = ~0ull;
    for (uint32_t i = 0; i < S.n; ++i) {
        const unsigned long long k = ((unsigned long long)orderable_host(fp[i]) << 32) |
                                     ((unsigned long long)i << 1);
        if (k < best) best = k;
    }
    const uint32_t zero = 0;
    HIP_TRY(err, hipStreamSynchronize(st));
    HIP_TRY(err, hipMemcpy(S.rows, rows.data(), sizeof(uint32_t) * rows.size(), hipMemcpyHostToDevice));
    HIP_TRY(err, hipMemcpy(S.st, stw.data(), sizeof(uint32_t) * S.n, hipMemcpyHostToDevice));
    HIP_TRY(err, hipMemcpy(S.fp, fp, sizeof(float) * S.n, hipMemcpyHostToDevice));
    const int e = launch_fill_trace(S, st);
    if (e) return hip_fail(err, (hipError_t)e, "trace fill launch");
    HIP_TRY(err, hipStreamSynchronize(st));
    HIP_TRY(err, hipMemcpy(S.keys + t % S.trace_cap, &best, sizeof best, hipMemcpyHostToDevice));
    HIP_TRY(err, hipMemcpy(S.cnt + t % S.trace_cap, &zero, sizeof zero, hipMemcpyHostToDevice));
    // The next generation finds gBest in sub-slot 0 of generation t's group.
    unsigned long long *slot0 = S.sub + (size_t)(t % kGroups) * kSubSlots * kSubStride;
    HIP_TRY(err, hipMemcpy(slot0, &best, sizeof best, hipMemcpyHostToDevice));
    return SSO_OK;
}

int get_trace(const SwarmDev &S, hipStream_t st, uint64_t t_now, uint64_t trace_base,
              std::string *err, uint64_t first, uint32_t count, float *fg, uint32_t *gidx,
              uint32_t *improved)
{
    if (count == 0) return SSO_OK;
    const uint64_t last = first + count - 1;
    const uint64_t oldest_kept = t_now + 3 > S.trace_cap ? t_now + 3 - S.trace_cap : 0;
    if (first < trace_base || first < oldest_kept || last > t_now) {
        *err = "requested generations are not in the trace window";
        return SSO_E_STATE;
    }
    HIP_TRY(err, hipStreamSynchronize(st));
    std::vector<unsigned long long> keys(S.trace_cap);
    std::vector<uint32_t> cnt(S.trace_cap);
    HIP_TRY(err, hipMemcpy(keys.data(), S.keys, sizeof(unsigned long long) * S.trace_cap, hipMemcpyDeviceToHost));
    HIP_TRY(err, hipMemcpy(cnt.data(), S.cnt, sizeof(uint32_t) * S.trace_cap, hipMemcpyDeviceToHost));
    if (last == t_now) {
        unsigned long long key = 0;
        uint32_t c = 0;
        const int rc = current_result(S, t_now, err, &key, &c);
        if (rc != SSO_OK) return rc;
        keys[t_now % S.trace_cap] = key;
        cnt[t_now % S.trace_cap] = c;
    }
    for (uint32_t k = 0; k < count; ++k) {
        const uint32_t slot = (uint32_t)((first + k) % S.trace_cap);
        if (fg) fg[k] = from_orderable((uint32_t)(keys[slot] >> 32));
        if (gidx) gidx[k] = (uint32_t)keys[slot] >> 1;
        if (improved) improved[k] = cnt[slot];
    }
    return SSO_OK;
}

}  // namespace host
}  // namespace sso
