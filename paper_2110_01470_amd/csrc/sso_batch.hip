// Host side of the batched-swarm C ABI (include/sso.h): validation, the
// workspace layout of many swarms, the workgroup mapping and its autotuner,
// and the graph that replays blocks of generations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "sso.h"
#include "sso_host.hpp"
#include "sso_layout.hpp"

using namespace sso;
using namespace sso::host;

namespace {

constexpr uint32_t kGraphBlock = 50;       // generations per replayed graph
constexpr uint32_t kMaxSwarms = 1u << 20;
constexpr uint32_t kBatchMaxD = 1024;      // LDS staging of s, w and gBest
constexpr uint32_t kMinWaves = 4;          // smallest workgroup the batched kernel is built for
constexpr uint32_t kSubPerSlot = 8;        // workgroups per gBest sub-slot, at most
const uint32_t kCandidates[] = {1, 2, 4, 8, 16};   // mapping rules (chunks per lane)
const uint32_t kWaveCandidates[] = {4, 8};          // waves per workgroup
constexpr uint32_t kDefaultCpl = 8;
constexpr uint32_t kDefaultWaves = kStreamWaves;

thread_local std::string g_err;

}  // namespace

struct sso_batch {
    std::vector<SwarmDev> S;          // host copies of the swarm table
    std::vector<uint32_t> fixed;      // lanes fixed by the config (0 = rule)
    std::vector<uint64_t> trace_base; // per swarm: oldest generation in its trace
    BatchDev B{};
    uint32_t *tiles_dev = nullptr;
    SwarmDev *table_dev = nullptr;
    size_t max_tiles = 0;
    uint32_t cpl = kDefaultCpl;
    uint32_t waves = kDefaultWaves;
    hipStream_t stream = nullptr;
    uint64_t t = 0;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

struct BatchLayout {
    size_t head, results, table, tiles, total;
    std::vector<size_t> rows, fp, st, s, w, keys, cnt, sub;
    size_t max_tiles;
    int storage;
};

int batch_storage(const sso_config &c) { return c.storage == SSO_STORAGE_F32 ? STORE_F32 : STORE_U24; }

uint32_t chunks_of(uint32_t d) { return (d + 3) / 4; }

// 32-bit words per row: the packed chunks, rounded up to 8 words so that
// every row starts on a 32-byte boundary.  Neighbouring particles' rows are
// written in different generations (each writes only the row that is not its
// pBest), and a row ending inside a 32-byte sector made partial-sector
// writes; on the 512-swarm workload the padding takes 3 % off the HBM bytes
// per generation (a 128-byte alignment moved more bytes than it saved).
constexpr uint32_t kBatchRowAlign = 8;
uint32_t row_words(uint32_t d, int storage)
{
    const uint32_t w = (storage == STORE_U24 ? 3u : 4u) * chunks_of(d);
    return (w + kBatchRowAlign - 1u) / kBatchRowAlign * kBatchRowAlign;
}

uint32_t lanes_cap(int storage) { return storage == STORE_U24 ? 32u : 64u; }

int validate_batch(const sso_config *cfgs, uint32_t count, std::string *why)
{
    if (!cfgs) {
        *why = "cfgs is NULL";
        return SSO_E_INVAL;
    }
    if (count == 0 || count > kMaxSwarms) {
        *why = "count must be in [1, 2^20]";
        return SSO_E_INVAL;
    }
    uint64_t tiles = 0;
    for (uint32_t k = 0; k < count; ++k) {
        const sso_config &c = cfgs[k];
        // Checked as a STREAM swarm: that is the engine a batch runs.
        sso_config cs = c;
        if (cs.engine == SSO_ENGINE_AUTO) cs.engine = SSO_ENGINE_STREAM;
        std::string w;
        const int rc = validate(&cs, &w);
        if (rc != SSO_OK) {
            *why = "swarm " + std::to_string(k) + ": " + w;
            return rc;
        }
        auto bad = [&](int code, const char *msg) {
            *why = "swarm " + std::to_string(k) + ": " + msg;
            return code;
        };
        if (c.kind != SSO_OBJ_SPHERE && c.kind != SSO_OBJ_RIPPLE)
            return bad(SSO_E_UNSUPPORTED, "batches take the separable objectives (SPHERE, RIPPLE)");
        if (c.engine != SSO_ENGINE_AUTO && c.engine != SSO_ENGINE_STREAM)
            return bad(SSO_E_UNSUPPORTED, "batches run on the STREAM engine");
        if (c.d > kBatchMaxD) return bad(SSO_E_UNSUPPORTED, "batched swarms need d <= 1024");
        if (c.kind != cfgs[0].kind) return bad(SSO_E_INVAL, "all swarms of a batch need the same kind");
        if (c.order != cfgs[0].order) return bad(SSO_E_INVAL, "all swarms of a batch need the same order");
        if (batch_storage(c) != batch_storage(cfgs[0]))
            return bad(SSO_E_INVAL, "all swarms of a batch need the same storage");
        tiles += (c.n + kMinWaves - 1) / kMinWaves;
    }
    if (tiles >= (1ull << 31)) {
        *why = "the batch needs more than 2^31 workgroups per launch";
        return SSO_E_UNSUPPORTED;
    }
    return SSO_OK;
}

BatchLayout make_batch_layout(const sso_config *cfgs, uint32_t count)
{
    BatchLayout L;
    L.storage = batch_storage(cfgs[0]);
    L.max_tiles = 0;
    for (uint32_t k = 0; k < count; ++k) {
        // The most workgroups a swarm can take: 64 lanes per particle,
        // 4 waves and so 4 particles per workgroup.
        L.max_tiles += (cfgs[k].n + kMinWaves - 1) / kMinWaves;
    }
    size_t off = 0;
    L.head = off;    off += 256;
    L.results = off; off += align256((size_t)count * 2 * sizeof(unsigned long long));
    L.table = off;   off += align256((size_t)count * sizeof(SwarmDev));
    L.tiles = off;   off += align256(L.max_tiles * 2 * sizeof(uint32_t));
    for (uint32_t k = 0; k < count; ++k) {
        const sso_config &c = cfgs[k];
        const uint32_t dp = 4 * chunks_of(c.d);
        const uint32_t cap = c.trace_cap ? c.trace_cap : kDefaultTraceCap;
        L.rows.push_back(off); off += align256((size_t)2 * c.n * row_words(c.d, L.storage) * 4);
        L.fp.push_back(off);   off += align256((size_t)c.n * 4);
        L.st.push_back(off);   off += align256((size_t)c.n * 4);
        L.s.push_back(off);    off += align256((size_t)dp * 4);
        L.w.push_back(off);    off += c.kind == SSO_OBJ_RIPPLE ? align256((size_t)dp * 4) : 0;
        L.keys.push_back(off); off += align256((size_t)cap * 8);
        L.cnt.push_back(off);  off += align256((size_t)cap * 4);
        L.sub.push_back(off);  off += align256((size_t)kSubWords * 8);
    }
    L.total = off;
    return L;
}

// Lanes per particle under rule cpl: the smallest power of two L with
// L * cpl >= chunks, at most 32 (24-bit rows) or 64 (FP32 rows).
uint32_t rule_lanes(uint32_t chunks, uint32_t cpl, int storage)
{
    uint32_t L = 1;
    while (L * cpl < chunks && L < lanes_cap(storage)) L <<= 1;
    return L;
}

// Sets every swarm's lanes and sub-slot count for rule cpl and workgroups
// of `waves` waves, and builds the tile table: swarms in decreasing order of
// per-lane chunk count (the longest workgroups are dispatched first), the
// blocks of a swarm consecutive.
std::vector<uint32_t> plan(sso_batch *b, uint32_t cpl, uint32_t waves)
{
    const uint32_t count = (uint32_t)b->S.size();
    std::vector<uint32_t> tiles_of(count);
    std::vector<uint32_t> work(count);
    for (uint32_t k = 0; k < count; ++k) {
        SwarmDev &S = b->S[k];
        const uint32_t L = b->fixed[k] ? b->fixed[k] : rule_lanes(S.chunks, cpl, S.storage);
        const uint32_t per_block = waves * (64 / L);
        S.lanes = L;
        tiles_of[k] = (S.n + per_block - 1) / per_block;
        uint32_t nsub = 1;
        while (nsub < kSubSlots && nsub * kSubPerSlot < tiles_of[k]) nsub <<= 1;
        S.nsub = nsub;
        work[k] = (S.chunks + L - 1) / L;
    }
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return work[a] > work[c]; });
    std::vector<uint32_t> tiles;
    for (uint32_t k : order)
        for (uint32_t blk = 0; blk < tiles_of[k]; ++blk) {
            tiles.push_back(k);
            tiles.push_back(blk);
        }
    b->cpl = cpl;
    b->waves = waves;
    return tiles;
}

#define BHIP(call)                                                  \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail(&b->err, e_, #call);  \
    } while (0)

void drop_graph(sso_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

// Uploads the mapping of rule cpl and workgroup size `waves` (swarm table
// and tile table); synchronous.
int apply_plan(sso_batch *b, uint32_t cpl, uint32_t waves)
{
    const std::vector<uint32_t> tiles = plan(b, cpl, waves);
    drop_graph(b);
    BHIP(hipStreamSynchronize(b->stream));
    BHIP(hipMemcpy(b->table_dev, b->S.data(), sizeof(SwarmDev) * b->S.size(), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(b->tiles_dev, tiles.data(), sizeof(uint32_t) * tiles.size(), hipMemcpyHostToDevice));
    b->B.ntiles = (uint32_t)(tiles.size() / 2);
    b->B.waves = waves;
    return SSO_OK;
}

// Clears every trace and sub-slot group and enqueues generation 0.
int start(sso_batch *b)
{
    int e = launch_batch_fill(b->B, b->stream);
    if (e) return hip_fail(&b->err, (hipError_t)e, "batch fill launch");
    e = launch_batch_init(b->B, b->stream);
    if (e) return hip_fail(&b->err, (hipError_t)e, "batch init launch");
    b->t = 0;
    std::fill(b->trace_base.begin(), b->trace_base.end(), 0);
    return SSO_OK;
}

int enqueue(sso_batch *b, uint32_t generations)
{
    int e = launch_batch_set_base(b->B, (uint32_t)b->t, b->stream);
    if (e) return hip_fail(&b->err, (hipError_t)e, "batch base launch");
    uint32_t left = generations;
    if (left >= kGraphBlock && !b->exec) {
        void *g = nullptr;
        e = batch_graph(b->B, kGraphBlock, &g);
        if (e) return hip_fail(&b->err, (hipError_t)e, "batch graph build");
        hipGraphExec_t ex = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ex, (hipGraph_t)g, nullptr, nullptr, 0);
        (void)hipGraphDestroy((hipGraph_t)g);
        if (ie != hipSuccess) return hip_fail(&b->err, ie, "batch graph instantiate");
        b->exec = ex;
    }
    while (left >= kGraphBlock) {
        BHIP(hipGraphLaunch(b->exec, b->stream));
        left -= kGraphBlock;
    }
    if (left) {
        e = launch_batch_generations(b->B, left, b->stream);
        if (e) return hip_fail(&b->err, (hipError_t)e, "batch generation launch");
    }
    return SSO_OK;
}

bool check_swarm(sso_batch *b, uint32_t k)
{
    if (k < b->S.size()) return true;
    b->err = "swarm index out of range";
    return false;
}

}  // namespace

extern "C" {

size_t sso_batch_workspace_bytes(const sso_config *cfgs, uint32_t count)
{
    std::string why;
    if (validate_batch(cfgs, count, &why) != SSO_OK) {
        g_err = why;
        return 0;
    }
    return make_batch_layout(cfgs, count).total;
}

int sso_batch_init(const sso_config *cfgs, uint32_t count, void *ws, size_t ws_bytes, void *stream,
                   sso_batch **out)
{
    if (!out) {
        g_err = "out is NULL";
        return SSO_E_INVAL;
    }
    *out = nullptr;
    std::string why;
    int rc = validate_batch(cfgs, count, &why);
    if (rc != SSO_OK) {
        g_err = why;
        return rc;
    }
    const BatchLayout L = make_batch_layout(cfgs, count);
    if (!ws || ((uintptr_t)ws & 255u)) {
        g_err = "workspace must be a non-NULL, 256-byte aligned device pointer";
        return SSO_E_INVAL;
    }
    if (ws_bytes < L.total) {
        g_err = "workspace smaller than sso_batch_workspace_bytes()";
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

    sso_batch *b = new sso_batch();
    b->stream = (hipStream_t)stream;
    char *base = (char *)ws;
    b->S.resize(count);
    b->fixed.resize(count);
    b->trace_base.assign(count, 0);
    uint32_t max_chunks = 1;
    for (uint32_t k = 0; k < count; ++k) {
        const sso_config &c = cfgs[k];
        SwarmDev &S = b->S[k];
        S = SwarmDev{};
        S.rows = (float *)(base + L.rows[k]);
        S.fp = (float *)(base + L.fp[k]);
        S.st = (uint32_t *)(base + L.st[k]);
        S.s = (const float *)(base + L.s[k]);
        S.w = c.kind == SSO_OBJ_RIPPLE ? (const float *)(base + L.w[k]) : nullptr;
        S.a = nullptr;
        S.keys = (unsigned long long *)(base + L.keys[k]);
        S.cnt = (uint32_t *)(base + L.cnt[k]);
        S.sub = (unsigned long long *)(base + L.sub[k]);
        S.n = c.n;
        S.d = c.d;
        S.chunks = chunks_of(c.d);
        S.dp = 4 * S.chunks;
        S.stride = row_words(c.d, L.storage);
        S.buf = (uint64_t)c.n * S.stride;
        S.storage = L.storage;
        S.trace_cap = c.trace_cap ? c.trace_cap : kDefaultTraceCap;
        set_params(c, S);
        b->fixed[k] = c.lanes;
        max_chunks = std::max(max_chunks, S.chunks);
    }
    b->table_dev = (SwarmDev *)(base + L.table);
    b->tiles_dev = (uint32_t *)(base + L.tiles);
    b->max_tiles = L.max_tiles;
    BatchDev &B = b->B;
    B.table = b->table_dev;
    B.tiles = b->tiles_dev;
    B.tbase = (uint32_t *)(base + L.head);
    B.results = (unsigned long long *)(base + L.results);
    B.count = count;
    B.kind = cfgs[0].kind;
    B.order = cfgs[0].order;
    B.storage = L.storage;
    B.lds = (uint32_t)batch_stage_bytes(B.kind, B.storage, max_chunks);

    auto fail = [&](int code) {
        g_err = b->err;
        drop_graph(b);
        delete b;
        return code;
    };
    for (uint32_t k = 0; k < count; ++k) {
        rc = upload_separable(cfgs[k], b->S[k], b->stream, &b->err);
        if (rc != SSO_OK) return fail(rc);
    }
    rc = apply_plan(b, kDefaultCpl, kDefaultWaves);
    if (rc != SSO_OK) return fail(rc);
    rc = start(b);
    if (rc != SSO_OK) return fail(rc);
    *out = b;
    return SSO_OK;
}

int sso_batch_run(sso_batch *b, uint32_t generations)
{
    if (!b) return SSO_E_INVAL;
    if (generations == 0) return SSO_OK;
    if (b->t + generations >= (1ull << 32)) {
        b->err = "generation counter would exceed 2^32 - 1";
        return SSO_E_UNSUPPORTED;
    }
    const int rc = enqueue(b, generations);
    if (rc == SSO_OK) b->t += generations;
    return rc;
}

int sso_batch_tune(sso_batch *b, uint32_t generations, uint32_t *cpl_out, uint32_t *waves_out,
                   float *ms_out)
{
    if (!b) return SSO_E_INVAL;
    if (b->t != 0) {
        b->err = "sso_batch_tune needs a batch that has run no generations";
        return SSO_E_STATE;
    }
    if (generations == 0) generations = 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        b->err = "hipEventCreate failed";
        return SSO_E_HIP;
    }
    constexpr uint32_t nw = sizeof kWaveCandidates / sizeof kWaveCandidates[0];
    constexpr uint32_t nc = sizeof kCandidates / sizeof kCandidates[0];
    int rc = SSO_OK;
    float best_ms = 0.0f;
    uint32_t best = kDefaultCpl, best_waves = kDefaultWaves;
    for (uint32_t q = 0; q < nc * nw && rc == SSO_OK; ++q) {
        const uint32_t cpl = kCandidates[q / nw], waves = kWaveCandidates[q % nw];
        rc = apply_plan(b, cpl, waves);
        if (rc == SSO_OK) rc = start(b);
        if (rc == SSO_OK && hipEventRecord(e0, b->stream) != hipSuccess) rc = SSO_E_HIP;
        if (rc == SSO_OK) rc = enqueue(b, generations);
        if (rc == SSO_OK && hipEventRecord(e1, b->stream) != hipSuccess) rc = SSO_E_HIP;
        float ms = 0.0f;
        if (rc == SSO_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = SSO_E_HIP;
        if (rc == SSO_E_HIP && b->err.empty()) b->err = "event timing failed";
        if (rc != SSO_OK) break;
        if (ms_out) ms_out[q] = ms;
        if (q == 0 || ms < best_ms) {
            best_ms = ms;
            best = cpl;
            best_waves = waves;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SSO_OK) rc = apply_plan(b, best, best_waves);
    if (rc == SSO_OK) rc = start(b);
    if (rc == SSO_OK && hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = "synchronise after tuning failed";
        rc = SSO_E_HIP;
    }
    if (rc == SSO_OK && cpl_out) *cpl_out = best;
    if (rc == SSO_OK && waves_out) *waves_out = best_waves;
    return rc;
}

int sso_batch_set_mapping(sso_batch *b, uint32_t cpl, uint32_t waves)
{
    if (!b) return SSO_E_INVAL;
    if (b->t != 0) {
        b->err = "sso_batch_set_mapping needs a batch that has run no generations";
        return SSO_E_STATE;
    }
    if (cpl == 0 || cpl > 64) {
        b->err = "mapping rule (chunks per lane) must be in 1..64";
        return SSO_E_INVAL;
    }
    if (std::find(std::begin(kWaveCandidates), std::end(kWaveCandidates), waves) == std::end(kWaveCandidates)) {
        b->err = "waves per workgroup must be 4 or 8";
        return SSO_E_INVAL;
    }
    int rc = apply_plan(b, cpl, waves);
    if (rc == SSO_OK) rc = start(b);
    return rc;
}

int sso_batch_mapping(sso_batch *b, uint32_t *cpl_out, uint32_t *waves_out, uint32_t *lanes_out,
                      uint32_t *tiles_out)
{
    if (!b) return SSO_E_INVAL;
    if (cpl_out) *cpl_out = b->cpl;
    if (waves_out) *waves_out = b->waves;
    if (lanes_out)
        for (size_t k = 0; k < b->S.size(); ++k) lanes_out[k] = b->S[k].lanes;
    if (tiles_out) *tiles_out = b->B.ntiles;
    return SSO_OK;
}

int sso_batch_get_results(sso_batch *b, float *f_out, uint32_t *idx_out, uint32_t *improved_out,
                          uint64_t *gen_out)
{
    if (!b) return SSO_E_INVAL;
    const int e = launch_batch_collect(b->B, (uint32_t)b->t, b->stream);
    if (e) return hip_fail(&b->err, (hipError_t)e, "batch collect launch");
    BHIP(hipStreamSynchronize(b->stream));
    std::vector<unsigned long long> res((size_t)2 * b->B.count);
    BHIP(hipMemcpy(res.data(), b->B.results, sizeof(unsigned long long) * res.size(), hipMemcpyDeviceToHost));
    for (uint32_t k = 0; k < b->B.count; ++k) {
        const unsigned long long key = res[2 * k];
        if (f_out) f_out[k] = from_orderable((uint32_t)(key >> 32));
        if (idx_out) idx_out[k] = (uint32_t)key >> 1;
        if (improved_out) improved_out[k] = (uint32_t)res[2 * k + 1];
    }
    if (gen_out) *gen_out = b->t;
    return SSO_OK;
}

int sso_batch_get_best(sso_batch *b, uint32_t k, float *g_out, float *f_out, uint32_t *idx_out)
{
    if (!b) return SSO_E_INVAL;
    if (!check_swarm(b, k)) return SSO_E_INVAL;
    return get_best(b->S[k], b->stream, b->t, &b->err, g_out, f_out, idx_out);
}

int sso_batch_get_state(sso_batch *b, uint32_t k, float *x, float *p, float *fp, uint64_t *t)
{
    if (!b) return SSO_E_INVAL;
    if (!check_swarm(b, k)) return SSO_E_INVAL;
    const int rc = get_state(b->S[k], b->stream, &b->err, x, p, fp);
    if (rc == SSO_OK && t) *t = b->t;
    return rc;
}

int sso_batch_set_state(sso_batch *b, uint32_t k, const float *x, const float *p, const float *fp,
                        uint64_t t)
{
    if (!b) return SSO_E_INVAL;
    if (!check_swarm(b, k)) return SSO_E_INVAL;
    if (!x || !p || !fp) {
        b->err = "x, p and fp are required";
        return SSO_E_INVAL;
    }
    if (t != b->t) {
        b->err = "a batched swarm's state must carry the batch's generation count";
        return SSO_E_STATE;
    }
    const int rc = set_state(b->S[k], b->stream, t, &b->err, x, p, fp);
    if (rc == SSO_OK) b->trace_base[k] = t;
    return rc;
}

int sso_batch_get_trace(sso_batch *b, uint32_t k, uint64_t first, uint32_t count, float *fg,
                        uint32_t *gidx, uint32_t *improved)
{
    if (!b) return SSO_E_INVAL;
    if (!check_swarm(b, k)) return SSO_E_INVAL;
    return get_trace(b->S[k], b->stream, b->t, b->trace_base[k], &b->err, first, count, fg, gidx,
                     improved);
}

void sso_batch_destroy(sso_batch *b)
{
    if (!b) return;
    drop_graph(b);
    delete b;
}

const char *sso_batch_last_error(const sso_batch *b) { return b ? b->err.c_str() : g_err.c_str(); }

}  // extern "C"
