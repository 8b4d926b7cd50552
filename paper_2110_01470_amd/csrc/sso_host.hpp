// Host helpers shared by the one-swarm API (sso_api.hip) and the batch API
// (sso_batch.hip): configuration checks, per-swarm parameters, uploads, and
// the state import/export of one swarm held in device memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "sso.h"
#include "sso_layout.hpp"

namespace sso {
namespace host {

constexpr uint32_t kDefaultTraceCap = 4096;

size_t align256(size_t x);
// Lanes per particle for the STREAM engine: the chunk count rounded up to a
// power of two, at least 8, at most 32 with 24-bit rows and 64 with FP32 rows
// (measured on the ripple workload with D=1000: U24 131.9 us at 32 lanes vs
// 135.1 at 64; F32 160.2 us at 64 vs 172.1 at 32).  The RESIDENT engine's
// kernel for Table 3.2's functions uses the same count.
uint32_t stream_lanes(uint32_t d, int storage);
// Table 3.2's functions on the RESIDENT engine (resident.hip): particles per
// thread for a swarm of n particles of d variables (0 if it does not fit).
uint32_t resident_paper_slots(uint32_t n, uint32_t d);
// Per function f1..f9, the most waves of particles per SIMD (n times lanes
// per particle over 256) for which AUTO picks the one-workgroup engine.
constexpr uint32_t kResidentPaperAutoWaves[9] = {16, 16, 14, 15, 11, 8, 10, 16, 9};
uint32_t round_up(uint32_t x, uint32_t m);
// ceil(c 2^32) for c in [0, 1] (exact: the product by 2^32 is exact).
uint64_t threshold(double c);
// SSO_OK or an error code with the reason in *why.
int validate(const sso_config *c, std::string *why);
// The same checks with the reason as a static string (no allocation).
int validate_msg(const sso_config *c, const char **why);
// Engine and row storage a valid configuration resolves to.
void resolve(const sso_config &c, int *engine, int *storage);
// The dense kernel's contraction (SSO_CONTRACT_F32, _BF16X3 or _F16X2) for a
// valid configuration; F32 for the other objectives.
int resolve_contraction(const sso_config &c);
int hip_fail(std::string *err, hipError_t e, const char *what);

// Integer thresholds of Eq. (2.1) in the configured order, the fresh-draw
// rescale, the box, the Philox key and swarm word, the kind and the order.
void set_params(const sso_config &c, SwarmDev &S);
// Copies s (and w for RIPPLE) zero-padded to S.dp floats; synchronous.
int upload_separable(const sso_config &c, const SwarmDev &S, hipStream_t st, std::string *err);

uint32_t orderable_host(float f);
float from_orderable(uint32_t o);

// The operations below act on one swarm whose generation count is t; the
// ones that read the device synchronise `st` first.
int current_result(const SwarmDev &S, uint64_t t, std::string *err, unsigned long long *key,
                   uint32_t *count);
int get_best(const SwarmDev &S, hipStream_t st, uint64_t t, std::string *err, float *g_out,
             float *f_out, uint32_t *idx_out);
int get_state(const SwarmDev &S, hipStream_t st, std::string *err, float *x, float *p, float *fp);
// Imports a state with generation count t: pBests into row 0, gBest = the
// lowest-index argmin of fp, trace ring restarted at t.
int set_state(const SwarmDev &S, hipStream_t st, uint64_t t, std::string *err, const float *x,
              const float *p, const float *fp);
int get_trace(const SwarmDev &S, hipStream_t st, uint64_t t_now, uint64_t trace_base,
              std::string *err, uint64_t first, uint32_t count, float *fg, uint32_t *gidx,
              uint32_t *improved);

}  // namespace host
}  // namespace sso
