// C ABI entry points: host-side validation, workspace accounting, kernel dispatch.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace vqmc;

namespace {
thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return VQMC_OK;
  return fail(VQMC_EHIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int kMaxSamplerH = 4096;  // units held per thread: 16 x 256
constexpr int kMaxEnergyCsrN = 160000;  // site bytes of the CSR energy kernel in one CU's LDS

size_t step_energy_offset(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  const size_t bw = logprob_ws_bytes(n, h, B, wdtype, true);
  const size_t sp = sample_plain_ws_bytes(n, h, B, wdtype);
  return (size_t)round_up((int64_t)std::max(bw, sp), 256);
}

// Step workspace: [sampling / backward region][energy region][Zs: B x ld(n) floats, the
// incremental sampler's s_d z_d, read by the backward][masked copy of P^T, h x ld(n)]
size_t step_zs_offset(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  return step_energy_offset(n, h, B, wdtype) +
         (size_t)round_up((int64_t)((n + 63) / 64) * B * (int64_t)sizeof(double), 256);
}

size_t step_pm_offset(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  return step_zs_offset(n, h, B, wdtype) + (size_t)round_up(B * round_up(n, kPad) * (int64_t)sizeof(float), 256);
}

// One auxiliary stream (default priority) and two events per device, created on first
// use and kept for the life of the process: vqmc_step without a band runs the energy and
// statistics on it while the main stream starts the recomputing backward.
struct StepAux {
  hipStream_t stream = nullptr;
  hipEvent_t sampled = nullptr, stats_done = nullptr;
};
std::mutex g_aux_mu;
StepAux g_aux[64];

hipError_t step_aux(StepAux** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  StepAux& a = g_aux[dev];
  if (!a.stream) {
    if ((e = hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.sampled, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.stats_done, hipEventDisableTiming)) != hipSuccess) return e;
  }
  *out = &a;
  return hipSuccess;
}

// SR direction workspace: [the Gram's or the backward's scratch, whichever is larger]
// [K: B x B floats][the solve's FP64 matrix and vectors][y: B floats]
struct SrDirLayout {
  size_t K, solve, y, total;
};
SrDirLayout sr_dir_layout(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  const size_t bws = (size_t)round_up((int64_t)logprob_ws_bytes(n, h, B, wdtype, true), 256) + mask_w2t_bytes(n, h);
  const size_t r0 = (size_t)round_up((int64_t)std::max(sr_gram_ws_bytes(n, h, B, wdtype), bws), 256);
  SrDirLayout L;
  L.K = r0;
  L.solve = L.K + (size_t)round_up(B * B * 4, 256);
  L.y = L.solve + (size_t)round_up((int64_t)sr_solve_ws_bytes(B), 256);
  L.total = L.y + (size_t)round_up(B * 4, 256);
  return L;
}

// Scratch of vqmc_logprob_noalloc: a fixed array in the library's device memory (one copy
// per GPU, which holds it until the process ends).  In host code the name `scratch` is only
// a host-side stand-in; its device address on each GPU comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is ever passed on.
static_assert(VQMC_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256 bytes");
static __device__ __align__(256) uint8_t scratch[VQMC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// TIM step workspace: [backward region (with the Rt slot)][masked copy of P^T][Zs: B x ld(n)
// floats][TIM local-energy workspace]
size_t tim_step_pm_offset(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  return (size_t)round_up((int64_t)logprob_ws_bytes(n, h, B, wdtype, true), 256);
}
size_t tim_step_zs_offset(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  return tim_step_pm_offset(n, h, B, wdtype) + (size_t)round_up((int64_t)mask_w2t_bytes(n, h), 256);
}
size_t tim_step_tim_offset(int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  return tim_step_zs_offset(n, h, B, wdtype) + (size_t)round_up(B * round_up(n, kPad) * (int64_t)sizeof(float), 256);
}

int check_made(const vqmc_made* m, bool need_pt) {
  if (!m) return fail(VQMC_EINVAL, "made is NULL");
  if (m->n < 2 || m->h < 1) return fail(VQMC_EINVAL, "need n >= 2 and h >= 1 (n=%d h=%d)", m->n, m->h);
  if (m->wdtype != VQMC_F32 && m->wdtype != VQMC_BF16)
    return fail(VQMC_EDTYPE, "weight dtype %d not supported (F32 or BF16)", m->wdtype);
  if (!m->P || !m->b1 || !m->b2 || !m->c) return fail(VQMC_EINVAL, "null parameter pointer");
  if (need_pt && !m->Pt) return fail(VQMC_EINVAL, "Pt is NULL");
  return VQMC_OK;
}
}  // namespace

extern "C" {

int64_t vqmc_ld(int64_t x) { return round_up(x, kPad); }

const char* vqmc_error_string(int status) {
  switch (status) {
    case VQMC_OK: return "ok";
    case VQMC_EINVAL: return "invalid argument";
    case VQMC_EDTYPE: return "unsupported dtype";
    case VQMC_EWORKSPACE: return "workspace too small";
    case VQMC_EHIP: return "HIP error";
    case VQMC_ENONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

const char* vqmc_last_error(void) { return g_err; }

size_t vqmc_workspace_bytes(int which, int32_t n, int32_t h, int64_t B, int32_t wdtype) {
  if (n < 2 || h < 1 || B < 1) return 0;
  switch (which) {
    case VQMC_WS_LOGPROB: return logprob_ws_bytes(n, h, B, wdtype, false);
    case VQMC_WS_BACKWARD: return logprob_ws_bytes(n, h, B, wdtype, true);
    case VQMC_WS_SAMPLE_PLAIN: return sample_plain_ws_bytes(n, h, B, wdtype);
    case VQMC_WS_STEP: return step_pm_offset(n, h, B, wdtype) + mask_w2t_bytes(n, h);
    case VQMC_WS_SR_GRAM: return sr_gram_ws_bytes(n, h, B, wdtype);
    case VQMC_WS_SR_JVP: return sr_jvp_ws_bytes(n, h, B, wdtype);
    case VQMC_WS_BACKWARD_SAMPLED:
      return (size_t)round_up((int64_t)logprob_ws_bytes(n, h, B, wdtype, true), 256) + mask_w2t_bytes(n, h);
    case VQMC_WS_SR_DIRECTION: return sr_dir_layout(n, h, B, wdtype).total;
    case VQMC_WS_TIM_ENERGY: return tim_ws_bytes(n, h, B, wdtype);
    case VQMC_WS_TIM_STEP: return tim_step_tim_offset(n, h, B, wdtype) + tim_ws_bytes(n, h, B, wdtype);
    default: return 0;
  }
}

int vqmc_pack(int32_t n, int32_t h, const float* W1, const float* W2, const int32_t* degrees,
              float* P32, int32_t* c, void* stream) {
  if (n < 2 || h < 1) return fail(VQMC_EINVAL, "need n >= 2 and h >= 1");
  if (!W1 || !W2 || !degrees || !P32 || !c) return fail(VQMC_EINVAL, "null pointer");
  for (int k = 0; k < h; ++k) {
    if (degrees[k] < 1 || degrees[k] > n - 1)
      return fail(VQMC_EINVAL, "degree[%d] = %d outside [1, n-1]", k, degrees[k]);
    if (k && degrees[k] < degrees[k - 1]) return fail(VQMC_EINVAL, "degrees not sorted at %d", k);
  }
  // c[d] = #{k : m(k) <= d} for 0-based site d (m is 1-based), counted on the device from
  // the degrees passed by value, so the call stays asynchronous
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_degree_counts(n, h, degrees, c, st);
  if (e != hipSuccess) return hip_status(e, "vqmc_pack degrees");
  return hip_status(launch_pack(n, h, W1, W2, c, P32, st), "vqmc_pack");
}

int vqmc_unpack(int32_t n, int32_t h, const float* P32, const int32_t* c, float* W1, float* W2,
                void* stream) {
  if (n < 2 || h < 1) return fail(VQMC_EINVAL, "need n >= 2 and h >= 1");
  if (!P32 || !c || !W1 || !W2) return fail(VQMC_EINVAL, "null pointer");
  return hip_status(launch_unpack(n, h, P32, c, W1, W2, (hipStream_t)stream), "vqmc_unpack");
}

int vqmc_cast(int32_t n, int32_t h, const float* P32, int32_t dtype, void* P, void* Pt, void* stream) {
  if (n < 2 || h < 1) return fail(VQMC_EINVAL, "need n >= 2 and h >= 1");
  if (dtype != VQMC_F32 && dtype != VQMC_BF16) return fail(VQMC_EDTYPE, "cast dtype %d", dtype);
  if (!P32 || !P || !Pt) return fail(VQMC_EINVAL, "null pointer");
  return hip_status(launch_cast(n, h, P32, dtype, P, Pt, (hipStream_t)stream), "vqmc_cast");
}

int vqmc_refresh(int32_t n, int32_t h, const float* P32, int32_t dtype, void* P, void* Pt, const float* b1,
                 const float* b2, const int32_t* c, float* band, int32_t* nonfinite, void* stream) {
  if (n < 2 || h < 1) return fail(VQMC_EINVAL, "need n >= 2 and h >= 1");
  if (dtype != VQMC_F32 && dtype != VQMC_BF16) return fail(VQMC_EDTYPE, "cast dtype %d", dtype);
  if (!P32 || !P || !Pt) return fail(VQMC_EINVAL, "null pointer");
  if (band && (!b1 || !b2 || !c)) return fail(VQMC_EINVAL, "band needs b1, b2 and c");
  if (nonfinite && (!b1 || !b2)) return fail(VQMC_EINVAL, "the non-finite check needs b1 and b2");
  if (band && ((uintptr_t)band & 15)) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_cast(n, h, P32, dtype, P, Pt, st, b2, c, band, b1, nonfinite);
  if (e != hipSuccess || !band) return hip_status(e, "vqmc_refresh");
  const vqmc_made m{n, h, dtype, P, Pt, b1, b2, c, band};
  return hip_status(launch_band(m, band, st, false), "vqmc_refresh");
}

int vqmc_check_nonfinite(int32_t flag) {
  if (flag) return fail(VQMC_ENONFINITE, "the parameters hold a NaN or an infinity (flag set by vqmc_refresh)");
  return VQMC_OK;
}

size_t vqmc_band_bytes(int32_t n, int32_t h, int32_t wdtype) {
  if (n < 2 || h < 1 || (wdtype != VQMC_F32 && wdtype != VQMC_BF16)) return 0;
  return sample_tables_bytes(n, h, wdtype);
}

int vqmc_band(const vqmc_made* m, float* band, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (!band) return fail(VQMC_EINVAL, "band is NULL");
  if ((uintptr_t)band & 15) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  return hip_status(launch_band(*m, band, (hipStream_t)stream), "vqmc_band");
}

int vqmc_sample(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset,
                uint32_t tag, int8_t* S, float* logp, void* stream) {
  int r = check_made(m, false);
  if (r) return r;
  if (B < 1) return fail(VQMC_EINVAL, "B must be >= 1");
  if (!S) return fail(VQMC_EINVAL, "S is NULL");
  if ((uintptr_t)S & 7) return fail(VQMC_EINVAL, "S must be 8-byte aligned");
  if (m->band && ((uintptr_t)m->band & 15)) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  if (sample_offset < 0) return fail(VQMC_EINVAL, "sample_offset < 0");
  if (m->h > kMaxSamplerH) return fail(VQMC_EINVAL, "h = %d exceeds the sampler limit %d", m->h, kMaxSamplerH);
  return hip_status(
      launch_sample_incremental(*m, B, seed, step, sample_offset, tag, S, logp, (hipStream_t)stream),
      "vqmc_sample");
}

int vqmc_sample_cycles(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int8_t* S, float* logp,
                       uint64_t* cycles, int32_t* waves, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || !S || !cycles || !waves) return fail(VQMC_EINVAL, "bad vqmc_sample_cycles arguments");
  if ((uintptr_t)S & 7) return fail(VQMC_EINVAL, "S must be 8-byte aligned");
  if (!m->band) return fail(VQMC_EINVAL, "vqmc_sample_cycles needs the band (vqmc_band)");
  if ((uintptr_t)m->band & 15) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  if (!sample_pipe_supported(m->n, m->h))
    return fail(VQMC_EINVAL, "h = %d too large for the pipelined sampler", m->h);
  *waves = sample_pipe_waves();
  return hip_status(launch_sample_pipe_cycles(*m, B, seed, step, S, logp, cycles, (hipStream_t)stream),
                    "vqmc_sample_cycles");
}

int vqmc_sample_fwd(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset,
                    uint32_t tag, int8_t* S, float* logp, float* Zs, void* Rt, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1) return fail(VQMC_EINVAL, "B must be >= 1");
  if (!S) return fail(VQMC_EINVAL, "S is NULL");
  if ((uintptr_t)S & 7) return fail(VQMC_EINVAL, "S must be 8-byte aligned");
  if (!m->band) return fail(VQMC_EINVAL, "vqmc_sample_fwd needs the band (vqmc_band)");
  if ((uintptr_t)m->band & 15) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  if ((Zs && ((uintptr_t)Zs & 15)) || (Rt && ((uintptr_t)Rt & 15)))
    return fail(VQMC_EINVAL, "Zs and Rt must be 16-byte aligned");
  if (sample_offset < 0) return fail(VQMC_EINVAL, "sample_offset < 0");
  if (!sample_pipe_supported(m->n, m->h))
    return fail(VQMC_EINVAL, "h = %d too large for the pipelined sampler", m->h);
  return hip_status(launch_sample_pipe(*m, B, seed, step, sample_offset, tag, S, logp, (hipStream_t)stream, Zs, Rt),
                    "vqmc_sample_fwd");
}

int vqmc_backward_sampled(const vqmc_made* m, const int8_t* S, int64_t B, const float* coef, const float* Zs,
                          const void* Rt, float* dP, float* db1, float* db2, void* ws, size_t ws_bytes,
                          void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || !S || !coef || !Zs || !Rt || !dP || !db1 || !db2 || !ws)
    return fail(VQMC_EINVAL, "bad backward arguments");
  const size_t need = vqmc_workspace_bytes(VQMC_WS_BACKWARD_SAMPLED, m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  void* Pm = (uint8_t*)ws + round_up((int64_t)logprob_ws_bytes(m->n, m->h, B, m->wdtype, true), 256);
  return hip_status(launch_backward_sampled(*m, S, B, coef, Zs, Rt, dP, db1, db2, ws, Pm, (hipStream_t)stream),
                    "vqmc_backward_sampled");
}

int vqmc_sample_plain(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset,
                      uint32_t tag, int8_t* S, float* logp, void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1) return fail(VQMC_EINVAL, "B must be >= 1");
  if (!S || !ws) return fail(VQMC_EINVAL, "null pointer");
  if (sample_offset < 0) return fail(VQMC_EINVAL, "sample_offset < 0");
  const size_t need = sample_plain_ws_bytes(m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_sample_plain(*m, B, seed, step, sample_offset, tag, S, logp, ws,
                                        (hipStream_t)stream),
                    "vqmc_sample_plain");
}

static int check_ham(const vqmc_hamiltonian* H) {
  if (!H) return fail(VQMC_EINVAL, "hamiltonian is NULL");
  if (H->n < 2) return fail(VQMC_EINVAL, "hamiltonian n < 2");
  if (H->kind == VQMC_H_DENSE_F32) {
    if (!H->J) return fail(VQMC_EINVAL, "dense J is NULL");
    return VQMC_OK;
  }
  if (H->kind != VQMC_H_CSR_INT && H->kind != VQMC_H_CSR_F32)
    return fail(VQMC_EINVAL, "unknown hamiltonian kind %d", H->kind);
  if (H->n > kMaxEnergyCsrN) return fail(VQMC_EINVAL, "CSR energy supports n <= %d", kMaxEnergyCsrN);
  if (!H->rowptr || (H->nnz > 0 && (!H->col || !H->w))) return fail(VQMC_EINVAL, "null CSR pointer");
  return VQMC_OK;
}

int vqmc_energy(const vqmc_hamiltonian* H, const int8_t* S, int64_t B, void* E, void* ws,
                size_t ws_bytes, void* stream) {
  int r = check_ham(H);
  if (r) return r;
  if (B < 1 || !S || !E) return fail(VQMC_EINVAL, "bad batch arguments");
  // the kernels read each spin row in 16-byte (CSR) or 8-byte (dense) pieces
  if ((uintptr_t)S & 15) return fail(VQMC_EINVAL, "S must be 16-byte aligned");
  const size_t need = energy_workspace_bytes(*H, B);
  if (ws_bytes < need || (need && !ws)) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_energy(*H, S, B, E, ws, (hipStream_t)stream), "vqmc_energy");
}

size_t vqmc_energy_workspace_bytes(const vqmc_hamiltonian* H, int64_t B) {
  if (!H || B < 1) return 0;
  return energy_workspace_bytes(*H, B);
}

int vqmc_batch_stats(const void* E, int32_t e_is_int, int64_t B, vqmc_stats* stats, float* coef,
                     void* stream) {
  if (!E || !stats || B < 1) return fail(VQMC_EINVAL, "bad stats arguments");
  return hip_status(launch_stats(E, e_is_int, B, stats, coef, (hipStream_t)stream), "vqmc_batch_stats");
}

int vqmc_logprob(const vqmc_made* m, const int8_t* S, int64_t B, float* logp, float* Z, void* ws,
                 size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || !S || !logp || !ws) return fail(VQMC_EINVAL, "bad logprob arguments");
  const size_t need = logprob_ws_bytes(m->n, m->h, B, m->wdtype, false);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_logprob(*m, S, B, logp, Z, ws, (hipStream_t)stream), "vqmc_logprob");
}

int vqmc_logprob_noalloc(const vqmc_made* m, const int8_t* S, int64_t B, float* logp, float* Z, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || !S || !logp) return fail(VQMC_EINVAL, "bad logprob arguments");
  // the size check comes before anything touches the device
  const size_t need = logprob_ws_bytes(m->n, m->h, B, m->wdtype, false);
  if (need > (size_t)VQMC_NOALLOC_SCRATCH_BYTES)
    return fail(VQMC_EWORKSPACE,
                "vqmc_logprob_noalloc: n=%d h=%d B=%lld needs %zu scratch bytes, more than its fixed %zu; "
                "use vqmc_logprob with a workspace",
                m->n, m->h, (long long)B, need, (size_t)VQMC_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  hipError_t e = noalloc_scratch(&ws);
  if (e != hipSuccess) return hip_status(e, "vqmc_logprob_noalloc scratch address");
  return hip_status(launch_logprob(*m, S, B, logp, Z, ws, (hipStream_t)stream), "vqmc_logprob_noalloc");
}

int vqmc_logprob_backward(const vqmc_made* m, const int8_t* S, int64_t B, const float* coef, float* dP,
                          float* db1, float* db2, void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || !S || !coef || !dP || !db1 || !db2 || !ws) return fail(VQMC_EINVAL, "bad backward arguments");
  const size_t need = logprob_ws_bytes(m->n, m->h, B, m->wdtype, true);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_backward(*m, S, B, coef, dP, db1, db2, ws, (hipStream_t)stream),
                    "vqmc_logprob_backward");
}

int vqmc_sr_gram(const vqmc_made* m, const int8_t* S, int64_t B, float* K, void* ws, size_t ws_bytes,
                 void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || B > 65536 || !S || !K || !ws) return fail(VQMC_EINVAL, "bad sr_gram arguments (1 <= B <= 65536)");
  const size_t need = sr_gram_ws_bytes(m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_sr_gram(*m, S, B, K, ws, (hipStream_t)stream), "vqmc_sr_gram");
}

int vqmc_sr_gram_sampled(const vqmc_made* m, const int8_t* S, int64_t B, const float* Zs, const void* Rt, float* K,
                         void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || B > 65536 || !S || !Zs || !Rt || !K || !ws)
    return fail(VQMC_EINVAL, "bad sr_gram_sampled arguments (1 <= B <= 65536)");
  if (((uintptr_t)Zs | (uintptr_t)Rt) & 15) return fail(VQMC_EINVAL, "Zs and Rt must be 16-byte aligned");
  const size_t need = sr_gram_ws_bytes(m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_sr_gram_sampled(*m, S, B, Zs, Rt, K, ws, (hipStream_t)stream), "vqmc_sr_gram_sampled");
}

int vqmc_sr_jvp(const vqmc_made* m, const int8_t* S, int64_t B, const float* gP, const float* gb1, const float* gb2,
                float* v, void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || !S || !gP || !gb1 || !gb2 || !v || !ws) return fail(VQMC_EINVAL, "bad sr_jvp arguments");
  const size_t need = sr_jvp_ws_bytes(m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_sr_jvp(*m, S, B, gP, gb1, gb2, v, ws, (hipStream_t)stream), "vqmc_sr_jvp");
}

size_t vqmc_sr_solve_workspace_bytes(int64_t B) { return B < 1 ? 0 : sr_solve_ws_bytes(B); }

int vqmc_sr_solve(int64_t B, const float* K, double shift, const float* rhs, double scale, float* y, void* ws,
                  size_t ws_bytes, void* stream) {
  if (B < 1 || B > 65536 || !K || !rhs || !y || !ws) return fail(VQMC_EINVAL, "bad sr_solve arguments (1 <= B <= 65536)");
  if (!(shift > 0.0) || !std::isfinite(shift)) return fail(VQMC_EINVAL, "shift must be finite and > 0 (got %g)", shift);
  if (!std::isfinite(scale)) return fail(VQMC_EINVAL, "scale must be finite");
  const size_t need = sr_solve_ws_bytes(B);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_sr_solve(K, B, shift, rhs, scale, y, ws, (hipStream_t)stream), "vqmc_sr_solve");
}

int vqmc_sr_direction(const vqmc_made* m, const int8_t* S, int64_t B, const float* coef, const float* Zs,
                      const void* Rt, double lambda, float* xP, float* xb1, float* xb2, float* K_out, void* ws,
                      size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if (B < 1 || B > 65536 || !S || !coef || !xP || !xb1 || !xb2 || !ws)
    return fail(VQMC_EINVAL, "bad sr_direction arguments (1 <= B <= 65536)");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(VQMC_EINVAL, "lambda must be finite and > 0");
  if ((Zs == nullptr) != (Rt == nullptr)) return fail(VQMC_EINVAL, "give both Zs and Rt, or neither");
  if (Zs && (((uintptr_t)Zs | (uintptr_t)Rt) & 15)) return fail(VQMC_EINVAL, "Zs and Rt must be 16-byte aligned");
  const SrDirLayout L = sr_dir_layout(m->n, m->h, B, m->wdtype);
  if (ws_bytes < L.total) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* w = (uint8_t*)ws;
  float* K = K_out ? K_out : (float*)(w + L.K);
  float* y = (float*)(w + L.y);
  hipError_t e = Zs ? launch_sr_gram_sampled(*m, S, B, Zs, Rt, K, ws, st) : launch_sr_gram(*m, S, B, K, ws, st);
  if (e != hipSuccess) return hip_status(e, "vqmc_sr_direction gram");
  // (K + lambda B I) y = B coef: the push-through form of (O^T O / B + lambda I) x = O^T coef
  if ((e = launch_sr_solve(K, B, lambda * (double)B, coef, (double)B, y, w + L.solve, st)) != hipSuccess)
    return hip_status(e, "vqmc_sr_direction solve");
  if (Zs) {
    void* Pm = w + round_up((int64_t)logprob_ws_bytes(m->n, m->h, B, m->wdtype, true), 256);
    e = launch_backward_sampled(*m, S, B, y, Zs, Rt, xP, xb1, xb2, ws, Pm, st);
  } else {
    e = launch_backward(*m, S, B, y, xP, xb1, xb2, ws, st);
  }
  return hip_status(e, "vqmc_sr_direction scores");
}

int vqmc_step(const vqmc_made* m, const vqmc_hamiltonian* H, int64_t B, uint64_t seed, uint64_t step,
              int64_t sample_offset, int32_t algo, int8_t* S, float* logp, void* E, vqmc_stats* stats,
              float* coef, float* dP, float* db1, float* db2, void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if ((r = check_ham(H))) return r;
  if (H->n != m->n) return fail(VQMC_EINVAL, "hamiltonian n=%d != model n=%d", H->n, m->n);
  if (B < 1 || !S || !E || !stats || !coef || !dP || !db1 || !db2 || !ws)
    return fail(VQMC_EINVAL, "bad step arguments");
  if (algo != 0 && algo != 1) return fail(VQMC_EINVAL, "algo must be 0 (incremental) or 1 (plain)");
  if (algo == 0 && m->h > kMaxSamplerH) return fail(VQMC_EINVAL, "h exceeds the sampler limit");
  if ((uintptr_t)S & 7) return fail(VQMC_EINVAL, "S must be 8-byte aligned");
  if (m->band && ((uintptr_t)m->band & 15)) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  const size_t need = vqmc_workspace_bytes(VQMC_WS_STEP, m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  // with the pipelined sampler the forward quantities of the backward (relu(A) and the
  // logits) come out of the sampling itself
  const bool fused = algo == 0 && m->Pt && m->band && sample_pipe_supported(m->n, m->h);
  float* Zs = (float*)((uint8_t*)ws + step_zs_offset(m->n, m->h, B, m->wdtype));
  hipError_t e = fused ? launch_sample_pipe(*m, B, seed, step, sample_offset, 0, S, logp, st, Zs,
                                            backward_rt_slot(*m, B, ws))
                 : (algo == 0) ? launch_sample_incremental(*m, B, seed, step, sample_offset, 0, S, logp, st)
                               : launch_sample_plain(*m, B, seed, step, sample_offset, 0, S, logp, ws, st);
  if (e != hipSuccess) return hip_status(e, "vqmc_step sample");
  void* ws_energy = (uint8_t*)ws + step_energy_offset(m->n, m->h, B, m->wdtype);
  if (fused) {
    // every backward product needs coef, so energy and statistics stay on the stream: a hop
    // to another stream and back would only add two synchronisations
    if ((e = launch_energy(*H, S, B, E, ws_energy, st)) != hipSuccess) return hip_status(e, "vqmc_step energy");
    if ((e = launch_stats(E, H->kind == VQMC_H_CSR_INT, B, stats, coef, st)) != hipSuccess)
      return hip_status(e, "vqmc_step stats");
    void* Pm = (uint8_t*)ws + step_pm_offset(m->n, m->h, B, m->wdtype);
    if ((e = launch_backward_sampled(*m, S, B, coef, Zs, backward_rt_slot(*m, B, ws), dP, db1, db2, ws, Pm, st)) !=
        hipSuccess)
      return hip_status(e, "vqmc_step backward");
    return VQMC_OK;
  }
  // energy + statistics on the auxiliary stream, overlapping the first backward product
  // (which only needs the spins); the main stream waits for them before reading coef
  StepAux* aux = nullptr;
  if ((e = step_aux(&aux)) != hipSuccess) return hip_status(e, "vqmc_step aux stream");
  if ((e = hipEventRecord(aux->sampled, st)) != hipSuccess) return hip_status(e, "vqmc_step record");
  if ((e = hipStreamWaitEvent(aux->stream, aux->sampled, 0)) != hipSuccess) return hip_status(e, "vqmc_step wait");
  if ((e = launch_energy(*H, S, B, E, ws_energy, aux->stream)) != hipSuccess) return hip_status(e, "vqmc_step energy");
  if ((e = launch_stats(E, H->kind == VQMC_H_CSR_INT, B, stats, coef, aux->stream)) != hipSuccess)
    return hip_status(e, "vqmc_step stats");
  if ((e = hipEventRecord(aux->stats_done, aux->stream)) != hipSuccess) return hip_status(e, "vqmc_step record");
  if ((e = launch_backward(*m, S, B, coef, dP, db1, db2, ws, st, aux->stats_done)) != hipSuccess)
    return hip_status(e, "vqmc_step backward");
  return VQMC_OK;
}

static int check_tim(const vqmc_made* m, const vqmc_tim* H) {
  if (!H) return fail(VQMC_EINVAL, "tim hamiltonian is NULL");
  if (H->n != m->n) return fail(VQMC_EINVAL, "tim hamiltonian n=%d != model n=%d", H->n, m->n);
  if (!H->alpha || !H->beta || !H->J) return fail(VQMC_EINVAL, "null tim coupling pointer");
  if (!tim_supported(m->n, m->h, m->wdtype))
    return fail(VQMC_EINVAL, "h = %d too large for the TIM local energy (BF16: h <= 1024, F32: h <= 512)", m->h);
  return VQMC_OK;
}

int vqmc_tim_energy(const vqmc_made* m, const vqmc_tim* H, const int8_t* S, int64_t B, double* E, float* D,
                    void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if ((r = check_tim(m, H))) return r;
  if (B < 1 || !S || !E || !ws) return fail(VQMC_EINVAL, "bad tim energy arguments");
  if ((uintptr_t)S & 15) return fail(VQMC_EINVAL, "S must be 16-byte aligned");
  const size_t need = tim_ws_bytes(m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return hip_status(launch_tim_energy(*m, *H, S, B, E, D, ws, (hipStream_t)stream), "vqmc_tim_energy");
}

int vqmc_tim_step(const vqmc_made* m, const vqmc_tim* H, int64_t B, uint64_t seed, uint64_t step,
                  int64_t sample_offset, int8_t* S, float* logp, double* E, vqmc_stats* stats, float* coef,
                  float* dP, float* db1, float* db2, void* ws, size_t ws_bytes, void* stream) {
  int r = check_made(m, true);
  if (r) return r;
  if ((r = check_tim(m, H))) return r;
  if (B < 1 || !S || !E || !stats || !coef || !dP || !db1 || !db2 || !ws)
    return fail(VQMC_EINVAL, "bad tim step arguments");
  if ((uintptr_t)S & 15) return fail(VQMC_EINVAL, "S must be 16-byte aligned");
  if (sample_offset < 0) return fail(VQMC_EINVAL, "sample_offset < 0");
  if (!m->band) return fail(VQMC_EINVAL, "vqmc_tim_step needs the band (vqmc_band)");
  if ((uintptr_t)m->band & 15) return fail(VQMC_EINVAL, "band must be 16-byte aligned");
  if (!sample_pipe_supported(m->n, m->h)) return fail(VQMC_EINVAL, "h = %d too large for the pipelined sampler", m->h);
  const size_t need = vqmc_workspace_bytes(VQMC_WS_TIM_STEP, m->n, m->h, B, m->wdtype);
  if (ws_bytes < need) return fail(VQMC_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* w = (uint8_t*)ws;
  float* Zs = (float*)(w + tim_step_zs_offset(m->n, m->h, B, m->wdtype));
  void* Rt = backward_rt_slot(*m, B, ws);
  hipError_t e = launch_sample_pipe(*m, B, seed, step, sample_offset, 0, S, logp, st, Zs, Rt);
  if (e != hipSuccess) return hip_status(e, "vqmc_tim_step sample");
  if ((e = launch_tim_energy(*m, *H, S, B, E, nullptr, w + tim_step_tim_offset(m->n, m->h, B, m->wdtype), st)) !=
      hipSuccess)
    return hip_status(e, "vqmc_tim_step energy");
  if ((e = launch_stats(E, 0, B, stats, coef, st)) != hipSuccess) return hip_status(e, "vqmc_tim_step stats");
  void* Pm = w + tim_step_pm_offset(m->n, m->h, B, m->wdtype);
  if ((e = launch_backward_sampled(*m, S, B, coef, Zs, Rt, dP, db1, db2, ws, Pm, st)) != hipSuccess)
    return hip_status(e, "vqmc_tim_step backward");
  return VQMC_OK;
}

int vqmc_uniforms(int32_t n, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset, uint32_t tag,
                  float* u, void* stream) {
  if (n < 1 || B < 1 || !u || sample_offset < 0) return fail(VQMC_EINVAL, "bad uniforms arguments");
  return hip_status(launch_uniforms(n, B, seed, step, sample_offset, tag, u, (hipStream_t)stream),
                    "vqmc_uniforms");
}

int vqmc_csr_from_edges(int32_t n, int64_t m, const int32_t* edges, const void* w, int32_t wkind,
                        int64_t* rowptr, int32_t* col, void* w_out) {
  if (n < 2 || m < 0) return fail(VQMC_EINVAL, "bad sizes");
  if (wkind != VQMC_H_CSR_INT && wkind != VQMC_H_CSR_F32) return fail(VQMC_EINVAL, "bad weight kind");
  if (m > 0 && (!edges || !w || !col || !w_out)) return fail(VQMC_EINVAL, "null pointer");
  if (!rowptr) return fail(VQMC_EINVAL, "rowptr is NULL");
  struct E3 { int32_t i, j; int64_t idx; };
  std::vector<E3> es((size_t)m);
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = edges[2 * e], b = edges[2 * e + 1];
    if (a < 0 || b < 0 || a >= n || b >= n) return fail(VQMC_EINVAL, "edge %lld out of range", (long long)e);
    if (a == b) return fail(VQMC_EINVAL, "self loop at edge %lld", (long long)e);
    if (a > b) std::swap(a, b);
    es[(size_t)e] = {a, b, e};
  }
  std::sort(es.begin(), es.end(), [](const E3& x, const E3& y) { return x.i != y.i ? x.i < y.i : x.j < y.j; });
  for (size_t e = 1; e < es.size(); ++e)
    if (es[e].i == es[e - 1].i && es[e].j == es[e - 1].j) return fail(VQMC_EINVAL, "duplicate edge");
  for (int i = 0; i <= n; ++i) rowptr[i] = 0;
  for (const E3& x : es) rowptr[x.i + 1]++;
  for (int i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
  for (size_t e = 0; e < es.size(); ++e) {
    col[e] = es[e].j;
    if (wkind == VQMC_H_CSR_INT) ((int32_t*)w_out)[e] = ((const int32_t*)w)[es[e].idx];
    else ((float*)w_out)[e] = ((const float*)w)[es[e].idx];
  }
  return VQMC_OK;
}

}  // extern "C"
