// Internal launchers (host functions) shared by the C ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vqmc.h"

namespace vqmc {

// pack.hip
// degrees travel to the device as kernel arguments, kDegreeChunk per launch
constexpr int kDegreeChunk = 960;
struct DegreeChunk {
  int32_t count;
  int32_t deg[kDegreeChunk];
};
hipError_t launch_degree_counts(int n, int h, const int32_t* degrees, int32_t* c, hipStream_t st);
hipError_t launch_pack(int n, int h, const float* W1, const float* W2, const int32_t* c, float* P32,
                       hipStream_t st);
hipError_t launch_unpack(int n, int h, const float* P32, const int32_t* c, float* W1, float* W2,
                         hipStream_t st);
// nonfinite (nullable): set to 1 if any of P32, b1, b2 is a NaN or an infinity (never cleared)
hipError_t launch_cast(int n, int h, const float* P32, int dtype, void* P, void* Pt, hipStream_t st,
                       const float* b2 = nullptr, const int32_t* c = nullptr, void* tables = nullptr,
                       const float* b1 = nullptr, int32_t* nonfinite = nullptr);

// energy.hip
hipError_t launch_energy(const vqmc_hamiltonian& H, const int8_t* S, int64_t B, void* E,
                         void* ws, hipStream_t st);
size_t energy_workspace_bytes(const vqmc_hamiltonian& H, int64_t B);
hipError_t launch_stats(const void* E, int e_is_int, int64_t B, vqmc_stats* stats, float* coef,
                        hipStream_t st);

// sample.hip
hipError_t launch_sample_incremental(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                                     int64_t offset, uint32_t tag, int8_t* S, float* logp,
                                     hipStream_t st);
bool sample_blocked_supported(int n, int h);
hipError_t launch_sample_blocked(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                                 uint32_t tag, int8_t* S, float* logp, hipStream_t st);
bool sample_pipe_supported(int n, int h);
size_t sample_tables_bytes(int n, int h, int wdtype);
// Zs (nullable): B x ld(n) floats s_d z_d; Rt (nullable): h x ld(B) relu(A) in the weight dtype
hipError_t launch_sample_pipe(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                              uint32_t tag, int8_t* S, float* logp, hipStream_t st, float* Zs = nullptr,
                              void* Rt = nullptr);
// the same sampler counting each wave's cycles between its per-block barriers (vqmc_sample_cycles)
int sample_pipe_waves();
hipError_t launch_sample_pipe_cycles(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int8_t* S,
                                     float* logp, uint64_t* cycles, hipStream_t st);
hipError_t launch_band(const vqmc_made& m, float* band, hipStream_t st, bool tiles = true);
void sample_tables_layout(int n, int h, int wdtype, int64_t* z, int64_t* u, int64_t* pm, int* nzt, int* nut);
hipError_t launch_mask_w2t(const vqmc_made& m, uint16_t* Pm, hipStream_t st);
hipError_t launch_uniforms(int n, int64_t B, uint64_t seed, uint64_t step, int64_t offset, uint32_t tag,
                           float* u, hipStream_t st);

// gemm.hip : masked forward / backward on MFMA
struct FwdWorkspace;
size_t logprob_ws_bytes(int n, int h, int64_t B, int dtype, bool backward);
hipError_t launch_logprob(const vqmc_made& m, const int8_t* S, int64_t B, float* logp, float* Z,
                          void* ws, hipStream_t st);
// coef_ready (nullable): event the output-layer product waits for before reading coef
hipError_t launch_backward(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                           float* dP, float* db1, float* db2, void* ws, hipStream_t st,
                           hipEvent_t coef_ready = nullptr);
// backward from the incremental sampler's Rt (written into the slot backward_rt_slot gives)
// and Zs (s_d z_d, B x ld(n)); ws as for launch_backward
void* backward_rt_slot(const vqmc_made& m, int64_t B, void* ws);
hipError_t launch_backward_sampled(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                                   const float* Zs, const void* Rt, float* dP, float* db1, float* db2, void* ws,
                                   void* Pm, hipStream_t st);
// SR Gram (sr.hip): the factor rows come from the backward engine with coef = 1
size_t sr_gram_ws_bytes(int n, int h, int64_t B, int dtype);
hipError_t launch_sr_gram(const vqmc_made& m, const int8_t* S, int64_t B, float* K, void* ws, hipStream_t st);
size_t sr_jvp_ws_bytes(int n, int h, int64_t B, int dtype);
hipError_t launch_sr_jvp(const vqmc_made& m, const int8_t* S, int64_t B, const float* gP, const float* gb1,
                         const float* gb2, float* v, void* ws, hipStream_t st);
hipError_t launch_sr_gram_sampled(const vqmc_made& m, const int8_t* S, int64_t B, const float* Zs, const void* Rt,
                                  float* K, void* ws, hipStream_t st);
// scratch of the sweeps: FP32, the items' partial sums + prefix lengths; BF16, the segment table and
// the segment-padded copies of G and S
size_t sr_gram_parts_bytes(int n, int h, int64_t B, int dtype);
// G (B x ld(n), the weight dtype) and S (B x ld(n) int8): row-major factors the BF16 form reads
hipError_t launch_sr_gram_sweeps(int dtype, const void* Gt, const void* Rt, const void* Dt, const void* St,
                                 int64_t ldb, const int32_t* c, int n, int h, int64_t B, float* parts, float* K,
                                 hipStream_t st, const void* G, const int8_t* S, int64_t ldn);
// chol.hip: (K + shift I) y = scale * rhs in FP64 (blocked Cholesky, forward and back substitution)
size_t sr_solve_ws_bytes(int64_t B);
hipError_t launch_sr_solve(const float* K, int64_t B, double shift, const float* rhs, double scale, float* y,
                           void* ws, hipStream_t st);
// gemm2.hip: BF16 backward products on the direct-to-LDS engine; Pm: h x ld(n) bf16 scratch
size_t mask_w2t_bytes(int n, int h);
// the hidden adjoint alone: Dt = [Rt > 0] (G Pm^T)^T, db1 partials per 64-sample tile (ld(h) each)
hipError_t launch_bwd_hidden2(const vqmc_made& m, int64_t B, const uint16_t* G, const uint16_t* Pm,
                              const uint16_t* Rt, uint16_t* Dt, float* db1_part, hipStream_t st);
// db1_part (np1 rows of ld(h)) and db2_part (np2 rows of ld(n)) are summed into db1 and db2
hipError_t launch_backward_products2(const vqmc_made& m, int64_t B, const uint16_t* G, const uint16_t* Gt,
                                     const uint16_t* St, const uint16_t* Rt, uint16_t* Dt, uint16_t* Pm,
                                     float* db1_part, int np1, const float* db2_part, int np2, float* dP, float* db1,
                                     float* db2, hipStream_t st, bool pm_ready);
// TIM local energy (tim.hip): forward quantities (gemm.hip), then the single-flip differences
hipError_t launch_tim_forward(const vqmc_made& m, const int8_t* S, int64_t B, float* Z, float* A, void* ws,
                              hipStream_t st);
bool tim_supported(int n, int h, int wdtype);
size_t tim_ws_bytes(int n, int h, int64_t B, int dtype);
// E: B doubles; D (nullable): B x ld(n) floats, log pi(s^(i)) - log pi(s)
hipError_t launch_tim_energy(const vqmc_made& m, const vqmc_tim& H, const int8_t* S, int64_t B, double* E, float* D,
                             void* ws, hipStream_t st);
size_t sample_plain_ws_bytes(int n, int h, int64_t B, int dtype);
hipError_t launch_sample_plain(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                               int64_t offset, uint32_t tag, int8_t* S, float* logp, void* ws,
                               hipStream_t st);

}  // namespace vqmc
