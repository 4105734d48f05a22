// Incremental autoregressive sampler (Algorithm 1 of the paper, "Autoregressive
// Sampling": for each site compute p(x_i | x_<i), draw x_i, write it into the state).
//
// Instead of a full forward pass per site, each sample keeps its h hidden
// pre-activations a_k = b1_k + sum_{d' received so far} W1[k][d'] s_d' in registers.
// With the packed layout P[d][k] (k < c[d]: W2[d][k]; k >= c[d]: W1[k][d]) site d is
//   z_d = b2_d + sum_{k < c[d]} P[d][k] relu(a_k)      (units k < c[d] are complete)
//   s_d = +1 iff u[b][d] < sigma(z_d),  logp += log sigma(s_d z_d)
//   a_k += s_d P[d][k]   for k >= c[d]                 (units that receive site d)
// which reproduces the conditionals of the n masked forward passes exactly (in exact
// arithmetic) at O(nh) work per sample instead of O(n^2 h).
//
// Mapping: one workgroup (4 waves) per tile of MS samples; thread t owns units
// k = t + 256 j.  Per site: one coalesced row load of P (prefetched one site ahead),
// per-thread partial dot products, a DPP wave reduction, one workgroup barrier, and
// the per-sample scalar work in lanes 0..MS-1 of every wave.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

template <typename WT, int MS, int J>
__global__ __launch_bounds__(256) void sample_incremental_kernel(
    const WT* __restrict__ P, int64_t ldh, const float* __restrict__ b1, const float* __restrict__ b2,
    const int32_t* __restrict__ c, int n, int h, int64_t B, uint64_t seed, uint64_t step,
    int64_t offset, uint32_t tag, int8_t* __restrict__ S, int64_t lds, float* __restrict__ logp) {
  __shared__ float red[2][MS][4];
  __shared__ float uu[64][MS];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * MS;

  float a[MS][J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = t + 256 * j;
    const float bv = (k < h) ? b1[k] : 0.f;
#pragma unroll
    for (int s = 0; s < MS; ++s) a[s][j] = bv;
  }
  float pw[J], pn[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = t + 256 * j;
    pn[j] = (k < h) ? to_f32(P[k]) : 0.f;
  }
  int cn = c[0];
  float bn = b2[0];
  float lp = 0.f;
  uint32_t word = 0;
  const int my_s = lane < MS ? lane : 0;
  const bool writer = (wv == 0) && (lane < MS) && (b0 + lane < B);

  for (int d = 0; d < n; ++d) {
    if ((d & 63) == 0) {
      __syncthreads();
      if (t < 16 * MS) {
        const int s = t >> 4, blk = t & 15;
        const float4 u4 =
            site_uniforms(seed, step, tag, (uint64_t)(b0 + s + offset), (uint32_t)((d >> 2) + blk));
        uu[blk * 4 + 0][s] = u4.x;
        uu[blk * 4 + 1][s] = u4.y;
        uu[blk * 4 + 2][s] = u4.z;
        uu[blk * 4 + 3][s] = u4.w;
      }
      __syncthreads();
    }
    const int cd = cn;
    const float b2d = bn;
#pragma unroll
    for (int j = 0; j < J; ++j) pw[j] = pn[j];
    if (d + 1 < n) {  // prefetch the next row
      const WT* row = P + (int64_t)(d + 1) * ldh;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int k = t + 256 * j;
        pn[j] = (k < h) ? to_f32(row[k]) : 0.f;
      }
      cn = c[d + 1];
      bn = b2[d + 1];
    }
    // partial logits over complete units k < c[d]
    float part[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) part[s] = 0.f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int k = t + 256 * j;
      const float wgt = (k < cd) ? pw[j] : 0.f;
#pragma unroll
      for (int s = 0; s < MS; ++s) part[s] = fmaf(wgt, fmaxf(a[s][j], 0.f), part[s]);
    }
#pragma unroll
    for (int s = 0; s < MS; ++s) part[s] = wave_sum(part[s]);
    const int buf = d & 1;
    if (lane == 0) {
#pragma unroll
      for (int s = 0; s < MS; ++s) red[buf][s][wv] = part[s];
    }
    __syncthreads();
    // per-sample scalar work: lane s < MS handles sample s (every wave redundantly)
    const float4 r = *(const float4*)&red[buf][my_s][0];
    const float z = b2d + ((r.x + r.y) + (r.z + r.w));
    const float u = uu[d & 63][my_s];
    const float sg = (u < sigmoid(z)) ? 1.f : -1.f;
    lp += log_sigmoid(sg * z);
    float sgn[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) sgn[s] = readlane_f(sg, s);
    // rank-1 update of the units that receive site d
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int k = t + 256 * j;
      const float wgt = (k >= cd) ? pw[j] : 0.f;
#pragma unroll
      for (int s = 0; s < MS; ++s) a[s][j] = fmaf(sgn[s], wgt, a[s][j]);
    }
    // spins: four sites per 32-bit store
    word |= ((uint32_t)(uint8_t)(int8_t)(int)sg) << (8 * (d & 3));
    if ((d & 3) == 3 || d == n - 1) {
      if (writer) *(uint32_t*)(S + (b0 + lane) * lds + (d & ~3)) = word;
      word = 0;
    }
  }
  if (writer) {
    for (int64_t col = round_up(n, 4); col < lds; col += 4) *(uint32_t*)(S + (b0 + lane) * lds + col) = 0u;
    if (logp) logp[b0 + lane] = lp;
  }
}

template <typename WT, int J>
static hipError_t launch_j(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                           uint32_t tag, int8_t* S, float* logp, hipStream_t st) {
  constexpr int MS = 8;
  const unsigned grid = (unsigned)((B + MS - 1) / MS);
  sample_incremental_kernel<WT, MS, J><<<grid, 256, 0, st>>>(
      (const WT*)m.P, round_up(m.h, kPad), m.b1, m.b2, m.c, m.n, m.h, B, seed, step, offset, tag, S,
      round_up(m.n, kPad), logp);
  return hipGetLastError();
}

template <typename WT>
static hipError_t launch_w(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                           uint32_t tag, int8_t* S, float* logp, hipStream_t st) {
  const int J = (m.h + 255) / 256;
  if (J <= 1) return launch_j<WT, 1>(m, B, seed, step, offset, tag, S, logp, st);
  if (J <= 2) return launch_j<WT, 2>(m, B, seed, step, offset, tag, S, logp, st);
  if (J <= 4) return launch_j<WT, 4>(m, B, seed, step, offset, tag, S, logp, st);
  if (J <= 8) return launch_j<WT, 8>(m, B, seed, step, offset, tag, S, logp, st);
  return launch_j<WT, 16>(m, B, seed, step, offset, tag, S, logp, st);
}

__global__ void uniforms_kernel(int n, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                                uint32_t tag, float* __restrict__ u) {
  const int nb = (n + 3) / 4;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * nb) return;
  const int64_t b = i / nb;
  const int blk = (int)(i % nb);
  const float4 v = site_uniforms(seed, step, tag, (uint64_t)(b + offset), (uint32_t)blk);
  const float vals[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int d = 4 * blk + e;
    if (d < n) u[b * n + d] = vals[e];
  }
}

hipError_t launch_uniforms(int n, int64_t B, uint64_t seed, uint64_t step, int64_t offset, uint32_t tag,
                           float* u, hipStream_t st) {
  const int64_t total = B * ((n + 3) / 4);
  uniforms_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(n, B, seed, step, offset, tag, u);
  return hipGetLastError();
}

hipError_t launch_sample_incremental(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                                     int64_t offset, uint32_t tag, int8_t* S, float* logp,
                                     hipStream_t st) {
  // the blocked MFMA sampler keeps 16 samples' state in LDS; beyond its LDS budget the
  // register-resident kernel above takes over
  if (m.Pt && m.band && sample_pipe_supported(m.n, m.h))
    return launch_sample_pipe(m, B, seed, step, offset, tag, S, logp, st);
  if (m.Pt && sample_blocked_supported(m.n, m.h))
    return launch_sample_blocked(m, B, seed, step, offset, tag, S, logp, st);
  if (m.wdtype == VQMC_BF16) return launch_w<bf16_t>(m, B, seed, step, offset, tag, S, logp, st);
  return launch_w<float>(m, B, seed, step, offset, tag, S, logp, st);
}

}  // namespace vqmc
