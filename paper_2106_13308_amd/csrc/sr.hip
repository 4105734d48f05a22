// Sample-space Gram of the per-sample scores, the B x B matrix that stochastic
// reconfiguration solves with (Sec. 2.1: Fisher information as the expectation of the
// outer product of grad log pi; Sec. 5.1: SR with a ridge; in sample space through the
// Woodbury identity):
//
//   K[b][b'] = <grad log pi(s_b), grad log pi(s_b')>    over every unmasked parameter.
//
// Per sample, with G = s sigma(-s z) (dlogp/dz), R = relu(A), D = dlogp/dA:
//   d/dP[d][k] = G_d R_k  (k < c[d], the W2 part)     d/db2_d = G_d
//   d/dP[d][k] = s_d D_k  (k >= c[d], the W1 part)    d/db1_k = D_k
// so, for a pair (b, b') and products xx'_j = x_b[j] x_b'[j],
//   K = sum_d GG'_d (1 + sum_{k < c[d]} RR'_k) + sum_k DD'_k (1 + sum_{d : c[d] <= k} ss'_d).
// Both sums are staircase prefix sums: one sweep over d (the RR' prefix advances to c[d])
// and one over k (the ss' prefix advances over the sites with c[d] <= k), 3 (n + h)
// multiply-adds per Gram entry, without forming the B x (nh + n + h) score matrix.
//
// This is elementwise FP32 work, not a contraction: every Gram entry carries its own
// running prefix.  Each workgroup owns a 64 x 64 tile of one of the two sums (tiles on or
// above the diagonal only; K is symmetric), each thread a 4 x 4 block; the factor rows are
// batch-contiguous (X[j][b], ld(B) columns), so a row of one factor feeds a tile with
// two 4-element loads per thread.  A combine pass adds the two sums and mirrors the
// upper tiles.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int GR_T = 64;  // Gram tile edge (samples)

template <typename T>
__device__ inline void load4(const T* p, float v[4]);
template <>
__device__ inline void load4<float>(const float* p, float v[4]) {
  const float4 x = *reinterpret_cast<const float4*>(p);
  v[0] = x.x;
  v[1] = x.y;
  v[2] = x.z;
  v[3] = x.w;
}
template <>
__device__ inline void load4<bf16_t>(const bf16_t* p, float v[4]) {
  const uint2 x = *reinterpret_cast<const uint2*>(p);
  v[0] = __uint_as_float(x.x << 16);
  v[1] = __uint_as_float(x.x & 0xFFFF0000u);
  v[2] = __uint_as_float(x.y << 16);
  v[3] = __uint_as_float(x.y & 0xFFFF0000u);
}

// blockIdx.x -> (row tile ti, column tile tj >= ti) of the upper triangle of an nt x nt grid
__device__ inline void upper_tile(int t, int nt, int& ti, int& tj) {
  int i = 0, rowlen = nt;
  while (t >= rowlen) {
    t -= rowlen;
    ++i;
    --rowlen;
  }
  ti = i;
  tj = i + t;
}

// part == 0: sum_d GG'_d (1 + prefix_{k < c[d]} RR'_k)            -> out0
// part == 1: sum_k DD'_k (1 + prefix_{d : c[d] <= k} ss'_d)        -> out1
// X1 (outer rows: G or D), X2 (prefix rows: R or S), both batch-contiguous with ldb columns.
template <typename T>
__global__ __launch_bounds__(256) void sr_gram_kernel(const T* __restrict__ Gt, const T* __restrict__ Rt,
                                                      const T* __restrict__ Dt, const T* __restrict__ St,
                                                      int64_t ldb, const int32_t* __restrict__ c, int n, int h,
                                                      int64_t B, int nt, float* __restrict__ out0,
                                                      float* __restrict__ out1) {
  int ti, tj;
  upper_tile(blockIdx.x, nt, ti, tj);
  const int part = blockIdx.y;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t br = (int64_t)ti * GR_T + 4 * ty;  // this thread's rows b
  const int64_t bc = (int64_t)tj * GR_T + 4 * tx;  // and columns b'
  float acc[4][4], pre[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = pre[i][j] = 0.f;
  float a[4], b[4];
  auto rank1 = [&](const T* X, int64_t row, float M[4][4]) {
    load4<T>(X + row * ldb + br, a);
    load4<T>(X + row * ldb + bc, b);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) M[i][j] = fmaf(a[i], b[j], M[i][j]);
  };
  auto outer = [&](const T* X, int64_t row) {
    load4<T>(X + row * ldb + br, a);
    load4<T>(X + row * ldb + bc, b);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const float t = a[i] * b[j];
        acc[i][j] = fmaf(t, pre[i][j], acc[i][j] + t);
      }
  };
  if (part == 0) {
    int kp = 0;
    for (int d = 0; d < n; ++d) {
      const int cd = c[d];
      for (; kp < cd; ++kp) rank1(Rt, kp, pre);
      outer(Gt, d);
    }
  } else {
    int dq = 0;
    for (int k = 0; k < h; ++k) {
      for (; dq < n && c[dq] <= k; ++dq) rank1(St, dq, pre);
      outer(Dt, k);
    }
  }
  float* out = part ? out1 : out0;
  for (int i = 0; i < 4; ++i) {
    const int64_t r = br + i;
    if (r >= B) break;
    for (int j = 0; j < 4; ++j)
      if (bc + j < B) out[r * B + bc + j] = acc[i][j];
  }
}

// K[b][b'] = P0[lo][hi] + P1[lo][hi] with (lo, hi) the pair ordered so that its tile lies on
// or above the diagonal (where the sweeps wrote it).
__global__ void sr_gram_combine_kernel(const float* __restrict__ P0, const float* __restrict__ P1, int64_t B,
                                       float* __restrict__ K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * B) return;
  const int64_t r = idx / B, q = idx - r * B;
  const bool upper = (r / GR_T) <= (q / GR_T);
  const int64_t src = upper ? idx : q * B + r;
  K[idx] = P0[src] + P1[src];
}

hipError_t launch_sr_gram_sweeps(int dtype, const void* Gt, const void* Rt, const void* Dt, const void* St,
                                 int64_t ldb, const int32_t* c, int n, int h, int64_t B, float* P0, float* P1,
                                 float* K, hipStream_t st) {
  const int nt = (int)((B + GR_T - 1) / GR_T);
  const int64_t pairs = (int64_t)nt * (nt + 1) / 2;
  if (pairs > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)pairs, 2);
  if (dtype == VQMC_BF16)
    sr_gram_kernel<bf16_t><<<grid, 256, 0, st>>>((const bf16_t*)Gt, (const bf16_t*)Rt, (const bf16_t*)Dt,
                                                 (const bf16_t*)St, ldb, c, n, h, B, nt, P0, P1);
  else
    sr_gram_kernel<float><<<grid, 256, 0, st>>>((const float*)Gt, (const float*)Rt, (const float*)Dt,
                                                (const float*)St, ldb, c, n, h, B, nt, P0, P1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = B * B;
  sr_gram_combine_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(P0, P1, B, K);
  return hipGetLastError();
}

}  // namespace vqmc
