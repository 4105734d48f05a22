// Masked MADE forward / backward on MFMA (gfx950), and the plain n-pass sampler.
//
// Forward (Sec. 5.1: MaskedFC1 -> ReLU -> MaskedFC2 -> Sigmoid; Sec. 2.3 MADE layer):
//   A[b][k] = b1[k] + sum_{d : c[d] <= k} S[b][d] P[d][k]         (first masked layer)
//   R = relu(A)
//   Z[b][d] = b2[d] + sum_{k < c[d]} R[b][k] P[d][k]              (second masked layer)
//   logp[b] = sum_d log sigma(S[b][d] Z[b][d])                  (autoregressive product)
// Backward of F = sum_b coef_b logp_b (the surrogate of the Sec. 2.1 score gradient):
//   G[b][d]  = coef_b S[b][d] sigma(-S[b][d] Z[b][d])            (dF/dZ)
//   D[b][k]  = [A[b][k] > 0] sum_{d : c[d] > k} G[b][d] P[d][k]   (dF/dA)
//   dP[d][k] = sum_b G[b][d] R[b][k]   if k < c[d]                 (dF/dW2)
//            = sum_b S[b][d] D[b][k]   otherwise                   (dF/dW1)
//   db2 = sum_b G, db1 = sum_b D.
// The masks are staircases in (d, k), so every product only visits the K range a
// tile can see (about half of the dense work) and masks inside the diagonal tiles.
//
// Tile engine: 64 x 64 output tile per workgroup of 4 waves (2 x 2 waves of 32 x 32,
// each 2 x 2 MFMA 16x16 blocks).  Operands are staged through LDS as [row][K] with K
// contiguous (one 16-byte load per thread per operand per K step).  T = bf16 uses
// v_mfma_f32_16x16x32_bf16 (BK = 32); T = float uses v_mfma_f32_16x16x4_f32 (BK = 16).
// Accumulation is always FP32.  Intermediates that a later product contracts over
// the batch (R, G, S, D) are written batch-contiguous (transposed) by the producing
// epilogue, which the MFMA accumulator layout makes a contiguous 4-element store.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int TM = 64, TN = 64;
constexpr int ROWB = 80;  // LDS row stride in bytes (64 data + 16 pad)

template <typename T>
struct Mfma;
template <>
struct Mfma<bf16_t> {
  static constexpr int BK = 32, VEC = 8;
  __device__ static inline void tile(const uint8_t* As, const uint8_t* Bs, int wm, int wn, int lane,
                                     floatx4_t acc[2][2]) {
    bf16x8_t a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *(const bf16x8_t*)(As + (wm + i * 16 + (lane & 15)) * ROWB + (lane >> 4) * 16);
      b[i] = *(const bf16x8_t*)(Bs + (wn + i * 16 + (lane & 15)) * ROWB + (lane >> 4) * 16);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  static constexpr int BK = 16, VEC = 4;
  __device__ static inline void tile(const uint8_t* As, const uint8_t* Bs, int wm, int wn, int lane,
                                     floatx4_t acc[2][2]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *(const float*)(As + (wm + i * 16 + (lane & 15)) * ROWB + (q * 4 + (lane >> 4)) * 4);
        b[i] = *(const float*)(Bs + (wn + i * 16 + (lane & 15)) * ROWB + (q * 4 + (lane >> 4)) * 4);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
};

// 16-byte vector of VEC elements of T
template <typename T>
struct Vec {
  T v[16 / sizeof(T)];
};

template <typename T>
__device__ inline T from_f32(float x);
template <>
__device__ inline float from_f32<float>(float x) { return x; }
template <>
__device__ inline bf16_t from_f32<bf16_t>(float x) { return f32_to_bf16(x); }

template <typename T>
__device__ inline T spin_val(int8_t s);  // exact +-1 / 0
template <>
__device__ inline float spin_val<float>(int8_t s) { return (float)s; }
template <>
__device__ inline bf16_t spin_val<bf16_t>(int8_t s) {
  return s == 0 ? (bf16_t)0 : (s > 0 ? (bf16_t)0x3F80 : (bf16_t)0xBF80);
}

__device__ inline void zero_acc(floatx4_t acc[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
}

// number of d in [0, n) with c[d] <= x  (c non-decreasing)
__device__ inline int count_le(const int32_t* c, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- stage helpers
// Thread t stages row r = t/4, element chunk q = (t%4)*VEC of a 64 x BK tile.
template <typename T>
__device__ inline void store_lds(uint8_t* tile, int t, const Vec<T>& v) {
  *(uint4*)(tile + (t >> 2) * ROWB + (t & 3) * 16) = *(const uint4*)&v;
}

// spins S[b][d0 .. d0+VEC) -> T  (rows b beyond B and sites beyond n read as 0)
template <typename T>
__device__ inline Vec<T> load_spins(const int8_t* S, int64_t lds, int64_t b, int64_t B, int d0, int n) {
  constexpr int VEC = 16 / sizeof(T);
  Vec<T> out;
  if (b < B && d0 + VEC <= n) {
    int8_t tmp[VEC];
    if constexpr (VEC == 8) *(uint2*)tmp = *(const uint2*)(S + b * lds + d0);
    else *(uint32_t*)tmp = *(const uint32_t*)(S + b * lds + d0);
#pragma unroll
    for (int e = 0; e < VEC; ++e) out.v[e] = spin_val<T>(tmp[e]);
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      out.v[e] = (b < B && d0 + e < n) ? spin_val<T>(S[b * lds + d0 + e]) : (T)0;
  }
  return out;
}

// row-major T matrix X[r][k0 .. k0+VEC), rows >= R or columns >= K read as 0
template <typename T>
__device__ inline Vec<T> load_rows(const T* X, int64_t ld, int64_t r, int64_t R, int k0, int K) {
  constexpr int VEC = 16 / sizeof(T);
  Vec<T> out;
  if (r < R && k0 + VEC <= K) {
    *(uint4*)&out = *(const uint4*)(X + r * ld + k0);
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) out.v[e] = (r < R && k0 + e < K) ? X[r * ld + k0 + e] : (T)0;
  }
  return out;
}

// ---------------------------------------------------------------- K1: first layer
// A = S * P_upper + b1 ; writes R = relu(A) (B x ldh) and optionally Rt (h x ldB).
template <typename T, bool WRITE_T>
__global__ __launch_bounds__(256) void fwd_hidden_kernel(const int8_t* __restrict__ S, int64_t lds,
                                                          const T* __restrict__ Pt, int64_t ldn,
                                                          const float* __restrict__ b1,
                                                          const int32_t* __restrict__ c, int n, int h,
                                                          int64_t B, T* __restrict__ R, int64_t ldh,
                                                          T* __restrict__ Rt, int64_t ldB) {
  constexpr int BK = Mfma<T>::BK, VEC = Mfma<T>::VEC;
  __shared__ __attribute__((aligned(16))) uint8_t As[TM * ROWB];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[TN * ROWB];
  __shared__ int kend_s;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int64_t m0 = (int64_t)blockIdx.y * TM;  // samples
  const int n0 = blockIdx.x * TN;               // units
  if (t == 0) kend_s = count_le(c, n, n0 + TN - 1);
  __syncthreads();
  const int kend = kend_s;
  floatx4_t acc[2][2];
  zero_acc(acc);
  const int r = t >> 2, q = (t & 3) * VEC;
  for (int k0 = 0; k0 < kend; k0 += BK) {
    store_lds<T>(As, t, load_spins<T>(S, lds, m0 + r, B, k0 + q, n));
    // B operand: Pt[unit][site], kept where c[site] <= unit
    {
      const int unit = n0 + r;
      Vec<T> v = load_rows<T>(Pt, ldn, unit, h, k0 + q, n);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int d = k0 + q + e;
        if (d >= n || c[d] > unit) v.v[e] = (T)0;
      }
      store_lds<T>(Bs, t, v);
    }
    __syncthreads();
    Mfma<T>::tile(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = n0 + wn + j * 16 + (lane & 15);
      const float bias = (k < h) ? b1[k] : 0.f;
      const int64_t bb = m0 + wm + i * 16 + 4 * (lane >> 4);
      T vals[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float a = acc[i][j][e] + bias;
        vals[e] = from_f32<T>((k < h) ? fmaxf(a, 0.f) : 0.f);
        if (bb + e < B && k < ldh) R[(bb + e) * ldh + k] = vals[e];
      }
      if (WRITE_T && k < h) {
        if (bb + 3 < ldB) {
          T tmp[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) tmp[e] = (bb + e < B) ? vals[e] : (T)0;
          if constexpr (sizeof(T) == 2) *(uint2*)(Rt + (int64_t)k * ldB + bb) = *(uint2*)tmp;
          else *(uint4*)(Rt + (int64_t)k * ldB + bb) = *(uint4*)tmp;
        }
      }
    }
}

// ---------------------------------------------------------------- K2: second layer
// MODE 0: logp partials (+ optional Z).  MODE 1: also G, Gt, St and db2 partials for
// the backward.  MODE 2: plain sampler: draw site `dsel` from the conditional.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void fwd_out_kernel(
    const T* __restrict__ R, int64_t ldh, const T* __restrict__ P, const float* __restrict__ b2,
    const int32_t* __restrict__ c, int n, int h, int64_t B, int8_t* __restrict__ S, int64_t lds,
    int64_t ldn, float* __restrict__ lp_part, float* __restrict__ Z, const float* __restrict__ coef,
    T* __restrict__ G, T* __restrict__ Gt, T* __restrict__ St, int64_t ldB,
    float* __restrict__ db2_part, int dsel, uint64_t seed, uint64_t step, int64_t offset,
    uint32_t tag, float* __restrict__ lp_acc) {
  constexpr int BK = Mfma<T>::BK, VEC = Mfma<T>::VEC;
  __shared__ __attribute__((aligned(16))) uint8_t As[TM * ROWB];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[TN * ROWB];
  __shared__ float rowacc[2][TM];
  __shared__ float colacc[2][TN];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int64_t m0 = (int64_t)blockIdx.y * TM;                       // samples
  const int d0 = (MODE == 2) ? (dsel / TN) * TN : blockIdx.x * TN;  // sites
  const int dlast = min(d0 + TN - 1, n - 1);
  const int kend = c[dlast];
  floatx4_t acc[2][2];
  zero_acc(acc);
  const int r = t >> 2, q = (t & 3) * VEC;
  for (int k0 = 0; k0 < kend; k0 += BK) {
    store_lds<T>(As, t, load_rows<T>(R, ldh, m0 + r, B, k0 + q, h));
    {
      const int d = d0 + r;
      Vec<T> v = load_rows<T>(P, ldh, d, n, k0 + q, h);
      const int cd = (d < n) ? c[d] : 0;
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (k0 + q + e >= cd) v.v[e] = (T)0;
      store_lds<T>(Bs, t, v);
    }
    __syncthreads();
    Mfma<T>::tile(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
  float rs[2][4];
  float cs[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) rs[i][e] = 0.f;
  cs[0] = cs[1] = 0.f;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int d = d0 + wn + j * 16 + (lane & 15);
    const bool dv = d < n;
    const float bias = dv ? b2[d] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t bb = m0 + wm + i * 16 + 4 * (lane >> 4);
      T gv[4], sv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t b = bb + e;
        const bool ok = dv && b < B;
        const float z = acc[i][j][e] + bias;
        if (MODE == 2) {
          if (ok && d == dsel) {
            const float4 u4 = site_uniforms(seed, step, tag, (uint64_t)(b + offset), (uint32_t)(d >> 2));
            const int w = d & 3;
            const float u = w == 0 ? u4.x : (w == 1 ? u4.y : (w == 2 ? u4.z : u4.w));
            const float sg = (u < sigmoid(z)) ? 1.f : -1.f;
            S[b * lds + d] = (int8_t)sg;
            lp_acc[b] += log_sigmoid(sg * z);
          }
          continue;
        }
        const float s = ok ? (float)S[b * lds + d] : 0.f;
        const float tt = s * z;
        if (ok) rs[i][e] += log_sigmoid(tt);
        if (Z && ok) Z[b * ldn + d] = z;
        if (MODE == 1) {
          const float g = ok ? coef[b] * s * sigmoid(-tt) : 0.f;
          cs[j] += g;
          gv[e] = from_f32<T>(g);
          sv[e] = spin_val<T>((int8_t)s);
          if (b < B && d < ldn) G[b * ldn + d] = gv[e];
        }
      }
      if (MODE == 1 && d < n && bb + 3 < ldB) {
        if constexpr (sizeof(T) == 2) {
          *(uint2*)(Gt + (int64_t)d * ldB + bb) = *(uint2*)gv;
          *(uint2*)(St + (int64_t)d * ldB + bb) = *(uint2*)sv;
        } else {
          *(uint4*)(Gt + (int64_t)d * ldB + bb) = *(uint4*)gv;
          *(uint4*)(St + (int64_t)d * ldB + bb) = *(uint4*)sv;
        }
      }
    }
  }
  if (MODE == 2) return;
  // row sums of log sigma over this tile's sites (16-lane rows, then the two wn waves)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float v = rs[i][e];
      v += VQMC_DPP(v, 0xB1);
      v += VQMC_DPP(v, 0x4E);
      v += VQMC_DPP(v, 0x141);
      v += VQMC_DPP(v, 0x140);
      rs[i][e] = v;
    }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) rowacc[wn >> 5][wm + i * 16 + 4 * (lane >> 4) + e] = rs[i][e];
  }
  if (MODE == 1) {
    // column sums of G over this tile's samples
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float v = cs[j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      cs[j] = v;
    }
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < 2; ++j) colacc[wm >> 5][wn + j * 16 + lane] = cs[j];
    }
  }
  __syncthreads();
  if (t < TM) {
    const int64_t b = m0 + t;
    if (b < B) lp_part[(int64_t)blockIdx.x * B + b] = rowacc[0][t] + rowacc[1][t];
  } else if (MODE == 1 && t < TM + TN) {
    const int d = d0 + (t - TM);
    if (d < ldn) db2_part[(int64_t)blockIdx.y * ldn + d] = colacc[0][t - TM] + colacc[1][t - TM];
  }
}

// ---------------------------------------------------------------- K3: hidden adjoint
// D = [A > 0] (G * P_lower) ; writes Dt (h x ldB) and db1 partials.
template <typename T>
__global__ __launch_bounds__(256) void bwd_hidden_kernel(const T* __restrict__ G, int64_t ldn,
                                                          const T* __restrict__ Pt,
                                                          const int32_t* __restrict__ c, int n, int h,
                                                          int64_t B, const T* __restrict__ Rt,
                                                          T* __restrict__ Dt, int64_t ldB,
                                                          float* __restrict__ db1_part, int64_t ldh) {
  constexpr int BK = Mfma<T>::BK, VEC = Mfma<T>::VEC;
  __shared__ __attribute__((aligned(16))) uint8_t As[TM * ROWB];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[TN * ROWB];
  __shared__ float colacc[2][TN];
  __shared__ int kbeg_s;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int64_t m0 = (int64_t)blockIdx.y * TM;  // samples
  const int n0 = blockIdx.x * TN;               // units
  if (t == 0) kbeg_s = count_le(c, n, n0);      // first site with c[d] > n0
  __syncthreads();
  const int kbeg = (kbeg_s / BK) * BK;
  floatx4_t acc[2][2];
  zero_acc(acc);
  const int r = t >> 2, q = (t & 3) * VEC;
  for (int k0 = kbeg; k0 < n; k0 += BK) {
    store_lds<T>(As, t, load_rows<T>(G, ldn, m0 + r, B, k0 + q, n));
    {
      const int unit = n0 + r;
      Vec<T> v = load_rows<T>(Pt, ldn, unit, h, k0 + q, n);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int d = k0 + q + e;
        if (d >= n || c[d] <= unit) v.v[e] = (T)0;
      }
      store_lds<T>(Bs, t, v);
    }
    __syncthreads();
    Mfma<T>::tile(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
  float cs[2] = {0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = n0 + wn + j * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t bb = m0 + wm + i * 16 + 4 * (lane >> 4);
      if (k < h && bb + 3 < ldB) {
        T rv[4], dvv[4];
        if constexpr (sizeof(T) == 2) *(uint2*)rv = *(const uint2*)(Rt + (int64_t)k * ldB + bb);
        else *(uint4*)rv = *(const uint4*)(Rt + (int64_t)k * ldB + bb);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float dl = (to_f32(rv[e]) > 0.f && bb + e < B) ? acc[i][j][e] : 0.f;
          cs[j] += dl;
          dvv[e] = from_f32<T>(dl);
        }
        if constexpr (sizeof(T) == 2) *(uint2*)(Dt + (int64_t)k * ldB + bb) = *(uint2*)dvv;
        else *(uint4*)(Dt + (int64_t)k * ldB + bb) = *(uint4*)dvv;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float v = cs[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    cs[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 2; ++j) colacc[wm >> 5][wn + j * 16 + lane] = cs[j];
  }
  __syncthreads();
  if (t < TN) {
    const int k = n0 + t;
    if (k < ldh) db1_part[(int64_t)blockIdx.y * ldh + k] = colacc[0][t] + colacc[1][t];
  }
}

// ---------------------------------------------------------------- K4: weight gradient
// dP[d][k] = sum_b Gt[d][b] Rt[k][b]  (k < c[d])  or  sum_b St[d][b] Dt[k][b]  (k >= c[d]).
template <typename T>
__global__ __launch_bounds__(256) void bwd_weight_kernel(const T* __restrict__ Gt, const T* __restrict__ St,
                                                          const T* __restrict__ Rt,
                                                          const T* __restrict__ Dt, int64_t ldB,
                                                          const int32_t* __restrict__ c, int n, int h,
                                                          float* __restrict__ dP) {
  constexpr int BK = Mfma<T>::BK, VEC = Mfma<T>::VEC;
  __shared__ __attribute__((aligned(16))) uint8_t As[TM * ROWB];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[TN * ROWB];
  __shared__ __attribute__((aligned(16))) uint8_t As2[TM * ROWB];
  __shared__ __attribute__((aligned(16))) uint8_t Bs2[TN * ROWB];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int d0 = blockIdx.y * TM;  // sites
  const int k0u = blockIdx.x * TN; // units
  const int dlast = min(d0 + TM - 1, n - 1);
  const bool lower = k0u < c[dlast];           // some (d, k) with k < c[d]
  const bool upper = k0u + TN - 1 >= c[d0];    // some (d, k) with k >= c[d]
  floatx4_t accL[2][2], accU[2][2];
  zero_acc(accL);
  zero_acc(accU);
  const int r = t >> 2, q = (t & 3) * VEC;
  for (int kb = 0; kb < ldB; kb += BK) {
    if (lower) {
      store_lds<T>(As, t, load_rows<T>(Gt, ldB, d0 + r, n, kb + q, (int)ldB));
      store_lds<T>(Bs, t, load_rows<T>(Rt, ldB, k0u + r, h, kb + q, (int)ldB));
    }
    if (upper) {
      store_lds<T>(As2, t, load_rows<T>(St, ldB, d0 + r, n, kb + q, (int)ldB));
      store_lds<T>(Bs2, t, load_rows<T>(Dt, ldB, k0u + r, h, kb + q, (int)ldB));
    }
    __syncthreads();
    if (lower) Mfma<T>::tile(As, Bs, wm, wn, lane, accL);
    if (upper) Mfma<T>::tile(As2, Bs2, wm, wn, lane, accU);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = k0u + wn + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int d = d0 + wm + i * 16 + 4 * (lane >> 4) + e;
        if (d < n && k < h) dP[(int64_t)d * h + k] = (k < c[d]) ? accL[i][j][e] : accU[i][j][e];
      }
    }
}

// ---------------------------------------------------------------- reductions
__global__ void sum_rows_kernel(const float* __restrict__ part, int nparts, int64_t stride, int64_t len,
                                float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * stride + i];
  out[i] = s;
}

__global__ void fill_kernel(float* __restrict__ x, int64_t len, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) x[i] = v;
}

__global__ void fill_i8_kernel(int8_t* __restrict__ x, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) x[i] = 0;
}

// ---------------------------------------------------------------- workspace layout
struct WsLayout {
  size_t R, Rt, G, Gt, St, Dt, lp_part, db2_part, db1_part, lp_acc, total;
};

static WsLayout layout(int n, int h, int64_t B, int dtype, int which) {
  const size_t es = (dtype == VQMC_BF16) ? 2 : 4;
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad), ldB = round_up(B, kPad);
  const int64_t ntile_n = ldn / TN, ntile_b = ldB / TM;
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up((int64_t)bytes, 256);
    return o;
  };
  L.R = take((size_t)B * ldh * es);
  L.lp_part = take((size_t)ntile_n * B * 4);
  if (which == 1) {  // backward
    L.Rt = take((size_t)h * ldB * es);
    L.G = take((size_t)B * ldn * es);
    L.Gt = take((size_t)n * ldB * es);
    L.St = take((size_t)n * ldB * es);
    L.Dt = take((size_t)h * ldB * es);
    L.db2_part = take((size_t)ntile_b * ldn * 4);
    L.db1_part = take((size_t)ntile_b * ldh * 4);
  }
  if (which == 2) L.lp_acc = take((size_t)B * 4);  // plain sampler
  L.total = off;
  return L;
}

size_t logprob_ws_bytes(int n, int h, int64_t B, int dtype, bool backward) {
  return layout(n, h, B, dtype, backward ? 1 : 0).total;
}
size_t sample_plain_ws_bytes(int n, int h, int64_t B, int dtype) { return layout(n, h, B, dtype, 2).total; }

template <typename T>
static hipError_t logprob_t(const vqmc_made& m, const int8_t* S, int64_t B, float* logp, float* Z,
                            void* ws, hipStream_t st) {
  const int n = m.n, h = m.h;
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad), ldB = round_up(B, kPad);
  const WsLayout L = layout(n, h, B, m.wdtype, 0);
  uint8_t* w = (uint8_t*)ws;
  T* R = (T*)(w + L.R);
  float* lp_part = (float*)(w + L.lp_part);
  dim3 g1((unsigned)(ldh / TN), (unsigned)(ldB / TM));
  fwd_hidden_kernel<T, false><<<g1, 256, 0, st>>>(S, ldn, (const T*)m.Pt, ldn, m.b1, m.c, n, h, B, R,
                                                  ldh, nullptr, ldB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2((unsigned)(ldn / TN), (unsigned)(ldB / TM));
  fwd_out_kernel<T, 0><<<g2, 256, 0, st>>>(R, ldh, (const T*)m.P, m.b2, m.c, n, h, B, (int8_t*)S, ldn,
                                           ldn, lp_part, Z, nullptr, nullptr, nullptr, nullptr, ldB,
                                           nullptr, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(lp_part, (int)(ldn / TN), B, B, logp);
  return hipGetLastError();
}

template <typename T>
static hipError_t backward_t(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                             float* dP, float* db1, float* db2, void* ws, hipStream_t st) {
  const int n = m.n, h = m.h;
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad), ldB = round_up(B, kPad);
  const WsLayout L = layout(n, h, B, m.wdtype, 1);
  uint8_t* w = (uint8_t*)ws;
  T* R = (T*)(w + L.R);
  T* Rt = (T*)(w + L.Rt);
  T* G = (T*)(w + L.G);
  T* Gt = (T*)(w + L.Gt);
  T* St = (T*)(w + L.St);
  T* Dt = (T*)(w + L.Dt);
  float* lp_part = (float*)(w + L.lp_part);
  float* db2_part = (float*)(w + L.db2_part);
  float* db1_part = (float*)(w + L.db1_part);
  hipError_t e;
  dim3 g1((unsigned)(ldh / TN), (unsigned)(ldB / TM));
  fwd_hidden_kernel<T, true><<<g1, 256, 0, st>>>(S, ldn, (const T*)m.Pt, ldn, m.b1, m.c, n, h, B, R, ldh,
                                                 Rt, ldB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dim3 g2((unsigned)(ldn / TN), (unsigned)(ldB / TM));
  fwd_out_kernel<T, 1><<<g2, 256, 0, st>>>(R, ldh, (const T*)m.P, m.b2, m.c, n, h, B, (int8_t*)S, ldn,
                                           ldn, lp_part, nullptr, coef, G, Gt, St, ldB, db2_part, 0, 0, 0,
                                           0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dim3 g3((unsigned)(ldh / TN), (unsigned)(ldB / TM));
  bwd_hidden_kernel<T><<<g3, 256, 0, st>>>(G, ldn, (const T*)m.Pt, m.c, n, h, B, Rt, Dt, ldB, db1_part,
                                           ldh);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dim3 g4((unsigned)(ldh / TN), (unsigned)(ldn / TM));
  bwd_weight_kernel<T><<<g4, 256, 0, st>>>(Gt, St, Rt, Dt, ldB, m.c, n, h, dP);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(db2_part, (int)(ldB / TM), ldn, n, db2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((h + 255) / 256), 256, 0, st>>>(db1_part, (int)(ldB / TM), ldh, h, db1);
  return hipGetLastError();
}

template <typename T>
static hipError_t sample_plain_t(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                                 int64_t offset, uint32_t tag, int8_t* S, float* logp, void* ws,
                                 hipStream_t st) {
  const int n = m.n, h = m.h;
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad), ldB = round_up(B, kPad);
  const WsLayout L = layout(n, h, B, m.wdtype, 2);
  uint8_t* w = (uint8_t*)ws;
  T* R = (T*)(w + L.R);
  float* lp_acc = (float*)(w + L.lp_acc);
  hipError_t e;
  // Algorithm 1's initial state: unsampled sites are never read (masks); start from 0.
  fill_i8_kernel<<<(unsigned)((B * ldn + 255) / 256), 256, 0, st>>>(S, B * ldn);
  fill_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(lp_acc, B, 0.f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dim3 g1((unsigned)(ldh / TN), (unsigned)(ldB / TM));
  dim3 g2(1, (unsigned)(ldB / TM));
  for (int d = 0; d < n; ++d) {
    // forward pass d over the partially drawn batch ...
    fwd_hidden_kernel<T, false><<<g1, 256, 0, st>>>(S, ldn, (const T*)m.Pt, ldn, m.b1, m.c, n, h, B, R,
                                                    ldh, nullptr, ldB);
    // ... then the output layer for the tile holding site d, and the draw of s_d
    fwd_out_kernel<T, 2><<<g2, 256, 0, st>>>(R, ldh, (const T*)m.P, m.b2, m.c, n, h, B, S, ldn, ldn,
                                             nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, ldB,
                                             nullptr, d, seed, step, offset, tag, lp_acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (logp) return hipMemcpyAsync(logp, lp_acc, (size_t)B * 4, hipMemcpyDeviceToDevice, st);
  return hipSuccess;
}

hipError_t launch_logprob(const vqmc_made& m, const int8_t* S, int64_t B, float* logp, float* Z,
                          void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return logprob_t<bf16_t>(m, S, B, logp, Z, ws, st);
  return logprob_t<float>(m, S, B, logp, Z, ws, st);
}

hipError_t launch_backward(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                           float* dP, float* db1, float* db2, void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return backward_t<bf16_t>(m, S, B, coef, dP, db1, db2, ws, st);
  return backward_t<float>(m, S, B, coef, dP, db1, db2, ws, st);
}

hipError_t launch_sample_plain(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                               int64_t offset, uint32_t tag, int8_t* S, float* logp, void* ws,
                               hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return sample_plain_t<bf16_t>(m, B, seed, step, offset, tag, S, logp, ws, st);
  return sample_plain_t<float>(m, B, seed, step, offset, tag, S, logp, ws, st);
}

}  // namespace vqmc
