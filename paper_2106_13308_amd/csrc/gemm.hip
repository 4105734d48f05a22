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
// Tile engine: a BM x BN output tile per workgroup of 4 waves (2 x 2 waves of
// BM/2 x BN/2, each a grid of MFMA 16x16 blocks).  Operands are staged through LDS as
// [row][K] with K contiguous; the K step after next is loaded into registers while
// the current one is multiplied, with two LDS buffers and one barrier per K step.  T = bf16
// uses v_mfma_f32_16x16x32_bf16 (BK = 32); T = float uses v_mfma_f32_16x16x4_f32
// (BK = 16).  Accumulation is always FP32.  Intermediates that a later product
// contracts over the batch (R, G, S, D) are written batch-contiguous (transposed) by
// the producing epilogue, which the MFMA accumulator layout makes a 4-element store.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int ROWB = 80;  // LDS row stride in bytes (64 data + 16 pad)

// 16-byte vector of T
template <typename T>
struct Vec {
  T v[16 / sizeof(T)];
};

template <typename T>
struct Mfma;
template <>
struct Mfma<bf16_t> {
  static constexpr int BK = 32, VEC = 8;
  template <int FM, int FN>
  __device__ static inline void tile(const uint8_t* As, const uint8_t* Bs, int wm, int wn, int lane,
                                     floatx4_t (&acc)[FM][FN]) {
    bf16x8_t a[FM], b[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      a[i] = *(const bf16x8_t*)(As + (wm + i * 16 + (lane & 15)) * ROWB + (lane >> 4) * 16);
#pragma unroll
    for (int j = 0; j < FN; ++j)
      b[j] = *(const bf16x8_t*)(Bs + (wn + j * 16 + (lane & 15)) * ROWB + (lane >> 4) * 16);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  static constexpr int BK = 16, VEC = 4;
  template <int FM, int FN>
  __device__ static inline void tile(const uint8_t* As, const uint8_t* Bs, int wm, int wn, int lane,
                                     floatx4_t (&acc)[FM][FN]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *(const float*)(As + (wm + i * 16 + (lane & 15)) * ROWB + (q * 4 + (lane >> 4)) * 4);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *(const float*)(Bs + (wn + j * 16 + (lane & 15)) * ROWB + (q * 4 + (lane >> 4)) * 4);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
};


template <typename T>
__device__ inline T spin_val(int8_t s);  // exact +-1 / 0
template <>
__device__ inline float spin_val<float>(int8_t s) { return (float)s; }
template <>
__device__ inline bf16_t spin_val<bf16_t>(int8_t s) {
  return s == 0 ? (bf16_t)0 : (s > 0 ? (bf16_t)0x3F80 : (bf16_t)0xBF80);
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

template <typename T>
__device__ inline void store4(T* p, const T (&v)[4]) {
  if constexpr (sizeof(T) == 2) *(uint2*)p = *(const uint2*)v;
  else *(uint4*)p = *(const uint4*)v;
}

// ---------------------------------------------------------------- operand loaders
// A loader stages 16-byte vectors of one operand.  fetch() only issues the global
// loads of vector v of the thread (row r0 + 64 v) at K index kq; finish() converts /
// masks the raw bytes when the stage is written to LDS.  Keeping the loaded values
// untouched until then lets the loads of later K steps stay in flight while the
// current step is multiplied.

// spins S[b][kq .. kq+VEC) (int8, rows = samples m0 + row) -> T
template <typename T>
struct SpinA {
  static constexpr int VEC = 16 / sizeof(T);
  struct Raw { int8_t s[VEC]; };
  const int8_t* S;
  int64_t lds, B, m0;
  int n, r0;
  __device__ Raw fetch(int v, int kq) const {
    Raw raw;
    const int64_t b = m0 + r0 + 64 * v;
    if (b < B && kq + VEC <= n) {
      if constexpr (VEC == 8) *(uint2*)raw.s = *(const uint2*)(S + b * lds + kq);
      else *(uint32_t*)raw.s = *(const uint32_t*)(S + b * lds + kq);
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) raw.s[e] = (b < B && kq + e < n) ? S[b * lds + kq + e] : (int8_t)0;
    }
    return raw;
  }
  __device__ Vec<T> finish(int, const Raw& raw, int) const {
    Vec<T> out;
#pragma unroll
    for (int e = 0; e < VEC; ++e) out.v[e] = spin_val<T>(raw.s[e]);
    return out;
  }
};

// row-major T matrix, rows R0 + row (< R), K index valid in [lo[v], hi[v]) and < K.
// The MADE staircase masks are prefixes / suffixes of each row, so one (lo, hi) pair
// per staged row expresses them.
template <typename T, int NV>
struct RowsA {
  static constexpr int VEC = 16 / sizeof(T);
  using Raw = uint4;
  const T* X;
  int64_t ld, R0, R;
  int K, r0;
  int lo[NV], hi[NV];
  __device__ Raw fetch(int v, int kq) const {
    uint4 raw = make_uint4(0, 0, 0, 0);
    const int64_t r = R0 + r0 + 64 * v;
    if (r < R && kq < hi[v] && kq + VEC > lo[v]) {
      if (kq + VEC <= K) {
        raw = *(const uint4*)(X + r * ld + kq);
      } else {
        T tmp[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) tmp[e] = (kq + e < K) ? X[r * ld + kq + e] : (T)0;
        raw = *(const uint4*)tmp;
      }
    }
    return raw;
  }
  __device__ Vec<T> finish(int v, const Raw& raw, int kq) const {
    Vec<T> out = *(const Vec<T>*)&raw;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      if (kq + e < lo[v] || kq + e >= hi[v]) out.v[e] = (T)0;
    return out;
  }
};

// ---------------------------------------------------------------- tile engine
// Thread t stages rows (t / 4) + 64 v, element chunk (t % 4) * VEC of each operand.
template <typename T, int BM, int BN, int PD = 6>
struct Engine {
  static constexpr int BK = Mfma<T>::BK, VEC = Mfma<T>::VEC;
  static constexpr int FM = BM / 32, FN = BN / 32;
  static constexpr int AV = BM / 64, BV = BN / 64;
  static constexpr int STAGE = (BM + BN) * ROWB;
  static constexpr int SMEM = 2 * STAGE;

  template <class LA, class LB>
  __device__ static void run(uint8_t* smem, int kbeg, int kend, const LA& la, const LB& lb,
                             floatx4_t (&acc)[FM][FN]) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv >> 1) * (BM / 2), wn = (wv & 1) * (BN / 2);
    const int r0 = t >> 2, q = (t & 3) * VEC;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    if (kbeg >= kend) return;
    // a ring of PD raw register sets: the stage multiplied at step i was fetched at step
    // i - PD + 1, so PD - 1 steps of work cover the global-memory latency
    typename LA::Raw ra[PD][AV];
    typename LB::Raw rb[PD][BV];
    const int nsteps = (kend - kbeg + BK - 1) / BK;
#pragma unroll
    for (int p = 0; p < PD; ++p)
      if (p < nsteps) {
#pragma unroll
        for (int v = 0; v < AV; ++v) ra[p][v] = la.fetch(v, kbeg + p * BK + q);
#pragma unroll
        for (int v = 0; v < BV; ++v) rb[p][v] = lb.fetch(v, kbeg + p * BK + q);
      }
    auto store = [&](uint8_t* st, int p, int k) {
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const Vec<T> x = la.finish(v, ra[p][v], k + q);
        *(uint4*)(st + (r0 + 64 * v) * ROWB + (t & 3) * 16) = *(const uint4*)&x;
      }
#pragma unroll
      for (int v = 0; v < BV; ++v) {
        const Vec<T> x = lb.finish(v, rb[p][v], k + q);
        *(uint4*)(st + (BM + r0 + 64 * v) * ROWB + (t & 3) * 16) = *(const uint4*)&x;
      }
    };
    store(smem, 0, kbeg);
    __syncthreads();
    for (int base = 0; base < nsteps; base += PD) {
#pragma unroll
      for (int p = 0; p < PD; ++p) {
        const int i = base + p;  // step being multiplied (its stage is in LDS buffer i & 1)
        if (i < nsteps) {
          // refill the ring slot of step i with step i + PD
          if (i + PD < nsteps) {
#pragma unroll
            for (int v = 0; v < AV; ++v) ra[p][v] = la.fetch(v, kbeg + (i + PD) * BK + q);
#pragma unroll
            for (int v = 0; v < BV; ++v) rb[p][v] = lb.fetch(v, kbeg + (i + PD) * BK + q);
          }
          const uint8_t* st = smem + (i & 1) * STAGE;
          Mfma<T>::template tile<FM, FN>(st, st + BM * ROWB, wm, wn, lane, acc);
          if (i + 1 < nsteps) store(smem + ((i + 1) & 1) * STAGE, (p + 1) % PD, kbeg + (i + 1) * BK);
          __syncthreads();
        }
      }
    }
  }
};

template <typename T, int NV>
__device__ inline RowsA<T, NV> rows_plain(const T* X, int64_t ld, int64_t R0, int64_t R, int K, int r0) {
  RowsA<T, NV> L{X, ld, R0, R, K, r0, {}, {}};
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    L.lo[v] = 0;
    L.hi[v] = K;
  }
  return L;
}

// tile shapes of the four products
// 64 x 64 tiles everywhere: many workgroups per CU hide latency that one cannot
constexpr int H_BM = 64, H_BN = 64;     // hidden-layer products (N = h)
constexpr int O_BM = 64, O_BN = 64;     // output-layer product (N = n)
constexpr int W_BM = 64, W_BN = 64;     // weight gradient (M = n, N = h)

// ---------------------------------------------------------------- K1: first layer
// A = S * P_upper + b1 ; writes R = relu(A) (B x ldh) and optionally Rt (h x ldB).
// Unit k receives site d iff c[d] <= k, i.e. d < count_le(c, k): a prefix of Pt's row.
// N tiles run in decreasing order of their K range (largest first).
// RELU = false writes the pre-activation itself (the first layer applied to a direction in
// parameter space, for the forward-mode product of the SR update; in FP32 (TR = float) for the
// single-flip differences of the TIM local energy).
template <typename T, bool WRITE_T, bool RELU = true, typename TR = T>
__global__ __launch_bounds__(256) void fwd_hidden_kernel(const int8_t* __restrict__ S, int64_t lds,
                                                          const T* __restrict__ Pt, int64_t ldn,
                                                          const float* __restrict__ b1,
                                                          const int32_t* __restrict__ c, int n, int h,
                                                          int64_t B, TR* __restrict__ R, int64_t ldh,
                                                          T* __restrict__ Rt, int64_t ldB) {
  using E = Engine<T, H_BM, H_BN>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[E::SMEM];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * (H_BM / 2), wn = (wv & 1) * (H_BN / 2);
  const int r0 = t >> 2;
  const int64_t m0 = (int64_t)blockIdx.y * H_BM;                   // samples
  const int n0 = (gridDim.x - 1 - blockIdx.x) * H_BN;              // units
  const int kend = count_le(c, n, n0 + H_BN - 1);
  const SpinA<T> la{S, lds, B, m0, n, r0};
  RowsA<T, E::BV> lb{Pt, ldn, n0, h, n, r0, {}, {}};
#pragma unroll
  for (int v = 0; v < E::BV; ++v) {
    const int unit = n0 + r0 + 64 * v;
    lb.lo[v] = 0;
    lb.hi[v] = (unit < h) ? count_le(c, n, unit) : 0;
  }
  floatx4_t acc[E::FM][E::FN];
  E::run(smem, 0, kend, la, lb, acc);
#pragma unroll
  for (int i = 0; i < E::FM; ++i)
#pragma unroll
    for (int j = 0; j < E::FN; ++j) {
      const int k = n0 + wn + j * 16 + (lane & 15);
      const float bias = (k < h) ? b1[k] : 0.f;
      const int64_t bb = m0 + wm + i * 16 + 4 * (lane >> 4);
      T vals[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float a = acc[i][j][e] + bias;
        const float v = (k < h && bb + e < B) ? (RELU ? fmaxf(a, 0.f) : a) : 0.f;
        vals[e] = from_f32<T>(v);
        if (bb + e < B && k < ldh) R[(bb + e) * ldh + k] = from_f32<TR>(v);
      }
      if (WRITE_T && k < h && bb + 3 < ldB) store4<T>(Rt + (int64_t)k * ldB + bb, vals);
    }
}

// ---------------------------------------------------------------- K2: second layer
// MODE 0: logp partials (+ optional Z).  MODE 1: also G, Gt, St and db2 partials for
// the backward.  MODE 2: plain sampler: draw site `dsel` from the conditional.
// Unit k feeds site d iff k < c[d]: a prefix of P's row d.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void fwd_out_kernel(
    const T* __restrict__ R, int64_t ldh, const T* __restrict__ P, const float* __restrict__ b2,
    const int32_t* __restrict__ c, int n, int h, int64_t B, int8_t* __restrict__ S, int64_t lds,
    int64_t ldn, float* __restrict__ lp_part, float* __restrict__ Z, const float* __restrict__ coef,
    T* __restrict__ G, T* __restrict__ Gt, T* __restrict__ St, int64_t ldB,
    float* __restrict__ db2_part, int dsel, uint64_t seed, uint64_t step, int64_t offset,
    uint32_t tag, float* __restrict__ lp_acc) {
  using E = Engine<T, O_BM, O_BN>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[E::SMEM];
  __shared__ float rowacc[2][O_BM];
  __shared__ float colacc[2][O_BN];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * (O_BM / 2), wn = (wv & 1) * (O_BN / 2);
  const int r0 = t >> 2;
  const int64_t m0 = (int64_t)blockIdx.y * O_BM;  // samples
  const int tile = (MODE == 2) ? dsel / O_BN : (int)(gridDim.x - 1 - blockIdx.x);
  const int d0 = tile * O_BN;                     // sites
  const int kend = c[min(d0 + O_BN - 1, n - 1)];
  const RowsA<T, E::AV> la = rows_plain<T, E::AV>(R, ldh, m0, B, h, r0);
  RowsA<T, E::BV> lb{P, ldh, d0, n, h, r0, {}, {}};
#pragma unroll
  for (int v = 0; v < E::BV; ++v) {
    const int d = d0 + r0 + 64 * v;
    lb.lo[v] = 0;
    lb.hi[v] = (d < n) ? c[d] : 0;
  }
  // the epilogue's spins and coefficients are loaded before the K loop so that their
  // latency is hidden behind it
  int8_t spre[E::FM][E::FN][4];
  float cpre[E::FM][4];
  if constexpr (MODE != 2) {
#pragma unroll
    for (int i = 0; i < E::FM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t b = m0 + wm + i * 16 + 4 * (lane >> 4) + e;
        cpre[i][e] = (MODE == 1 && b < B) ? coef[b] : 0.f;
#pragma unroll
        for (int j = 0; j < E::FN; ++j) {
          const int d = d0 + wn + j * 16 + (lane & 15);
          spre[i][j][e] = (b < B && d < n) ? S[b * lds + d] : (int8_t)0;
        }
      }
  }
  floatx4_t acc[E::FM][E::FN];
  E::run(smem, 0, kend, la, lb, acc);
  if constexpr (MODE == 2) {
    // draw s_d for d = dsel from sigma(z_d): the lanes holding column dsel park the
    // logits in LDS, then one thread per sample draws
    const int col = dsel - d0 - wn;  // column inside this wave's sub-tile
    if (col >= 0 && col < O_BN / 2 && (col & 15) == (lane & 15)) {
#pragma unroll
      for (int j = 0; j < E::FN; ++j)
        if (j == (col >> 4)) {
#pragma unroll
          for (int i = 0; i < E::FM; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) rowacc[0][wm + i * 16 + 4 * (lane >> 4) + e] = acc[i][j][e];
        }
    }
    __syncthreads();
    if (t < O_BM && m0 + t < B) {
      const int64_t b = m0 + t;
      const float z = rowacc[0][t] + b2[dsel];
      const float4 u4 = site_uniforms(seed, step, tag, (uint64_t)(b + offset), (uint32_t)(dsel >> 2));
      const int w = dsel & 3;
      const float u = w == 0 ? u4.x : (w == 1 ? u4.y : (w == 2 ? u4.z : u4.w));
      const float sg = (u < sigmoid(z)) ? 1.f : -1.f;
      S[b * lds + dsel] = (int8_t)sg;
      lp_acc[b] += log_sigmoid(sg * z);
    }
    return;
  }
  float rs[E::FM][4];
  float cs[E::FN];
#pragma unroll
  for (int i = 0; i < E::FM; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) rs[i][e] = 0.f;
#pragma unroll
  for (int j = 0; j < E::FN; ++j) cs[j] = 0.f;
#pragma unroll
  for (int j = 0; j < E::FN; ++j) {
    const int d = d0 + wn + j * 16 + (lane & 15);
    const bool dv = d < n;
    const float bias = dv ? b2[d] : 0.f;
#pragma unroll
    for (int i = 0; i < E::FM; ++i) {
      const int64_t bb = m0 + wm + i * 16 + 4 * (lane >> 4);
      T gv[4], sv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t b = bb + e;
        const bool ok = dv && b < B;
        const float z = acc[i][j][e] + bias;
        const float s = (float)spre[i][j][e];
        const float tt = s * z;
        if (ok) rs[i][e] += log_sigmoid(tt);
        if (Z && ok) Z[b * ldn + d] = z;
        if (MODE == 1) {
          const float g = ok ? cpre[i][e] * s * sigmoid(-tt) : 0.f;
          cs[j] += g;
          gv[e] = from_f32<T>(g);
          sv[e] = spin_val<T>((int8_t)s);
          if (b < B && d < ldn) G[b * ldn + d] = gv[e];
        }
      }
      if (MODE == 1 && d < n && bb + 3 < ldB) {
        store4<T>(Gt + (int64_t)d * ldB + bb, gv);
        store4<T>(St + (int64_t)d * ldB + bb, sv);
      }
    }
  }
  // row sums of log sigma over this tile's sites (16-lane rows, then the two wn waves)
#pragma unroll
  for (int i = 0; i < E::FM; ++i)
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
    for (int i = 0; i < E::FM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) rowacc[wv & 1][wm + i * 16 + 4 * (lane >> 4) + e] = rs[i][e];
  }
  if (MODE == 1) {
    // column sums of G over this tile's samples
#pragma unroll
    for (int j = 0; j < E::FN; ++j) {
      float v = cs[j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      cs[j] = v;
    }
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < E::FN; ++j) colacc[wv >> 1][wn + j * 16 + lane] = cs[j];
    }
  }
  __syncthreads();
  if (t < O_BM) {
    const int64_t b = m0 + t;
    if (b < B) lp_part[(int64_t)tile * B + b] = rowacc[0][t] + rowacc[1][t];
  } else if (MODE == 1) {
    const int dl = t - O_BM;
    const int d = d0 + dl;
    if (dl < O_BN && d < ldn) db2_part[(int64_t)blockIdx.y * ldn + d] = colacc[0][dl] + colacc[1][dl];
  }
}

// ---------------------------------------------------------------- K3: hidden adjoint
// D = [A > 0] (G * P_lower) ; writes Dt (h x ldB) and db1 partials.
// Unit k feeds site d iff c[d] > k, i.e. d >= count_le(c, k): a suffix of Pt's row.
// Tiles of small k have the longest K range and come first in the grid.
template <typename T>
__global__ __launch_bounds__(256) void bwd_hidden_kernel(const T* __restrict__ G, int64_t ldn,
                                                          const T* __restrict__ Pt,
                                                          const int32_t* __restrict__ c, int n, int h,
                                                          int64_t B, const T* __restrict__ Rt,
                                                          T* __restrict__ Dt, int64_t ldB,
                                                          float* __restrict__ db1_part, int64_t ldh) {
  using E = Engine<T, H_BM, H_BN>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[E::SMEM];
  __shared__ float colacc[2][H_BN];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * (H_BM / 2), wn = (wv & 1) * (H_BN / 2);
  const int r0 = t >> 2;
  const int64_t m0 = (int64_t)blockIdx.y * H_BM;  // samples
  const int n0 = blockIdx.x * H_BN;               // units
  const int kbeg = (count_le(c, n, n0) / E::BK) * E::BK;
  const RowsA<T, E::AV> la = rows_plain<T, E::AV>(G, ldn, m0, B, n, r0);
  RowsA<T, E::BV> lb{Pt, ldn, n0, h, n, r0, {}, {}};
#pragma unroll
  for (int v = 0; v < E::BV; ++v) {
    const int unit = n0 + r0 + 64 * v;
    lb.lo[v] = (unit < h) ? count_le(c, n, unit) : n;
    lb.hi[v] = n;
  }
  floatx4_t acc[E::FM][E::FN];
  E::run(smem, kbeg, n, la, lb, acc);
  float cs[E::FN];
#pragma unroll
  for (int j = 0; j < E::FN; ++j) cs[j] = 0.f;
#pragma unroll
  for (int j = 0; j < E::FN; ++j) {
    const int k = n0 + wn + j * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < E::FM; ++i) {
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
        store4<T>(Dt + (int64_t)k * ldB + bb, dvv);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < E::FN; ++j) {
    float v = cs[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    cs[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < E::FN; ++j) colacc[wv >> 1][wn + j * 16 + lane] = cs[j];
  }
  __syncthreads();
  if (t < H_BN) {
    const int k = n0 + t;
    if (k < ldh) db1_part[(int64_t)blockIdx.y * ldh + k] = colacc[0][t] + colacc[1][t];
  }
}

// ---------------------------------------------------------------- K4: weight gradient
// UPPER = false: dP[d][k] = sum_b Gt[d][b] Rt[k][b] where k < c[d]   (dF/dW2)
// UPPER = true:  dP[d][k] = sum_b St[d][b] Dt[k][b] where k >= c[d]  (dF/dW1)
// Tiles without any element of their half return at once.
template <typename T, bool UPPER>
__global__ __launch_bounds__(256) void bwd_weight_kernel(const T* __restrict__ X, const T* __restrict__ Y,
                                                          int64_t ldB, const int32_t* __restrict__ c,
                                                          int n, int h, float* __restrict__ dP) {
  using E = Engine<T, W_BM, W_BN>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[E::SMEM];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * (W_BM / 2), wn = (wv & 1) * (W_BN / 2);
  const int r0 = t >> 2;
  const int d0 = blockIdx.y * W_BM;   // sites
  const int k0u = blockIdx.x * W_BN;  // units
  const int dlast = min(d0 + W_BM - 1, n - 1);
  const bool any = UPPER ? (k0u + W_BN - 1 >= c[d0]) : (k0u < c[dlast]);
  if (!any) return;
  const RowsA<T, E::AV> la = rows_plain<T, E::AV>(X, ldB, d0, n, (int)ldB, r0);
  const RowsA<T, E::BV> lb = rows_plain<T, E::BV>(Y, ldB, k0u, h, (int)ldB, r0);
  floatx4_t acc[E::FM][E::FN];
  E::run(smem, 0, (int)ldB, la, lb, acc);
#pragma unroll
  for (int i = 0; i < E::FM; ++i)
#pragma unroll
    for (int j = 0; j < E::FN; ++j) {
      const int k = k0u + wn + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int d = d0 + wm + i * 16 + 4 * (lane >> 4) + e;
        if (d < n && k < h && (UPPER ? (k >= c[d]) : (k < c[d]))) dP[(int64_t)d * h + k] = acc[i][j][e];
      }
    }
}

// ---------------------------------------------------------------- K2': output adjoint from
// the sampler's logits.  The incremental sampler has already evaluated every logit; with
// zs = s_d z_d it gives G = coef_b s_d sigma(-zs) directly (G, and batch-contiguous Gt, St,
// and db2 partials, as K2 MODE 1 writes them).  64 samples x 64 sites per workgroup; the
// transposed stores go through LDS.
template <typename T>
__global__ __launch_bounds__(256) void grad_out_kernel(const float* __restrict__ Zs, const int8_t* __restrict__ S,
                                                        int64_t ldn, const float* __restrict__ coef, int n, int64_t B,
                                                        T* __restrict__ G, T* __restrict__ Gt, T* __restrict__ St,
                                                        int64_t ldB, float* __restrict__ db2_part) {
  __shared__ float gs[64][65];
  __shared__ int8_t sv[64][68];
  const int t = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * 64;  // samples
  const int d0 = blockIdx.x * 64;               // sites
  {
    const int r = t >> 2, q = (t & 3) * 16;
    const int64_t b = m0 + r;
    float z[16];
    int8_t s[16];
    float cb = 0.f;
    if (b < B) {
      const float* zrow = Zs + b * ldn + d0 + q;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float4 x = *(const float4*)(zrow + 4 * v);
        z[4 * v] = x.x; z[4 * v + 1] = x.y; z[4 * v + 2] = x.z; z[4 * v + 3] = x.w;
      }
      *(uint4*)s = *(const uint4*)(S + b * ldn + d0 + q);
      cb = coef[b];
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        z[e] = 0.f;
        s[e] = 0;
      }
    }
    T gv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const bool ok = b < B && d0 + q + e < n;
      const float g = ok ? cb * (float)s[e] * sigmoid(-z[e]) : 0.f;
      gv[e] = from_f32<T>(g);
      gs[r][q + e] = g;
      sv[r][q + e] = ok ? s[e] : (int8_t)0;
    }
    if (b < B) {
      T* grow = G + b * ldn + d0 + q;
      if constexpr (sizeof(T) == 2) {
        *(uint4*)grow = *(const uint4*)gv;
        *(uint4*)(grow + 8) = *(const uint4*)(gv + 8);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) *(uint4*)(grow + 4 * v) = *(const uint4*)(gv + 4 * v);
      }
    }
  }
  __syncthreads();
  {
    const int dl = t >> 2, bq = (t & 3) * 16;
    const int d = d0 + dl;
    float colsum = 0.f;
    T gv[16], svv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const float g = gs[bq + e][dl];
      colsum += g;
      gv[e] = from_f32<T>(g);
      svv[e] = spin_val<T>(sv[bq + e][dl]);
    }
    if (d < n) {
      T* go = Gt + (int64_t)d * ldB + m0 + bq;
      T* so = St + (int64_t)d * ldB + m0 + bq;
      if constexpr (sizeof(T) == 2) {
        *(uint4*)go = *(const uint4*)gv;
        *(uint4*)(go + 8) = *(const uint4*)(gv + 8);
        *(uint4*)so = *(const uint4*)svv;
        *(uint4*)(so + 8) = *(const uint4*)(svv + 8);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          *(uint4*)(go + 4 * v) = *(const uint4*)(gv + 4 * v);
          *(uint4*)(so + 4 * v) = *(const uint4*)(svv + 4 * v);
        }
      }
    }
    // the 4 threads of a site are adjacent lanes: fixed-order butterfly
    colsum += __shfl_xor(colsum, 1);
    colsum += __shfl_xor(colsum, 2);
    if ((t & 3) == 0 && d < ldn) db2_part[(int64_t)blockIdx.y * ldn + d] = colsum;
  }
}

// ---------------------------------------------------------------- reductions
// out[i] = sum_p part[p][i] in the fixed order of sum_parts
__global__ void sum_rows_kernel(const float* __restrict__ part, int nparts, int64_t stride, int64_t len,
                                float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  out[i] = sum_parts(part, nparts, stride, i);
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
struct Geom {
  int n, h;
  int64_t B, ldh, ldn, ldB;
  int mt_h, nt_h;   // hidden-layer grid: M tiles (batch) x N tiles (units)
  int mt_o, nt_o;   // output-layer grid: M tiles (batch) x N tiles (sites)
  int mt_w, nt_w;   // weight-gradient grid: M tiles (sites) x N tiles (units)
};

static Geom geom(int n, int h, int64_t B) {
  Geom g;
  g.n = n;
  g.h = h;
  g.B = B;
  g.ldh = round_up(h, kPad);
  g.ldn = round_up(n, kPad);
  g.ldB = round_up(B, kPad);
  g.mt_h = (int)((g.ldB + H_BM - 1) / H_BM);
  g.nt_h = (int)((g.ldh + H_BN - 1) / H_BN);
  g.mt_o = (int)((g.ldB + O_BM - 1) / O_BM);
  g.nt_o = (int)((g.ldn + O_BN - 1) / O_BN);
  g.mt_w = (int)((g.ldn + W_BM - 1) / W_BM);
  g.nt_w = (int)((g.ldh + W_BN - 1) / W_BN);
  return g;
}

struct WsLayout {
  size_t R, Rt, G, Gt, St, Dt, lp_part, db2_part, db1_part, lp_acc, total;
};

static WsLayout layout(int n, int h, int64_t B, int dtype, int which) {
  const size_t es = (dtype == VQMC_BF16) ? 2 : 4;
  const Geom g = geom(n, h, B);
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up((int64_t)bytes, 256);
    return o;
  };
  L.R = take((size_t)B * g.ldh * es);
  L.lp_part = take((size_t)g.nt_o * B * 4);
  if (which == 1) {  // backward
    L.Rt = take((size_t)h * g.ldB * es);
    L.G = take((size_t)B * g.ldn * es);
    L.Gt = take((size_t)n * g.ldB * es);
    L.St = take((size_t)n * g.ldB * es);
    L.Dt = take((size_t)h * g.ldB * es);
    L.db2_part = take((size_t)g.mt_o * g.ldn * 4);
    L.db1_part = take((size_t)g.mt_h * g.ldh * 4);
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
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 0);
  uint8_t* w = (uint8_t*)ws;
  T* R = (T*)(w + L.R);
  float* lp_part = (float*)(w + L.lp_part);
  fwd_hidden_kernel<T, false><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, (const T*)m.Pt, g.ldn, m.b1,
                                                                     m.c, m.n, m.h, B, R, g.ldh, nullptr, g.ldB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fwd_out_kernel<T, 0><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(
      R, g.ldh, (const T*)m.P, m.b2, m.c, m.n, m.h, B, (int8_t*)S, g.ldn, g.ldn, lp_part, Z, nullptr, nullptr,
      nullptr, nullptr, g.ldB, nullptr, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(lp_part, g.nt_o, B, B, logp);
  return hipGetLastError();
}

template <typename T>
static hipError_t backward_t(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                             float* dP, float* db1, float* db2, void* ws, hipStream_t st, hipEvent_t coef_ready) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 1);
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
  fwd_hidden_kernel<T, true><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, (const T*)m.Pt, g.ldn, m.b1, m.c,
                                                                    m.n, m.h, B, R, g.ldh, Rt, g.ldB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the first product does not read coef; it may overlap the work that produces it
  if (coef_ready && (e = hipStreamWaitEvent(st, coef_ready, 0)) != hipSuccess) return e;
  fwd_out_kernel<T, 1><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(
      R, g.ldh, (const T*)m.P, m.b2, m.c, m.n, m.h, B, (int8_t*)S, g.ldn, g.ldn, lp_part, nullptr, coef, G, Gt,
      St, g.ldB, db2_part, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  bwd_hidden_kernel<T><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(G, g.ldn, (const T*)m.Pt, m.c, m.n, m.h, B, Rt, Dt,
                                                             g.ldB, db1_part, g.ldh);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  bwd_weight_kernel<T, false><<<dim3(g.nt_w, g.mt_w), 256, 0, st>>>(Gt, Rt, g.ldB, m.c, m.n, m.h, dP);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  bwd_weight_kernel<T, true><<<dim3(g.nt_w, g.mt_w), 256, 0, st>>>(St, Dt, g.ldB, m.c, m.n, m.h, dP);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((m.n + 255) / 256), 256, 0, st>>>(db2_part, g.mt_o, g.ldn, m.n, db2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((m.h + 255) / 256), 256, 0, st>>>(db1_part, g.mt_h, g.ldh, m.h, db1);
  return hipGetLastError();
}

// Factors of the per-sample scores for the SR Gram: the recompute path of backward_t with
// coef = 1 leaves Rt = relu(A), Gt = s sigma(-s z), St = s and Dt = dlogp/dA in the
// workspace, batch-contiguous; sr.hip turns them into K.  Workspace: the backward layout,
// then B ones, then the sweeps' B x B partial sums.
static size_t sr_extra_offset(int n, int h, int64_t B, int dtype) {
  return (size_t)round_up((int64_t)layout(n, h, B, dtype, 1).total, 256);
}
size_t sr_gram_ws_bytes(int n, int h, int64_t B, int dtype) {
  return sr_extra_offset(n, h, B, dtype) + (size_t)round_up(B * 4, 256) + sr_gram_parts_bytes(n, h, B, dtype);
}

// The hidden adjoint of the Gram's factors: BF16 with the sampler tables on the direct-to-LDS
// engine (their masked copy of P^T), else the register-staged one.
template <typename T>
static hipError_t sr_hidden_adjoint(const vqmc_made& m, int64_t B, const Geom& g, const T* G, const T* Rt, T* Dt,
                                    float* db1_part, hipStream_t st) {
  if (sizeof(T) == 2 && m.band) {
    int64_t zo, uo, po;
    int nzt, nut;
    sample_tables_layout(m.n, m.h, m.wdtype, &zo, &uo, &po, &nzt, &nut);
    return launch_bwd_hidden2(m, B, (const uint16_t*)G, (const uint16_t*)((const uint8_t*)m.band + po),
                              (const uint16_t*)Rt, (uint16_t*)Dt, db1_part, st);
  }
  bwd_hidden_kernel<T><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(G, g.ldn, (const T*)m.Pt, m.c, m.n, m.h, B, Rt, Dt,
                                                             g.ldB, db1_part, g.ldh);
  return hipGetLastError();
}

template <typename T>
static hipError_t sr_gram_t(const vqmc_made& m, const int8_t* S, int64_t B, float* K, void* ws, hipStream_t st) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 1);
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
  const size_t xo = sr_extra_offset(m.n, m.h, B, m.wdtype);
  float* ones = (float*)(w + xo);
  float* parts = (float*)(w + xo + round_up(B * 4, 256));
  hipError_t e;
  fill_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(ones, B, 1.f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fwd_hidden_kernel<T, true><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, (const T*)m.Pt, g.ldn, m.b1, m.c,
                                                                    m.n, m.h, B, R, g.ldh, Rt, g.ldB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fwd_out_kernel<T, 1><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(
      R, g.ldh, (const T*)m.P, m.b2, m.c, m.n, m.h, B, (int8_t*)S, g.ldn, g.ldn, lp_part, nullptr, ones, G, Gt,
      St, g.ldB, db2_part, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sr_hidden_adjoint<T>(m, B, g, G, Rt, Dt, db1_part, st)) != hipSuccess) return e;
  return launch_sr_gram_sweeps(m.wdtype, Gt, Rt, Dt, St, g.ldB, m.c, m.n, m.h, B, parts, K, st, G, S, g.ldn);
}

// The same Gram from the incremental sampler's byproducts: Zs (s_d z_d) gives G through the
// output-layer adjoint with coef = 1 and Rt (relu(A)) is used as it is, so the two
// forward products are not recomputed.
template <typename T>
static hipError_t sr_gram_sampled_t(const vqmc_made& m, const int8_t* S, int64_t B, const float* Zs, const T* Rt,
                                    float* K, void* ws, hipStream_t st) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 1);
  uint8_t* w = (uint8_t*)ws;
  T* G = (T*)(w + L.G);
  T* Gt = (T*)(w + L.Gt);
  T* St = (T*)(w + L.St);
  T* Dt = (T*)(w + L.Dt);
  float* db2_part = (float*)(w + L.db2_part);
  float* db1_part = (float*)(w + L.db1_part);
  const size_t xo = sr_extra_offset(m.n, m.h, B, m.wdtype);
  float* ones = (float*)(w + xo);
  float* parts = (float*)(w + xo + round_up(B * 4, 256));
  hipError_t e;
  fill_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(ones, B, 1.f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  grad_out_kernel<T><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(Zs, S, g.ldn, ones, m.n, B, G, Gt, St, g.ldB, db2_part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sr_hidden_adjoint<T>(m, B, g, G, Rt, Dt, db1_part, st)) != hipSuccess) return e;
  return launch_sr_gram_sweeps(m.wdtype, Gt, Rt, Dt, St, g.ldB, m.c, m.n, m.h, B, parts, K, st, G, S, g.ldn);
}

hipError_t launch_sr_gram_sampled(const vqmc_made& m, const int8_t* S, int64_t B, const float* Zs, const void* Rt,
                                  float* K, void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return sr_gram_sampled_t<bf16_t>(m, S, B, Zs, (const bf16_t*)Rt, K, ws, st);
  return sr_gram_sampled_t<float>(m, S, B, Zs, (const float*)Rt, K, ws, st);
}

hipError_t launch_sr_gram(const vqmc_made& m, const int8_t* S, int64_t B, float* K, void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return sr_gram_t<bf16_t>(m, S, B, K, ws, st);
  return sr_gram_t<float>(m, S, B, K, ws, st);
}

// Forward-mode product of the SR update: v[b] = <grad log pi(s_b), g> for a direction
// g = (gP, gb1, gb2) in parameter space (gP packed like P, n x h float32):
//   v_b = sum_d G_bd (gb2_d + sum_{k < c[d]} R_bk gP[d][k]) + sum_k D_bk (gb1_k + sum_{d : c[d] <= k} s_bd gP[d][k])
// i.e. the two masked layers applied with g in place of the weights (the first without its
// ReLU), each contracted with the score factors G and D of the same sample.
template <typename T>
__global__ __launch_bounds__(256) void sr_jvp_dot_kernel(const T* __restrict__ G, const float* __restrict__ U,
                                                         int64_t ldn, int n, const T* __restrict__ Dt,
                                                         const T* __restrict__ Vt, int64_t ldb, int h, int64_t B,
                                                         float* __restrict__ v) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // one wave per sample
  if (b >= B) return;
  float s = 0.f;
  for (int d = lane; d < n; d += 64) s = fmaf(to_f32<T>(G[b * ldn + d]), U[b * ldn + d], s);
  for (int k = lane; k < h; k += 64) s = fmaf(to_f32<T>(Dt[(int64_t)k * ldb + b]), to_f32<T>(Vt[(int64_t)k * ldb + b]), s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) v[b] = s;
}

size_t sr_jvp_ws_bytes(int n, int h, int64_t B, int dtype) {
  const size_t es = (dtype == VQMC_BF16) ? 2 : 4;
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad);
  return sr_extra_offset(n, h, B, dtype) + (size_t)round_up(B * 4, 256) + (size_t)round_up(n * ldh * es, 256) +
         (size_t)round_up(h * ldn * es, 256) + (size_t)round_up(B * ldn * 4, 256);
}

template <typename T>
static hipError_t sr_jvp_t(const vqmc_made& m, const int8_t* S, int64_t B, const float* gP, const float* gb1,
                           const float* gb2, float* v, void* ws, hipStream_t st) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 1);
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
  const size_t es = sizeof(T);
  size_t off = sr_extra_offset(m.n, m.h, B, m.wdtype);
  float* ones = (float*)(w + off);
  off += round_up(B * 4, 256);
  T* gPw = (T*)(w + off);
  off += round_up(m.n * g.ldh * (int64_t)es, 256);
  T* gPtw = (T*)(w + off);
  off += round_up(m.h * g.ldn * (int64_t)es, 256);
  float* U = (float*)(w + off);
  hipError_t e;
  fill_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(ones, B, 1.f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // score factors: R (and Rt), G with coef = 1, D
  fwd_hidden_kernel<T, true><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, (const T*)m.Pt, g.ldn, m.b1, m.c,
                                                                    m.n, m.h, B, R, g.ldh, Rt, g.ldB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fwd_out_kernel<T, 1><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(
      R, g.ldh, (const T*)m.P, m.b2, m.c, m.n, m.h, B, (int8_t*)S, g.ldn, g.ldn, lp_part, nullptr, ones, G, Gt,
      St, g.ldB, db2_part, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  bwd_hidden_kernel<T><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(G, g.ldn, (const T*)m.Pt, m.c, m.n, m.h, B, Rt, Dt,
                                                             g.ldB, db1_part, g.ldh);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the direction in the kernels' layouts
  if ((e = launch_cast(m.n, m.h, gP, m.wdtype, gPw, gPtw, st)) != hipSuccess) return e;
  // U = gb2 + R (masked gW2)^T
  fwd_out_kernel<T, 0><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(
      R, g.ldh, gPw, gb2, m.c, m.n, m.h, B, (int8_t*)S, g.ldn, g.ldn, lp_part, U, nullptr, nullptr, nullptr,
      nullptr, g.ldB, nullptr, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // V = gb1 + S (masked gW1)^T without the ReLU, batch-contiguous in the Rt slot (R no longer needed)
  fwd_hidden_kernel<T, true, false><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, gPtw, g.ldn, gb1, m.c, m.n,
                                                                           m.h, B, R, g.ldh, Rt, g.ldB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sr_jvp_dot_kernel<T><<<(unsigned)((B + 3) / 4), 256, 0, st>>>(G, U, g.ldn, m.n, Dt, Rt, g.ldB, m.h, B, v);
  return hipGetLastError();
}

hipError_t launch_sr_jvp(const vqmc_made& m, const int8_t* S, int64_t B, const float* gP, const float* gb1,
                         const float* gb2, float* v, void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return sr_jvp_t<bf16_t>(m, S, B, gP, gb1, gb2, v, ws, st);
  return sr_jvp_t<float>(m, S, B, gP, gb1, gb2, v, ws, st);
}

// Backward from the incremental sampler's byproducts: Rt (relu(A), batch-contiguous, in
// the workspace's Rt slot) and Zs (s_d z_d): the two forward products are not recomputed.
template <typename T>
static hipError_t backward_sampled_t(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                                     const float* Zs, const T* Rt, float* dP, float* db1, float* db2, void* ws,
                                     void* Pm, hipStream_t st) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 1);
  uint8_t* w = (uint8_t*)ws;
  T* G = (T*)(w + L.G);
  T* Gt = (T*)(w + L.Gt);
  T* St = (T*)(w + L.St);
  T* Dt = (T*)(w + L.Dt);
  float* db2_part = (float*)(w + L.db2_part);
  float* db1_part = (float*)(w + L.db1_part);
  hipError_t e;
  grad_out_kernel<T><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(Zs, S, g.ldn, coef, m.n, B, G, Gt, St, g.ldB, db2_part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if constexpr (sizeof(T) == 2) {
    // BF16: the direct-to-LDS engine, the adjoint's mask on a masked copy of P^T
    // the masked copy of P^T comes with the sampler tables when there are any
    bool ready = false;
    if (m.band) {
      int64_t zo, uo, po;
      int nzt, nut;
      sample_tables_layout(m.n, m.h, m.wdtype, &zo, &uo, &po, &nzt, &nut);
      Pm = (uint8_t*)m.band + po;
      ready = true;
    }
    // (the weight-gradient launch also sums the bias-gradient partials)
    return launch_backward_products2(m, B, G, Gt, St, Rt, Dt, (bf16_t*)Pm, db1_part, g.mt_h, db2_part, g.mt_o, dP,
                                     db1, db2, st, ready);
  } else {
    bwd_hidden_kernel<T><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(G, g.ldn, (const T*)m.Pt, m.c, m.n, m.h, B, Rt, Dt,
                                                               g.ldB, db1_part, g.ldh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bwd_weight_kernel<T, false><<<dim3(g.nt_w, g.mt_w), 256, 0, st>>>(Gt, Rt, g.ldB, m.c, m.n, m.h, dP);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bwd_weight_kernel<T, true><<<dim3(g.nt_w, g.mt_w), 256, 0, st>>>(St, Dt, g.ldB, m.c, m.n, m.h, dP);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  sum_rows_kernel<<<(unsigned)((m.n + 255) / 256), 256, 0, st>>>(db2_part, g.mt_o, g.ldn, m.n, db2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_rows_kernel<<<(unsigned)((m.h + 255) / 256), 256, 0, st>>>(db1_part, g.mt_h, g.ldh, m.h, db1);
  return hipGetLastError();
}

void* backward_rt_slot(const vqmc_made& m, int64_t B, void* ws) {
  return (uint8_t*)ws + layout(m.n, m.h, B, m.wdtype, 1).Rt;
}

hipError_t launch_backward_sampled(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                                   const float* Zs, const void* Rt, float* dP, float* db1, float* db2, void* ws,
                                   void* Pm, hipStream_t st) {
  if (m.wdtype == VQMC_BF16)
    return backward_sampled_t<bf16_t>(m, S, B, coef, Zs, (const bf16_t*)Rt, dP, db1, db2, ws, Pm, st);
  return backward_sampled_t<float>(m, S, B, coef, Zs, (const float*)Rt, dP, db1, db2, ws, Pm, st);
}

template <typename T>
static hipError_t sample_plain_t(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                                 int64_t offset, uint32_t tag, int8_t* S, float* logp, void* ws,
                                 hipStream_t st) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 2);
  uint8_t* w = (uint8_t*)ws;
  T* R = (T*)(w + L.R);
  float* lp_acc = (float*)(w + L.lp_acc);
  hipError_t e;
  // Algorithm 1's initial state: unsampled sites are never read (masks); start from 0.
  fill_i8_kernel<<<(unsigned)((B * g.ldn + 255) / 256), 256, 0, st>>>(S, B * g.ldn);
  fill_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(lp_acc, B, 0.f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int d = 0; d < m.n; ++d) {
    // forward pass d over the partially drawn batch ...
    fwd_hidden_kernel<T, false><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, (const T*)m.Pt, g.ldn, m.b1,
                                                                       m.c, m.n, m.h, B, R, g.ldh, nullptr,
                                                                       g.ldB);
    // ... then the output layer for the tile holding site d, and the draw of s_d
    fwd_out_kernel<T, 2><<<dim3(1, g.mt_o), 256, 0, st>>>(R, g.ldh, (const T*)m.P, m.b2, m.c, m.n, m.h, B, S,
                                                          g.ldn, g.ldn, nullptr, nullptr, nullptr, nullptr,
                                                          nullptr, nullptr, g.ldB, nullptr, d, seed, step,
                                                          offset, tag, lp_acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (logp) return hipMemcpyAsync(logp, lp_acc, (size_t)B * 4, hipMemcpyDeviceToDevice, st);
  return hipSuccess;
}

// The forward quantities of the TIM single-flip differences: logits Z (B x ldn) and the FP32
// pre-activations A (B x ldh); ws holds the log p forward region (R, lp_part).
template <typename T>
static hipError_t tim_forward_t(const vqmc_made& m, const int8_t* S, int64_t B, float* Z, float* A, void* ws,
                                hipStream_t st) {
  const Geom g = geom(m.n, m.h, B);
  const WsLayout L = layout(m.n, m.h, B, m.wdtype, 0);
  uint8_t* w = (uint8_t*)ws;
  T* R = (T*)(w + L.R);
  float* lp_part = (float*)(w + L.lp_part);
  fwd_hidden_kernel<T, false><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(S, g.ldn, (const T*)m.Pt, g.ldn, m.b1, m.c, m.n,
                                                                     m.h, B, R, g.ldh, nullptr, g.ldB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fwd_out_kernel<T, 0><<<dim3(g.nt_o, g.mt_o), 256, 0, st>>>(
      R, g.ldh, (const T*)m.P, m.b2, m.c, m.n, m.h, B, (int8_t*)S, g.ldn, g.ldn, lp_part, Z, nullptr, nullptr,
      nullptr, nullptr, g.ldB, nullptr, 0, 0, 0, 0, 0, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fwd_hidden_kernel<T, false, false, float><<<dim3(g.nt_h, g.mt_h), 256, 0, st>>>(
      S, g.ldn, (const T*)m.Pt, g.ldn, m.b1, m.c, m.n, m.h, B, A, g.ldh, (T*)nullptr, g.ldB);
  return hipGetLastError();
}

hipError_t launch_tim_forward(const vqmc_made& m, const int8_t* S, int64_t B, float* Z, float* A, void* ws,
                              hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return tim_forward_t<bf16_t>(m, S, B, Z, A, ws, st);
  return tim_forward_t<float>(m, S, B, Z, A, ws, st);
}

hipError_t launch_logprob(const vqmc_made& m, const int8_t* S, int64_t B, float* logp, float* Z,
                          void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return logprob_t<bf16_t>(m, S, B, logp, Z, ws, st);
  return logprob_t<float>(m, S, B, logp, Z, ws, st);
}

hipError_t launch_backward(const vqmc_made& m, const int8_t* S, int64_t B, const float* coef,
                           float* dP, float* db1, float* db2, void* ws, hipStream_t st, hipEvent_t coef_ready) {
  if (m.wdtype == VQMC_BF16) return backward_t<bf16_t>(m, S, B, coef, dP, db1, db2, ws, st, coef_ready);
  return backward_t<float>(m, S, B, coef, dP, db1, db2, ws, st, coef_ready);
}

hipError_t launch_sample_plain(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step,
                               int64_t offset, uint32_t tag, int8_t* S, float* logp, void* ws,
                               hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return sample_plain_t<bf16_t>(m, B, seed, step, offset, tag, S, logp, ws, st);
  return sample_plain_t<float>(m, B, seed, step, offset, tag, S, logp, ws, st);
}

}  // namespace vqmc
