// Diagonal local energy and batch statistics.
//
// Local energy (Sec. 2.1): l(x) = (H psi)(x) / psi(x), which for a diagonal H
// (alpha_i = 0 in eq. hamiltonian) is H_xx = sum_{i<j} J_ij s_i s_j with beta_i = 0.
// Statistics (Sec. 2.1, eq. stochastic_variance and the gradient population form):
// mean, population variance, min/argmin and baseline coefficients c_b = (E_b - mean)/B.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <type_traits>

namespace vqmc {

// ---------------------------------------------------------------- sparse (CSR upper)
// One workgroup of 1024 threads handles EMSE samples.  Their spins are staged in LDS as
// one byte per site (bit q = [s_q = +1]), so an edge costs one byte read for all samples,
// and so is the row pointer (int32) when it fits.  Thread t walks rows i = t, t + 1024,
// ..., two edges per step with their loads issued together.  Row i of the upper triangle
// contributes
//   s_iq sum_j w_ij s_jq = s_iq (2 Y_q - W_i),  Y_q = sum_j w_ij [s_jq = +1],  W_i = sum_j w_ij,
// accumulated exactly in int64 (integer weights) or in double (float weights, whose sums
// of exact terms only differ from the oracle's by summation order).  A fixed thread -> row
// map and fixed-shape reductions make the result deterministic.
constexpr int EMSE = 8;
constexpr int EB_THREADS = 1024;
template <typename WT, typename AT, bool RP_LDS>
__global__ __launch_bounds__(EB_THREADS) void energy_csr_bits_kernel(int n, int64_t lds,
                                                                    const int64_t* __restrict__ rowptr,
                                                                    const int32_t* __restrict__ col,
                                                                    const WT* __restrict__ w,
                                                                    const int8_t* __restrict__ S, int64_t B,
                                                                    int nst, AT* __restrict__ E) {
  // nst bytes of site bits, then the row pointer (n + 1 int32, if staged), then scratch
  extern __shared__ __attribute__((aligned(16))) uint8_t shb[];
  uint8_t* bits = shb;
  int32_t* rp = (int32_t*)(shb + nst);
  AT* red = (AT*)(shb + nst + (RP_LDS ? round_up((int64_t)(n + 1) * 4, 16) : 0));
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * EMSE;
  const int nq = (int)min<int64_t>(EMSE, B - b0);
  // nst = round_up(n, 16) <= lds: every 16-byte chunk lies inside the padded row.  The
  // spins are +1 = 0x01 and -1 = 0xFF: bit 7 of a byte is clear exactly for +1 (the row
  // padding, 0, also reads +1 and is never referenced).
  for (int c0 = t; c0 < nst / 16; c0 += EB_THREADS) {
    uint32_t a[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < EMSE; ++q) {
      if (q < nq) {
        const uint4 v = *(const uint4*)(S + (b0 + q) * lds + 16 * c0);
        a[0] |= ((~v.x >> 7) & 0x01010101u) << q;
        a[1] |= ((~v.y >> 7) & 0x01010101u) << q;
        a[2] |= ((~v.z >> 7) & 0x01010101u) << q;
        a[3] |= ((~v.w >> 7) & 0x01010101u) << q;
      }
    }
    *(uint4*)(bits + 16 * c0) = make_uint4(a[0], a[1], a[2], a[3]);
  }
  if constexpr (RP_LDS)
    for (int i = t; i <= n; i += EB_THREADS) rp[i] = (int32_t)rowptr[i];
  __syncthreads();
  auto rowp = [&](int i) -> int64_t {
    if constexpr (RP_LDS) return rp[i];
    else return rowptr[i];
  };
  AT acc[EMSE];
#pragma unroll
  for (int q = 0; q < EMSE; ++q) acc[q] = 0;
  // row sums Y: int32 for integer weights while the row's sum of |w| fits (then no partial
  // sum can overflow; a row beyond that is summed again in int64), else AT
  constexpr bool INT = std::is_integral<WT>::value;
  typedef typename std::conditional<INT, int32_t, AT>::type RT;
  for (int i = t; i < n; i += EB_THREADS) {
    const int64_t e0 = rowp(i), e1 = rowp(i + 1);
    RT y[EMSE];
#pragma unroll
    for (int q = 0; q < EMSE; ++q) y[q] = 0;
    AT wsum = 0;
    int64_t wabs = 0;
    int64_t e = e0;
    for (; e + 1 < e1; e += 2) {  // two edges per step: their loads are issued together
      const int j0 = col[e], j1 = col[e + 1];
      const RT w0 = (RT)w[e], w1 = (RT)w[e + 1];
      const uint32_t m0 = bits[j0], m1 = bits[j1];
      wsum += (AT)w0 + (AT)w1;
      if constexpr (INT) wabs += llabs((int64_t)w0) + llabs((int64_t)w1);
#pragma unroll
      for (int q = 0; q < EMSE; ++q) y[q] += (((m0 >> q) & 1u) ? w0 : (RT)0) + (((m1 >> q) & 1u) ? w1 : (RT)0);
    }
    if (e < e1) {
      const RT w0 = (RT)w[e];
      const uint32_t m0 = bits[col[e]];
      wsum += (AT)w0;
      if constexpr (INT) wabs += llabs((int64_t)w0);
#pragma unroll
      for (int q = 0; q < EMSE; ++q) y[q] += ((m0 >> q) & 1u) ? w0 : (RT)0;
    }
    AT ya[EMSE];
#pragma unroll
    for (int q = 0; q < EMSE; ++q) ya[q] = (AT)y[q];
    if (INT && wabs > (int64_t)INT32_MAX) {
#pragma unroll
      for (int q = 0; q < EMSE; ++q) ya[q] = 0;
      for (int64_t f = e0; f < e1; ++f) {
        const AT wf = (AT)w[f];
        const uint32_t mf = bits[col[f]];
#pragma unroll
        for (int q = 0; q < EMSE; ++q) ya[q] += ((mf >> q) & 1u) ? wf : (AT)0;
      }
    }
    const uint32_t mi = bits[i];
#pragma unroll
    for (int q = 0; q < EMSE; ++q) {
      const AT r = 2 * ya[q] - wsum;
      acc[q] += ((mi >> q) & 1u) ? r : -r;
    }
  }
  // per sample: fixed butterfly over the wave, then the sixteen waves in order
  constexpr int NW = EB_THREADS / 64;
#pragma unroll
  for (int q = 0; q < EMSE; ++q) {
    AT v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[q * NW + wv] = v;
  }
  __syncthreads();
  if (t < nq) {
    AT s = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[t * NW + k];
    E[b0 + t] = s;
  }
}

// ---------------------------------------------------------------- sparse, byte lanes
// Integer weights, same rows and sums as above, with each site staged as eight bytes (byte q =
// [s_q = +1]) instead of eight bits: then w * site adds w to all eight samples' row sums Y_q at
// once, each in its own byte, as two 32-bit multiply-adds per edge.  A byte holds Y_q exactly
// while the row's weights are non-negative and sum to at most 255 (every Max-Cut graph with
// small integer weights); a row outside that range is summed again sample by sample.
template <bool RP_LDS>
__global__ __launch_bounds__(EB_THREADS) void energy_csr_bytes_kernel(int n, int64_t lds,
                                                                     const int64_t* __restrict__ rowptr,
                                                                     const int32_t* __restrict__ col,
                                                                     const int32_t* __restrict__ w,
                                                                     const int8_t* __restrict__ S, int64_t B,
                                                                     int nsp, int64_t* __restrict__ E) {
  // nsp uint2 site words (n rounded up to 16), then the row pointer (n + 1 int32, if staged),
  // then scratch
  extern __shared__ __attribute__((aligned(16))) uint8_t shb[];
  uint2* sw = (uint2*)shb;
  int32_t* rp = (int32_t*)(shb + (size_t)nsp * 8);
  int64_t* red = (int64_t*)(shb + (size_t)nsp * 8 + (RP_LDS ? round_up((int64_t)(n + 1) * 4, 16) : 0));
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * EMSE;
  const int nq = (int)min<int64_t>(EMSE, B - b0);
  // sixteen sites per item: one 16-byte piece of each sample's row (inside the padded row),
  // gathered into a bit per sample, then spread to a byte per sample
  for (int c0 = t; c0 < nsp / 16; c0 += EB_THREADS) {
    uint32_t a[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < EMSE; ++q) {
      if (q < nq) {
        const uint4 v = *(const uint4*)(S + (b0 + q) * lds + 16 * c0);
        a[0] |= ((~v.x >> 7) & 0x01010101u) << q;
        a[1] |= ((~v.y >> 7) & 0x01010101u) << q;
        a[2] |= ((~v.z >> 7) & 0x01010101u) << q;
        a[3] |= ((~v.w >> 7) & 0x01010101u) << q;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t m = (a[e >> 2] >> (8 * (e & 3))) & 0xFFu;
      // bit k of a 4-bit value to bit 8k: the four shifted copies (x 1, 2^7, 2^14, 2^21) do not
      // overlap, so the product carries nothing
      sw[16 * c0 + e] = make_uint2(((m & 0xFu) * 0x00204081u) & 0x01010101u, ((m >> 4) * 0x00204081u) & 0x01010101u);
    }
  }
  if constexpr (RP_LDS)
    for (int i = t; i <= n; i += EB_THREADS) rp[i] = (int32_t)rowptr[i];
  __syncthreads();
  auto rowp = [&](int i) -> int64_t {
    if constexpr (RP_LDS) return rp[i];
    else return rowptr[i];
  };
  int64_t acc[EMSE];
#pragma unroll
  for (int q = 0; q < EMSE; ++q) acc[q] = 0;
  for (int i = t; i < n; i += EB_THREADS) {
    const int64_t e0 = rowp(i), e1 = rowp(i + 1);
    uint32_t ylo = 0u, yhi = 0u;  // Y_q in byte q (q < 4 in ylo)
    int64_t wsum = 0;
    bool small = true;
    int64_t e = e0;
    for (; e + 1 < e1; e += 2) {  // two edges per step: their loads are issued together
      const int j0 = col[e], j1 = col[e + 1];
      const int32_t w0 = w[e], w1 = w[e + 1];
      const uint2 s0 = sw[j0], s1 = sw[j1];
      wsum += (int64_t)w0 + (int64_t)w1;
      small = small && (uint32_t)w0 <= 255u && (uint32_t)w1 <= 255u;
      ylo += (uint32_t)w0 * s0.x + (uint32_t)w1 * s1.x;
      yhi += (uint32_t)w0 * s0.y + (uint32_t)w1 * s1.y;
    }
    if (e < e1) {
      const int32_t w0 = w[e];
      const uint2 s0 = sw[col[e]];
      wsum += (int64_t)w0;
      small = small && (uint32_t)w0 <= 255u;
      ylo += (uint32_t)w0 * s0.x;
      yhi += (uint32_t)w0 * s0.y;
    }
    int64_t ya[EMSE];
    if (small && wsum <= 255) {
#pragma unroll
      for (int q = 0; q < EMSE; ++q) ya[q] = (int64_t)(((q < 4 ? ylo : yhi) >> (8 * (q & 3))) & 0xFFu);
    } else {  // the row again, one int64 sum per sample
#pragma unroll
      for (int q = 0; q < EMSE; ++q) ya[q] = 0;
      for (int64_t f = e0; f < e1; ++f) {
        const int64_t wf = w[f];
        const uint2 sf = sw[col[f]];
#pragma unroll
        for (int q = 0; q < EMSE; ++q) ya[q] += (((q < 4 ? sf.x : sf.y) >> (8 * (q & 3))) & 1u) ? wf : 0;
      }
    }
    const uint2 si = sw[i];
#pragma unroll
    for (int q = 0; q < EMSE; ++q) {
      const int64_t r = 2 * ya[q] - wsum;
      acc[q] += (((q < 4 ? si.x : si.y) >> (8 * (q & 3))) & 1u) ? r : -r;
    }
  }
  // per sample: fixed butterfly over the wave, then the sixteen waves in order
  constexpr int NW = EB_THREADS / 64;
#pragma unroll
  for (int q = 0; q < EMSE; ++q) {
    int64_t v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[q * NW + wv] = v;
  }
  __syncthreads();
  if (t < nq) {
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[t * NW + k];
    E[b0 + t] = s;
  }
}

// ---------------------------------------------------------------- dense J (FP64)
// E_b = sum_i s_bi * y_bi with y_bi = sum_{j>i} J_ij s_bj (strict upper triangle only).
// Tile: 64 samples x 64 rows i per workgroup, K loop over j >= i0 in chunks of 32,
// FP64 MFMA 16x16x4 on exact operands (+-1 and float32 J widened to double).
// Each workgroup writes one partial per sample; a second pass sums the partials of
// the row tiles in a fixed order.
constexpr int DT = 64, DK = 32;
constexpr int DKT = DK / 4;  // stage columns per thread (4 threads per row)
__global__ __launch_bounds__(256) void energy_dense_kernel(int n, int64_t lds, const float* __restrict__ J,
                                                            const int8_t* __restrict__ S, int64_t B,
                                                            double* __restrict__ part) {
  __shared__ double Ss[DT][DK + 1];
  __shared__ double Js[DT][DK + 1];
  __shared__ double rowsum[2][DT];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;  // wave sub-tile: samples x rows
  const int64_t m0 = (int64_t)blockIdx.y * DT;          // samples
  const int i0 = blockIdx.x * DT;                       // rows i
  doublex4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (doublex4_t){0, 0, 0, 0};
  const int jbeg = (i0 / DK) * DK;
  // stage: 64 rows x DK columns of each operand, DKT elements per thread.  The next stage's
  // values are loaded into registers before the current stage is multiplied, so the loads
  // overlap the products.
  const int r = t >> 2, q = (t & 3) * DKT;
  const int64_t bq = m0 + r;
  const int iq = i0 + r;
  uint2 sv = make_uint2(0u, 0u);  // DKT = 8 spins (int8), columns j0 + q .. (inside the padded row)
  float jv[DKT];
  const bool vec = (n & 3) == 0 && ((uintptr_t)J & 15) == 0;  // rows of J start 16-byte aligned
  auto fetch = [&](int j0) {
    sv = (bq < B) ? *(const uint2*)(S + bq * lds + j0 + q) : make_uint2(0u, 0u);
    const int jq = j0 + q;
    if (vec && iq < n && jq + DKT <= n) {  // eight columns inside the row: two 16-byte loads
      const float4 a0 = *(const float4*)(J + (int64_t)iq * n + jq), a1 = *(const float4*)(J + (int64_t)iq * n + jq + 4);
      const float v8[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
      for (int e = 0; e < DKT; ++e) jv[e] = (jq + e > iq) ? v8[e] : 0.f;
    } else {
#pragma unroll
      for (int e = 0; e < DKT; ++e) {
        const int j = jq + e;
        jv[e] = (iq < n && j < n && j > iq) ? J[(int64_t)iq * n + j] : 0.f;
      }
    }
  };
  static_assert(DKT == 8, "the spin fetch reads eight bytes");
  fetch(jbeg);
  for (int j0 = jbeg; j0 < n; j0 += DK) {
#pragma unroll
    for (int e = 0; e < DKT; ++e) {
      const uint32_t w = (e < 4) ? sv.x : sv.y;
      Ss[r][q + e] = (j0 + q + e < n) ? (double)(int8_t)(w >> (8 * (e & 3))) : 0.0;
      Js[r][q + e] = (double)jv[e];
    }
    __syncthreads();
    if (j0 + DK < n) fetch(j0 + DK);
#pragma unroll
    for (int kk = 0; kk < DK; kk += 4) {
      double a[2], bb[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) a[mi] = Ss[wm + mi * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) bb[ni] = Js[wn + ni * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], bb[ni], acc[mi][ni], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: the FP64 MFMA accumulator layout puts element e of lane l at row
  // 4*e + l/16, column l%16 (unlike the FP32 16x16 layout, row 4*(l/16) + e);
  // multiply by s_bi and sum over i.
  double ps[2][4];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double v = 0.0;
      const int64_t b = m0 + wm + mi * 16 + 4 * e + (lane >> 4);
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const int i = i0 + wn + ni * 16 + (lane & 15);
        const double si = (b < B && i < n) ? (double)S[b * lds + i] : 0.0;
        v += si * acc[mi][ni][e];
      }
      ps[mi][e] = v;
    }
  // reduce over the 16 lanes of a row (lane & 15) with a fixed butterfly
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double v = ps[mi][e];
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
      ps[mi][e] = v;
    }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int e = 0; e < 4; ++e) rowsum[wn >> 5][wm + mi * 16 + 4 * e + (lane >> 4)] = ps[mi][e];
  }
  __syncthreads();
  if (t < DT) {
    const int64_t b = m0 + t;
    if (b < B) part[(int64_t)blockIdx.x * B + b] = rowsum[0][t] + rowsum[1][t];
  }
}

__global__ void sum_partials_kernel(const double* __restrict__ part, int ntiles, int64_t B,
                                    double* __restrict__ E) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int tt = 0; tt < ntiles; ++tt) s += part[(int64_t)tt * B + b];
  E[b] = s;
}

size_t energy_workspace_bytes(const vqmc_hamiltonian& H, int64_t B) {
  if (H.kind != VQMC_H_DENSE_F32) return 0;
  const int64_t ntiles = (H.n + DT - 1) / DT;
  return (size_t)(ntiles * B * sizeof(double));
}

hipError_t launch_energy(const vqmc_hamiltonian& H, const int8_t* S, int64_t B, void* E, void* ws,
                         hipStream_t st) {
  const int n = H.n;
  const int64_t lds = round_up(n, kPad);
  if (H.kind == VQMC_H_DENSE_F32) {
    const int ntiles = (n + DT - 1) / DT;
    dim3 grid(ntiles, (unsigned)((B + DT - 1) / DT));
    energy_dense_kernel<<<grid, 256, 0, st>>>(n, lds, H.J, S, B, (double*)ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_partials_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>((const double*)ws, ntiles, B,
                                                                       (double*)E);
    return hipGetLastError();
  }
  const int nst = (int)round_up(n, 16);
  // site bytes and reduction scratch always in LDS; the row pointer too when two
  // workgroups still fit on a CU
  const size_t rpb = (size_t)round_up((int64_t)(n + 1) * 4, 16);
  const size_t redb = (size_t)EMSE * (EB_THREADS / 64) * 8;
  const bool rp_lds = H.nnz < (int64_t)1 << 31 && (size_t)nst + rpb + redb <= 64 * 1024;
  const size_t shbytes = (size_t)nst + (rp_lds ? rpb : 0) + redb;
  const unsigned grid = (unsigned)((B + EMSE - 1) / EMSE);
  hipError_t e;
  auto go = [&](auto kern, auto wptr, auto eptr) {
    e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shbytes);
    if (e != hipSuccess) return;
    kern<<<grid, EB_THREADS, shbytes, st>>>(n, lds, H.rowptr, H.col, wptr, S, B, nst, eptr);
    e = hipGetLastError();
  };
  if (H.kind == VQMC_H_CSR_INT) {
    // byte lanes when the site words fit in one CU's LDS (the row pointer too if it fits)
    const size_t swb = (size_t)nst * 8;
    if (H.nnz < (int64_t)1 << 31 && swb + redb <= 160 * 1024) {
      const bool rpl = swb + rpb + redb <= 160 * 1024;
      const size_t sb = swb + (rpl ? rpb : 0) + redb;
      auto kern = rpl ? energy_csr_bytes_kernel<true> : energy_csr_bytes_kernel<false>;
      if ((e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sb)) !=
          hipSuccess)
        return e;
      kern<<<grid, EB_THREADS, sb, st>>>(n, lds, H.rowptr, H.col, (const int32_t*)H.w, S, B, nst, (int64_t*)E);
      return hipGetLastError();
    }
    if (rp_lds) go(energy_csr_bits_kernel<int32_t, int64_t, true>, (const int32_t*)H.w, (int64_t*)E);
    else go(energy_csr_bits_kernel<int32_t, int64_t, false>, (const int32_t*)H.w, (int64_t*)E);
  } else {
    if (rp_lds) go(energy_csr_bits_kernel<float, double, true>, (const float*)H.w, (double*)E);
    else go(energy_csr_bits_kernel<float, double, false>, (const float*)H.w, (double*)E);
  }
  return e;
}

// ---------------------------------------------------------------- statistics
// One workgroup of 1024 threads; every reduction has a fixed shape, so the result is
// bit-reproducible.  int64 energies are summed exactly before the single division.
template <typename ET>
__global__ __launch_bounds__(1024) void stats_kernel(const ET* __restrict__ E, int64_t B,
                                                      vqmc_stats* __restrict__ out,
                                                      float* __restrict__ coef) {
  constexpr int NW = 1024 / 64;
  __shared__ ET wsum[NW];
  __shared__ ET wmin[NW];
  __shared__ int64_t warg[NW];
  __shared__ double wsd[NW];
  __shared__ double s_mean;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  ET s = 0;
  ET mn = 0;
  int64_t am = -1;
  for (int64_t b = t; b < B; b += 1024) {
    const ET v = E[b];
    s += v;
    if (am < 0 || v < mn) {
      mn = v;
      am = b;
    }
  }
  // butterflies over the wave (lane 0's result is used), then the sixteen waves in order
  auto better = [](ET m1, int64_t a1, ET m0, int64_t a0) {  // (m1, a1) replaces (m0, a0)
    return a1 >= 0 && (a0 < 0 || m1 < m0 || (m1 == m0 && a1 < a0));
  };
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o);
    const ET mo = __shfl_xor(mn, o);
    const int64_t ao = __shfl_xor(am, o);
    if (better(mo, ao, mn, am)) {
      mn = mo;
      am = ao;
    }
  }
  if (lane == 0) {
    wsum[wv] = s;
    wmin[wv] = mn;
    warg[wv] = am;
  }
  __syncthreads();
  if (t == 0) {
    ET ts = wsum[0], tm = wmin[0];
    int64_t ta = warg[0];
    for (int k = 1; k < NW; ++k) {
      ts += wsum[k];
      if (better(wmin[k], warg[k], tm, ta)) {
        tm = wmin[k];
        ta = warg[k];
      }
    }
    s_mean = (double)ts / (double)B;
    out->mean_E = s_mean;
    out->min_E = (double)tm;
    out->argmin = ta;
    out->sum_E = (double)ts;
  }
  __syncthreads();
  const double mean = s_mean;
  double v2 = 0.0;
  for (int64_t b = t; b < B; b += 1024) {
    const double dv = (double)E[b] - mean;
    v2 += dv * dv;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v2 += __shfl_xor(v2, o);
  if (lane == 0) wsd[wv] = v2;
  __syncthreads();
  if (t == 0) {
    double tv = wsd[0];
    for (int k = 1; k < NW; ++k) tv += wsd[k];
    out->var_E = tv / (double)B;
  }
  if (coef)
    for (int64_t b = t; b < B; b += 1024) coef[b] = (float)(((double)E[b] - mean) / (double)B);
}

hipError_t launch_stats(const void* E, int e_is_int, int64_t B, vqmc_stats* stats, float* coef,
                        hipStream_t st) {
  if (e_is_int)
    stats_kernel<int64_t><<<1, 1024, 0, st>>>((const int64_t*)E, B, stats, coef);
  else
    stats_kernel<double><<<1, 1024, 0, st>>>((const double*)E, B, stats, coef);
  return hipGetLastError();
}

}  // namespace vqmc
