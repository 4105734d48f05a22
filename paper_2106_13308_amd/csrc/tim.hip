// Local energy of the transverse-field Ising model (TIM) for a MADE trial state.
//
// eq. (hamiltonian) with the TIM couplings of eq. (e:tim): in the basis of spin strings s the
// matrix has the diagonal entry H_ss = -sum_i beta_i s_i - sum_{i<j} beta_ij s_i s_j and, for
// each site i, the off-diagonal entry -alpha_i between s and s^(i) (s with site i negated).
// With the non-negative trial state psi = sqrt(pi) of Sec. 2.3, the local energy of Sec. 2.1 is
//
//     l(s) = H_ss - sum_i alpha_i exp(D_i / 2),   D_i = log pi(s^(i)) - log pi(s).
//
// D_i is where the work is: the paper evaluates it with one forward pass per flipped string
// (n passes per sample, Sec. 4 cost model).  Here every D_i of a sample comes from the state
// of one forward pass.  Flipping site i leaves every conditional before i unchanged, adds
// -2 s_i W1[k][i] to the pre-activation a_k of each unit k that receives site i (k >= c[i]),
// and so changes the logit of every later site d by
//
//     dz[i][d] = sum_{c[i] <= k < c[d]} W2[d][k] dR[i][k],   dR[i][k] = relu(a_k - 2 s_i W1[k][i]) - relu(a_k),
//
// a product of the n x h matrix dR (one per sample) with the masked second layer: a dense
// contraction, run on MFMA.  Then, with t_d = s_d z_d,
//
//     D_i = -t_i + sum_{d > i} [log sigma(t_d + s_d dz[i][d]) - log sigma(t_d)].
//
// The sum is fused into the product's epilogue.  Each difference of log-sigmoids is
// [min(u,0) - min(t,0)] - log1p(x), u = t + s dz, x = (e^-|u| - e^-|t|) / (1 + e^-|t|), the form
// without cancellation between the two terms (x is 0 when dz is 0); the log1p terms of a row
// are collected as a running product of w = fl(1 + x) plus the sum of the rounding errors
// x - (w - 1) (log(1 + x) = log w + (x - (w - 1)) / w, the second factor taken as 1: its error
// is below one ulp of the term), so an element costs one exponential and no logarithm.
//
// Workgroup = (block of 64 flipped sites, one sample), 4 waves.  The block's dR rows (K from
// the first unit any of its sites feeds to h) are built once into LDS; the workgroup then sweeps
// the 128-site blocks d from the one holding its first site to the last, each wave taking 32
// columns d in two groups of 16: A fragments from LDS, each used by both groups, B fragments (rows
// of the masked second layer) from global memory, 8 MFMA blocks of 16 x 16 per K step.  Elements
// with d <= i contribute exactly 0 (their dz is an exact 0), so the diagonal blocks need no mask.  Workgroups are numbered block-major: the ones that run together
// on an XCD share their flip block and so stream the same rows of the second layer through that
// XCD's L2, and the longest sweeps (the first blocks) start first.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int TIM_BM = 64;       // flipped sites per workgroup
constexpr int TIM_BN = 128;      // sites d per block of the sweep: 32 per wave, two groups of 16
constexpr int TIM_RENORM = 32;   // site blocks between renormalisations of the running products
                                 // (64 factors in (1/2, 2) each: far inside the float range)
constexpr float TIM_L2E = 1.4426950408889634f;   // log2(e)
constexpr float TIM_LN2 = 0.6931471805599453f;   // ln(2)

template <typename T>
struct TimK {
  static constexpr int KS = sizeof(T) == 2 ? 32 : 4;  // K of one MFMA step
};

// LDS row stride of dR in elements: at least kw, rows 16 bytes apart modulo 256 bytes (BF16) /
// 4 floats apart modulo 64 (F32), so the 16 rows of one fragment read fall in distinct banks.
template <typename T>
__host__ __device__ constexpr int tim_ldr(int kw) {
  return sizeof(T) == 2 ? (kw - 8 + 127) / 128 * 128 + 8 : (kw - 4 + 63) / 64 * 64 + 4;
}

// dR holds K columns [kbase, kbase + kw) of the block's rows, kw <= kalloc (the plain sweep:
// round_up(h, KS); the pipelined one: 32 NF, so that its row stride is a compile-time constant)
template <typename T>
__host__ __device__ inline size_t tim_lds_bytes(int h, int kalloc) {
  return (size_t)TIM_BM * tim_ldr<T>(kalloc) * sizeof(T) + (size_t)round_up(h, 32) * 4 + 4 * TIM_BM * 4 +
         TIM_BM * 8;
}

// P2[d][k] = W2[d][k] = P[d][k] where unit k feeds site d (k < c[d]), else 0; n x ldh.
template <typename T>
__global__ void tim_w2_kernel(const T* __restrict__ P, const int32_t* __restrict__ c, int n, int64_t ldh,
                              T* __restrict__ P2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * ldh) return;
  const int64_t d = idx / ldh, k = idx - d * ldh;
  P2[idx] = (k < c[d]) ? P[idx] : (T)0;
}

// One site block's contribution for this lane: acc[mi][r] is dz for row 16 mi + 4 (lane >> 4) + r
// and the lane's column (spin sd, t = sd z_d, p = e^-|t|, rd = 1 / (1 + p), nmt = -min(t, 0)).
//   lin  += min(u, 0) - min(t, 0), as (u - |u|) / 2 - min(t, 0) (exactly 0 when dz is 0)
//   prod *= 1 + x, x = (e^-|u| - p) rd, one rounding per element (x is exactly 0 when dz is 0)
__device__ inline void tim_epilogue(const floatx4_t (&acc)[4], float sd, float td, float pd, float rd, float nmt,
                                    float (&lin)[4][4], float (&prod)[4][4]) {
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float u = fmaf(sd, acc[mi][r], td);
      lin[mi][r] += fmaf(u - fabsf(u), 0.5f, nmt);
      const float e = __builtin_amdgcn_exp2f(-fabsf(u) * TIM_L2E);
      prod[mi][r] = fmaf(prod[mi][r], (e - pd) * rd, prod[mi][r]);
    }
}

// Raw buffer loads of the masked second layer: base and size in scalar registers, the lane's byte
// offset in a vector register.  An offset at or past the size reads zeros without touching
// memory, so the sweep issues the same loads on every path (fixed wait counts) and fetches
// only the K steps a block needs.
typedef __amdgpu_buffer_rsrc_t tim_rsrc_t;
constexpr uint32_t TIM_OOB = 0x7FFFFF00u;
__device__ inline tim_rsrc_t tim_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, (int)bytes, 0x00020000);
}
// voff: the lane's byte offset (or TIM_OOB), soff: a uniform byte offset added after it
__device__ inline uint4 tim_ld16(tim_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}

// dR rows of the flip block, the per-lane running sums, and the final reduction are shared by
// both sweeps below; NF > 0 selects the pipelined BF16 sweep (register-prefetched operands),
// NF = 0 the plain one (FP32 weights, or K ranges too long to prefetch).
template <typename T, int NF>
__global__ __launch_bounds__(256) void tim_flip_kernel(
    const int8_t* __restrict__ S, int64_t lds, const float* __restrict__ A, int64_t ldh,
    const float* __restrict__ Z, int64_t ldz, const T* __restrict__ P, const T* __restrict__ P2,
    const int32_t* __restrict__ c, int n, int h, int64_t B, int nbi, const float* __restrict__ alpha,
    const float* __restrict__ beta, double* __restrict__ part, float* __restrict__ Dout, int64_t ldd) {
  constexpr int KS = TimK<T>::KS;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const int kwmax = (int)round_up(h, KS);
  const int ldr = NF > 0 ? tim_ldr<T>(32 * NF) : tim_ldr<T>(kwmax);
  T* dR = (T*)smem;
  float* a_s = (float*)(smem + (size_t)TIM_BM * ldr * sizeof(T));
  float* red = a_s + round_up(h, 32);                // [4 waves][64 rows]
  double* contrib = (double*)(red + 4 * TIM_BM);     // [64 rows]

  const int64_t wg = blockIdx.x;
  const int q = (int)(wg / B);
  const int64_t b = wg - (int64_t)q * B;
  const int i0 = q * TIM_BM;
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int8_t* Sb = S + b * lds;
  const float* Zb = Z + b * ldz;

  // K range of the block: units that receive any of its sites (k >= c[i0]), aligned to KS
  const int kbase = (c[i0] / KS) * KS;
  const int kw = kwmax - kbase;

  for (int k = t; k < kwmax; k += 256) a_s[k] = k < h ? A[b * ldh + k] : 0.f;
  __syncthreads();
  // dR rows of the block: wave wv builds rows wv + 4 j (j < 16).  A lane covers CPL consecutive
  // columns (16 bytes of weights) per pass; the 16 rows' weights are fetched together (buffer
  // loads: columns past the block's K range and rows past n read zeros), then dR goes to LDS in
  // 16-byte stores.
  {
    constexpr int CPL = 16 / (int)sizeof(T);
    const tim_rsrc_t rp = tim_rsrc(P, (uint32_t)((int64_t)n * ldh * sizeof(T)));
    for (int c0 = 0; c0 < kw; c0 += 64 * CPL) {
      const int kk = c0 + CPL * lane;                  // first column of the lane (relative to kbase)
      const bool col_ok = kk < kw;
      uint4 pv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = i0 + wv + 4 * j;
        const uint32_t off = (uint32_t)(((int64_t)i * ldh + kbase + kk) * sizeof(T));
        pv[j] = tim_ld16(rp, (col_ok && i < n) ? off : TIM_OOB, 0);
      }
      if (col_ok) {
        float av[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) av[e] = a_s[kbase + kk + e];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int r = wv + 4 * j, i = i0 + r;
          const int ci = i < n ? c[i] : h;             // rows past n: no unit receives them
          const float two_s = i < n ? 2.f * (float)Sb[i] : 0.f;
          union {
            uint4 u;
            T e[CPL];
          } w, o;
          w.u = pv[j];
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            const int k = kbase + kk + e;
            const float v = fmaxf(av[e] - two_s * to_f32<T>(w.e[e]), 0.f) - fmaxf(av[e], 0.f);
            o.e[e] = from_f32<T>((k >= ci && k < h) ? v : 0.f);
          }
          *(uint4*)(dR + (size_t)r * ldr + kk) = o.u;
        }
      }
    }
  }
  __syncthreads();

  // per lane: rows 16 mi + 4 (lane >> 4) + r of the block, for the lane's column of each site block
  float lin[4][4], prod[4][4];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      lin[mi][r] = 0.f;
      prod[mi][r] = 1.f;
    }
  const int nbd = (n + TIM_BN - 1) / TIM_BN;
  const int grow = lane >> 4, gcol = lane & 15;
  int since = 0;
  auto renorm = [&]() {
    if (++since == TIM_RENORM) {
      since = 0;
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          lin[mi][r] -= TIM_LN2 * __builtin_amdgcn_logf(prod[mi][r]);
          prod[mi][r] = 1.f;
        }
    }
  };
  if constexpr (NF > 0) {
    // Per block: the products (B fragments already in registers, A fragments from LDS one K
    // step ahead), then the next block's loads (its K end read a block ahead through the
    // scalar cache, its spins and logits, only the B fragments it needs), then this block's
    // epilogue, which covers their latency.
    const tim_rsrc_t rs = tim_rsrc(P2, (uint32_t)((int64_t)n * ldh * 2));
    const bf16_t* arow = (const bf16_t*)dR + (size_t)gcol * ldr + 8 * grow;
    auto kend = [&](int qd) -> int {   // wave-uniform K end of block qd (kbase when it is past n)
      const int dw = qd * TIM_BN + 32 * wv;
      if (dw >= n) return kbase;
      return min((int)round_up(c[min(dw + 31, n - 1)], 32), kwmax);
    };
    // the sweep starts at the site block holding the first flipped site (sites d <= i add 0)
    const int qd0 = i0 / TIM_BN;
    uint4 bfr[2][NF];  // the two column groups' B fragments
    int nk = (kend(qd0) - kbase) / 32;
    int dl[2], s_raw[2];
    float z_raw[2];
    uint32_t roff[2];
    auto operands = [&](int dw) {  // spins, logits and B row offsets of the wave's 32 columns from dw
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        dl[g] = min(dw + 16 * g + gcol, n - 1);
        s_raw[g] = Sb[dl[g]];
        z_raw[g] = Zb[dl[g]];
        roff[g] = (uint32_t)(((int64_t)dl[g] * ldh + kbase + 8 * grow) * 2);
      }
    };
    operands(qd0 * TIM_BN + 32 * wv);
    // B fragments in groups of four behind a uniform branch: the out-of-range loads still pass
    // through the address unit, so only the last group of a block carries any
    auto fetch_b = [&](int need) {
#pragma unroll
      for (int g4 = 0; g4 < NF / 4; ++g4) {
        if (4 * g4 < need) {
#pragma unroll
          for (int f = 4 * g4; f < 4 * g4 + 4; ++f)
#pragma unroll
            for (int g = 0; g < 2; ++g) bfr[g][f] = tim_ld16(rs, f < need ? roff[g] : TIM_OOB, 64u * f);
        }
      }
    };
    fetch_b(nk);
    for (int qd = qd0;; ++qd) {
      const int dw = qd * TIM_BN + 32 * wv;
      if (dw >= n) break;
      const int nk_next = (kend(qd + 1) - kbase) / 32;
      floatx4_t acc[2][4];
      if (nk <= 0) {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) acc[g][mi] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
      } else {
        constexpr int LDR = tim_ldr<bf16_t>(32 * NF);   // == ldr: every LDS offset below is an immediate
        uint4 a[2][4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) a[0][mi] = *(const uint4*)(arow + 16 * mi * LDR);
        // a guarded body rather than an early exit, so that the loop unrolls fully; the next
        // step's A fragments are read whether or not it is needed (within the row; unused)
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          if (f < nk) {
            if (f + 1 < NF) {
#pragma unroll
              for (int mi = 0; mi < 4; ++mi)
                a[(f + 1) & 1][mi] = *(const uint4*)(arow + 16 * mi * LDR + 32 * (f + 1));
            }
            // each A fragment serves both column groups: half the LDS reads per product
#pragma unroll
            for (int g = 0; g < 2; ++g) {
              const bf16x8_t bf = __builtin_bit_cast(bf16x8_t, bfr[g][f]);
#pragma unroll
              for (int mi = 0; mi < 4; ++mi)
                acc[g][mi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8_t, a[f & 1][mi]), bf,
                    f == 0 ? (floatx4_t){0.f, 0.f, 0.f, 0.f} : acc[g][mi], 0, 0, 0);
            }
          }
        }
      }
      float sd[2], td[2], pd[2], rd[2], nmt[2];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const bool valid = dw + 16 * g + gcol < n;
        sd[g] = valid ? (float)s_raw[g] : 0.f;
        td[g] = valid ? sd[g] * z_raw[g] : 0.f;
        pd[g] = __builtin_amdgcn_exp2f(-fabsf(td[g]) * TIM_L2E);
        rd[g] = __builtin_amdgcn_rcpf(1.f + pd[g]);
        nmt[g] = -0.5f * (td[g] - fabsf(td[g]));
      }
      // the next block's operands
      operands(dw + TIM_BN);
      fetch_b(nk_next);
#pragma unroll
      for (int g = 0; g < 2; ++g) tim_epilogue(acc[g], sd[g], td[g], pd[g], rd[g], nmt[g], lin, prod);
      renorm();
      nk = nk_next;
    }
  } else {
    for (int qd = i0 / TIM_BN; qd < nbd; ++qd) {
      const int dw0 = qd * TIM_BN + 32 * wv;   // first column of this wave
      if (dw0 >= n) break;                      // wave-uniform: nothing left for this wave
      for (int g = 0; g < 2; ++g) {           // two groups of 16 columns
        const int dw = dw0 + 16 * g;
        const int d = dw + gcol;
        const bool valid = d < n;
        const float sd = valid ? (float)Sb[d] : 0.f;
        const float td = valid ? sd * Zb[d] : 0.f;
        const float pd = __builtin_amdgcn_exp2f(-fabsf(td) * TIM_L2E);
        const float rd = __builtin_amdgcn_rcpf(1.f + pd);
        const float nmt = -0.5f * (td - fabsf(td));
        // K end of the wave: the units feeding its last valid column
        const int kd = min((int)round_up(__builtin_amdgcn_readfirstlane(c[min(dw + 15, n - 1)]), KS), kwmax);
        floatx4_t acc[4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) acc[mi] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
        const T* brow = P2 + (int64_t)(valid ? d : n - 1) * ldh;
        if constexpr (sizeof(T) == 2) {
          for (int k = kbase; k < kd; k += KS) {
            const int kc = k + 8 * grow;
            const bf16x8_t bf = __builtin_bit_cast(bf16x8_t, *(const uint4*)(brow + kc));
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
              const uint4 av = *(const uint4*)(dR + (size_t)(16 * mi + gcol) * ldr + (kc - kbase));
              acc[mi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av), bf, acc[mi], 0, 0, 0);
            }
          }
        } else {
          for (int k = kbase; k < kd; k += KS) {
            const int kc = k + grow;
            const float bv = (float)brow[kc];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
              const float av = (float)dR[(size_t)(16 * mi + gcol) * ldr + (kc - kbase)];
              acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[mi], 0, 0, 0);
            }
          }
        }
        tim_epilogue(acc, sd, td, pd, rd, nmt, lin, prod);
      }
      renorm();
    }
  }
  // row values of this lane's columns, summed over the 16 columns of the wave (a DPP row)
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = lin[mi][r] - TIM_LN2 * __builtin_amdgcn_logf(prod[mi][r]);
      v += VQMC_DPP(v, 0xB1);   // quad_perm [1,0,3,2]
      v += VQMC_DPP(v, 0x4E);   // quad_perm [2,3,0,1]
      v += VQMC_DPP(v, 0x141);  // row_half_mirror
      v += VQMC_DPP(v, 0x140);  // row_mirror: every lane of the DPP row holds the row sum
      if (gcol == 0) red[wv * TIM_BM + 16 * mi + 4 * grow + r] = v;
    }
  __syncthreads();
  if (t < TIM_BM) {
    const int i = i0 + t;
    double cterm = 0.0;
    if (i < n) {
      const float si = (float)Sb[i];
      const float Di = ((red[t] + red[TIM_BM + t]) + (red[2 * TIM_BM + t] + red[3 * TIM_BM + t])) - si * Zb[i];
      if (Dout) Dout[b * ldd + i] = Di;
      cterm = (double)alpha[i] * exp(0.5 * (double)Di) + (double)beta[i] * (double)si;
    }
    contrib[t] = cterm;
  }
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int r = 0; r < TIM_BM; ++r) s += contrib[r];
    part[b * nbi + q] = s;
  }
}

// E[b] = -(E_zz[b] + sum_q part[b][q]) (fixed order)
__global__ void tim_combine_kernel(const double* __restrict__ Ezz, const double* __restrict__ part, int nbi,
                                   int64_t B, double* __restrict__ E) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = Ezz[b];
  for (int q = 0; q < nbi; ++q) s += part[b * nbi + q];
  E[b] = -s;
}

bool tim_supported(int n, int h, int wdtype) {
  if (n < 2 || h < 1) return false;
  // the kernels address P and the masked second layer (n x ld(h)) with 32-bit byte offsets
  if ((int64_t)n * round_up(h, kPad) * 4 >= (int64_t)TIM_OOB) return false;
  return wdtype == VQMC_BF16 ? h <= 1024 : h <= 512;
}

// workspace: [log p forward region][Z: B x ldn f32][A: B x ldh f32][P2: n x ldh][part: B x nbi f64]
//            [Ezz: B f64][dense-energy partials]
struct TimLayout {
  size_t Z, A, P2, part, Ezz, ews, total;
};
static TimLayout tim_layout(int n, int h, int64_t B, int dtype) {
  const int64_t ldn = round_up(n, kPad), ldh = round_up(h, kPad);
  const int nbi = (n + TIM_BM - 1) / TIM_BM;
  const size_t es = dtype == VQMC_BF16 ? 2 : 4;
  TimLayout L;
  size_t off = (size_t)round_up((int64_t)logprob_ws_bytes(n, h, B, dtype, false), 256);
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (size_t)round_up((int64_t)bytes, 256);
    return o;
  };
  L.Z = take((size_t)B * ldn * 4);
  L.A = take((size_t)B * ldh * 4);
  L.P2 = take((size_t)n * ldh * es);
  L.part = take((size_t)B * nbi * 8);
  L.Ezz = take((size_t)B * 8);
  vqmc_hamiltonian Hd{};
  Hd.n = n;
  Hd.kind = VQMC_H_DENSE_F32;
  L.ews = take(energy_workspace_bytes(Hd, B));
  L.total = off;
  return L;
}

size_t tim_ws_bytes(int n, int h, int64_t B, int dtype) { return tim_layout(n, h, B, dtype).total; }

template <typename T>
static hipError_t tim_energy_t(const vqmc_made& m, const vqmc_tim& H, const int8_t* S, int64_t B, double* E,
                               float* D, void* ws, hipStream_t st) {
  const int n = m.n, h = m.h;
  const int64_t ldn = round_up(n, kPad), ldh = round_up(h, kPad);
  const int nbi = (n + TIM_BM - 1) / TIM_BM;
  const TimLayout L = tim_layout(n, h, B, m.wdtype);
  uint8_t* w = (uint8_t*)ws;
  float* Z = (float*)(w + L.Z);
  float* A = (float*)(w + L.A);
  T* P2 = (T*)(w + L.P2);
  double* part = (double*)(w + L.part);
  double* Ezz = (double*)(w + L.Ezz);
  hipError_t e = launch_tim_forward(m, S, B, Z, A, ws, st);
  if (e != hipSuccess) return e;
  const int64_t np2 = (int64_t)n * ldh;
  tim_w2_kernel<T><<<(unsigned)((np2 + 255) / 256), 256, 0, st>>>((const T*)m.P, m.c, n, ldh, P2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the pipelined sweep holds NF K steps of B fragments in registers: K ranges up to 32 NF
  auto kern = tim_flip_kernel<T, 0>;
  int kalloc = (int)round_up(h, TimK<T>::KS);
  if constexpr (sizeof(T) == 2) {
    if (kalloc <= 32 * 8) {
      kern = tim_flip_kernel<T, 8>;
      kalloc = 32 * 8;
    } else if (kalloc <= 32 * 16) {
      kern = tim_flip_kernel<T, 16>;
      kalloc = 32 * 16;
    }
  }
  const size_t lds_bytes = tim_lds_bytes<T>(h, kalloc);
  if ((e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)) !=
      hipSuccess)
    return e;
  kern<<<(unsigned)(nbi * B), 256, lds_bytes, st>>>(S, ldn, A, ldh, Z, ldn, (const T*)m.P, P2, m.c, n, h, B, nbi,
                                                    H.alpha, H.beta, part, D, ldn);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  vqmc_hamiltonian Hd{};
  Hd.n = n;
  Hd.kind = VQMC_H_DENSE_F32;
  Hd.J = H.J;
  if ((e = launch_energy(Hd, S, B, Ezz, w + L.ews, st)) != hipSuccess) return e;
  tim_combine_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(Ezz, part, nbi, B, E);
  return hipGetLastError();
}

hipError_t launch_tim_energy(const vqmc_made& m, const vqmc_tim& H, const int8_t* S, int64_t B, double* E, float* D,
                             void* ws, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return tim_energy_t<bf16_t>(m, H, S, B, E, D, ws, st);
  return tim_energy_t<float>(m, H, S, B, E, D, ws, st);
}

}  // namespace vqmc
