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
// the site blocks d from its own to the last, each wave taking 16 columns d: A fragments from
// LDS, B fragments (rows of the masked second layer) from global memory, 4 MFMA blocks of 16 x 16
// per K step.  Elements with d <= i contribute exactly 0 (their dz is an exact 0), so the
// diagonal block needs no mask.  Workgroups are numbered block-major: the ones that run together
// on an XCD share their flip block and so stream the same rows of the second layer through that
// XCD's L2, and the longest sweeps (the first blocks) start first.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int TIM_BM = 64;       // flipped sites per workgroup
constexpr int TIM_BN = 64;       // sites d per block of the sweep, 16 per wave
constexpr int TIM_RENORM = 64;   // site blocks between renormalisations of the running products
constexpr float TIM_L2E = 1.4426950408889634f;   // log2(e)
constexpr float TIM_LN2 = 0.6931471805599453f;   // ln(2)

template <typename T>
struct TimK {
  static constexpr int KS = sizeof(T) == 2 ? 32 : 4;  // K of one MFMA step
};

// LDS row stride of dR in elements: at least kw, rows 16 bytes apart modulo 256 bytes (BF16) /
// 4 floats apart modulo 64 (F32), so the 16 rows of one fragment read fall in distinct banks.
template <typename T>
__host__ __device__ inline int tim_ldr(int kw) {
  if (sizeof(T) == 2) return (int)(round_up(kw - 8, 128) + 8);
  return (int)(round_up(kw - 4, 64) + 4);
}

template <typename T>
__host__ __device__ inline size_t tim_lds_bytes(int h) {
  const int kw = (int)round_up(h, TimK<T>::KS);
  return (size_t)TIM_BM * tim_ldr<T>(kw) * sizeof(T) + (size_t)round_up(h, 4) * 4 + 4 * TIM_BM * 4 +
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

template <typename T>
__global__ __launch_bounds__(256) void tim_flip_kernel(
    const int8_t* __restrict__ S, int64_t lds, const float* __restrict__ A, int64_t ldh,
    const float* __restrict__ Z, int64_t ldz, const T* __restrict__ P, const T* __restrict__ P2,
    const int32_t* __restrict__ c, int n, int h, int64_t B, int nbi, const float* __restrict__ alpha,
    const float* __restrict__ beta, double* __restrict__ part, float* __restrict__ Dout, int64_t ldd) {
  constexpr int KS = TimK<T>::KS;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const int kwmax = (int)round_up(h, KS);
  const int ldr = tim_ldr<T>(kwmax);
  T* dR = (T*)smem;
  float* a_s = (float*)(smem + (size_t)TIM_BM * ldr * sizeof(T));
  float* red = a_s + round_up(h, 4);                 // [4 waves][64 rows]
  double* contrib = (double*)(red + 4 * TIM_BM);     // [64 rows]

  const int64_t wg = blockIdx.x;
  const int q = (int)(wg / B);
  const int64_t b = wg - (int64_t)q * B;
  const int i0 = q * TIM_BM;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int8_t* Sb = S + b * lds;
  const float* Zb = Z + b * ldz;

  // K range of the block: units that receive any of its sites (k >= c[i0]), aligned to KS
  const int kbase = (c[i0] / KS) * KS;
  const int kw = kwmax - kbase;

  for (int k = t; k < h; k += 256) a_s[k] = A[b * ldh + k];
  __syncthreads();
  // dR rows of the block: wave wv builds rows wv, wv + 4, ...
  for (int r = wv; r < TIM_BM; r += 4) {
    const int i = i0 + r;
    T* row = dR + (size_t)r * ldr;
    if (i < n) {
      const int ci = c[i];
      const float two_s = 2.f * (float)Sb[i];
      const T* Pi = P + (int64_t)i * ldh;
      for (int kk = lane; kk < kw; kk += 64) {
        const int k = kbase + kk;
        float v = 0.f;
        if (k >= ci && k < h) {
          const float a = a_s[k];
          v = fmaxf(a - two_s * to_f32<T>(Pi[k]), 0.f) - fmaxf(a, 0.f);
        }
        row[kk] = from_f32<T>(v);
      }
    } else {
      for (int kk = lane; kk < kw; kk += 64) row[kk] = (T)0;
    }
  }
  __syncthreads();

  // per lane: rows 16 mi + 4 (lane >> 4) + r of the block, for the lane's column of each site block
  float lin[4][4], comp[4][4], prod[4][4], lgs[4][4];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      lin[mi][r] = 0.f;
      comp[mi][r] = 0.f;
      prod[mi][r] = 1.f;
      lgs[mi][r] = 0.f;
    }
  const int nbd = (n + TIM_BN - 1) / TIM_BN;
  const int grow = lane >> 4, gcol = lane & 15;
  int since = 0;
  for (int qd = q; qd < nbd; ++qd) {
    const int dw = qd * TIM_BN + 16 * wv;   // first column of this wave
    if (dw >= n) break;                      // wave-uniform: nothing left for this wave
    const int d = dw + gcol;
    const bool valid = d < n;
    const float sd = valid ? (float)Sb[d] : 0.f;
    const float td = valid ? sd * Zb[d] : 0.f;
    const float pd = __builtin_amdgcn_exp2f(-fabsf(td) * TIM_L2E);
    const float rd = 1.f / (1.f + pd);
    const float mtd = fminf(td, 0.f);
    // K end of the wave: the units feeding its last valid column
    const int kd = min((int)round_up(c[min(dw + 15, n - 1)], KS), kwmax);
    floatx4_t acc[4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) acc[mi] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    const T* brow = P2 + (int64_t)(valid ? d : n - 1) * ldh;
    if constexpr (sizeof(T) == 2) {
      for (int k = kbase; k < kd; k += KS) {
        const int kc = k + 8 * grow;
        uint4 bv = *(const uint4*)(brow + kc);
        if (!valid) bv = make_uint4(0u, 0u, 0u, 0u);
        const bf16x8_t bf = __builtin_bit_cast(bf16x8_t, bv);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
          const uint4 av = *(const uint4*)(dR + (size_t)(16 * mi + gcol) * ldr + (kc - kbase));
          acc[mi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av), bf, acc[mi], 0, 0, 0);
        }
      }
    } else {
      for (int k = kbase; k < kd; k += KS) {
        const int kc = k + grow;
        const float bv = valid ? (float)brow[kc] : 0.f;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
          const float av = (float)dR[(size_t)(16 * mi + gcol) * ldr + (kc - kbase)];
          acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[mi], 0, 0, 0);
        }
      }
    }
    // epilogue: acc[mi][r] = dz for row 16 mi + 4 grow + r, column d
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float u = fmaf(sd, acc[mi][r], td);
        const float e = __builtin_amdgcn_exp2f(-fabsf(u) * TIM_L2E);
        const float x = (e - pd) * rd;
        const float w = 1.f + x;
        comp[mi][r] += x - (w - 1.f);
        prod[mi][r] *= w;
        lin[mi][r] += fminf(u, 0.f) - mtd;
      }
    if (++since == TIM_RENORM) {
      since = 0;
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          lgs[mi][r] += __builtin_amdgcn_logf(prod[mi][r]);
          prod[mi][r] = 1.f;
        }
    }
  }
  // row values of this lane's columns, summed over the 16 columns of the wave (a DPP row)
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = lin[mi][r] - (TIM_LN2 * (lgs[mi][r] + __builtin_amdgcn_logf(prod[mi][r])) + comp[mi][r]);
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
  const size_t lds_bytes = tim_lds_bytes<T>(h);
  if ((e = hipFuncSetAttribute((const void*)tim_flip_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes)) != hipSuccess)
    return e;
  tim_flip_kernel<T><<<(unsigned)(nbi * B), 256, lds_bytes, st>>>(S, ldn, A, ldh, Z, ldn, (const T*)m.P, P2, m.c, n,
                                                                    h, B, nbi, H.alpha, H.beta, part, D, ldn);
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
