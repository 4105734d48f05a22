// Blocked incremental sampler (Algorithm 1 of the paper, with the per-site forward
// pass replaced by an incremental update of the hidden pre-activations).
//
// Notation: packed weights P[d][k] (k < c[d]: W2[d][k]; k >= c[d]: W1[k][d]), state
// A[s][k] = b1[k] + sum_{received sites d'} s_d' P[d'][k] of each sample s.  Site d is
//   z_d = b2[d] + sum_{k < c[d]} P[d][k] relu(A[k]),  s_d = +1 iff u < sigma(z_d)
// and afterwards every unit k >= c[d] adds s_d P[d][k].
//
// Sites are processed in blocks [d0, d1) of at most 64 sites.  With c0 = c[d0] and
// c1 = c[d1-1]:
//  phase 1  units k < c0 are complete before the block starts, so their whole
//           contribution to every site of the block is one product
//           Zp[d][s] = b2[d] + sum_{k<c0} P[d][k] relu(A[s][k])           (MFMA)
//  phase 2  the units [c0, c1) complete inside the block; they are the only serial
//           part.  The block is split into runs of consecutive sites with equal c[d];
//           the sites of a run depend only on units already complete, so a whole run
//           is decided at once, then the in-block units receive the run's spins, and
//           the units completing after the run add their contribution to the pending
//           sites.
//  phase 3  units k >= c1 receive the block's spins in one rank-T update
//           A[s][k] += sum_{d in block} s_d P[d][k]                       (MFMA)
// In exact arithmetic this is the same sequence of conditionals as n full forward
// passes.
//
// Arithmetic: the state is FP32.  With BF16 weights both products run on
// v_mfma_f32_16x16x32_bf16: phase 3 multiplies exact +-1 spins by BF16 weights, and
// phase 1 splits each FP32 activation into three BF16 terms (hi + mid + lo represents
// it exactly), so both are FP32-accurate.  With FP32 weights phase 1 uses
// v_mfma_f32_16x16x4_f32 and phase 3 splits the weights into three BF16 terms.
// The Bernoulli draw compares z with logit(u), which is the draw u < sigma(z).
//
// One workgroup (4 waves) owns 16 samples; the state lives in LDS as [16][LDA] floats.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int SB_MS = 16;   // samples per workgroup
constexpr int SB_T = 64;    // max sites per block
constexpr int SB_UB = 32;   // in-block units whose weights are staged in LDS
constexpr int PD1 = 6;      // phase-1 weight chunks in flight per wave
constexpr int PD3 = 6;      // phase-3 weight tiles in flight per wave

__host__ __device__ inline int sb_lda(int h) { return (int)round_up(h, 32) + 4; }

__host__ inline size_t sb_smem_bytes(int h) {
  const size_t st = (size_t)SB_MS * sb_lda(h) * 4;
  const size_t red = 2 * SB_T * SB_MS * 4;
  const size_t zp = SB_MS * SB_T * 4, thr = SB_MS * SB_T * 4;
  const size_t pb = SB_T * SB_UB * 4;
  const size_t sbk = SB_MS * SB_T, cb = (SB_T + 4) * 4;
  return st + red + zp + thr + pb + sbk + cb;
}

// exact 3-term BF16 split of 8 floats
__device__ inline void split3(const float r[8], bf16x8_t& hi, bf16x8_t& mid, bf16x8_t& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const bf16_t h = f32_to_bf16(r[e]);
    const float r1 = r[e] - bf16_to_f32(h);
    const bf16_t m = f32_to_bf16(r1);
    const float r2 = r1 - bf16_to_f32(m);
    const bf16_t l = f32_to_bf16(r2);
    hi[e] = __builtin_bit_cast(__bf16, h);
    mid[e] = __builtin_bit_cast(__bf16, m);
    lo[e] = __builtin_bit_cast(__bf16, l);
  }
}

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bf16x8_t load_bf16x8(const bf16_t* p) {
  return __builtin_bit_cast(bf16x8_t, *(const uint4*)p);
}
__device__ inline void load_bf16x4x2(const bf16_t* p0, const bf16_t* p1, bf16x8_t& out) {
  const uint2 a = *(const uint2*)p0, b = *(const uint2*)p1;
  out = __builtin_bit_cast(bf16x8_t, make_uint4(a.x, a.y, b.x, b.y));
}

// Weight fragments of the two products, fetched ahead of their use.
//  phase 1, chunk of K units at k0, the wave's two M tiles (rows = sites):
//   BF16: units k0+4g..+3 and k0+16+4g..+3 of row d (the K order of the state operand)
//   FP32: unit k0+g of row d
//  phase 3, one 16-unit tile (rows = units), both 32-site halves of the block
template <typename WT>
struct Frags;
template <>
struct Frags<bf16_t> {
  static constexpr int KC = 32;
  struct P1 { uint2 a[2][2]; };
  struct P3 { uint4 a[2]; };
};
template <>
struct Frags<float> {
  static constexpr int KC = 4;
  struct P1 { float a[2]; };
  struct P3 { uint4 a[2][2]; };
};

template <typename WT>
__global__ __launch_bounds__(256) void sample_blocked_kernel(
    const WT* __restrict__ P, const WT* __restrict__ Pt, int64_t ldh, int64_t ldn,
    const float* __restrict__ b1, const float* __restrict__ b2, const int32_t* __restrict__ c,
    int n, int h, int LDA, int64_t B, uint64_t seed, uint64_t step, int64_t offset, uint32_t tag,
    int8_t* __restrict__ S, int64_t lds, float* __restrict__ logp) {
  using F = Frags<WT>;
  constexpr int KC = F::KC;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float* st = (float*)smem;                 // [16][LDA]   state A
  float* red = st + SB_MS * LDA;            // [2][64][16] phase-1 partials
  float* zp = red + 2 * SB_T * SB_MS;       // [16][64]    logits of the block before phase 2
  float* thr = zp + SB_MS * SB_T;           // [16][64]    logit(u)
  float* pb = thr + SB_MS * SB_T;           // [64][UB]    P[d0+j][c0+u]
  int8_t* sbk = (int8_t*)(pb + SB_T * SB_UB);  // [16][64] spins of the block
  int* cb = (int*)(sbk + SB_MS * SB_T);     // [65]        c[d0+j], sentinel c1

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int kh = wv & 1, mh = wv >> 1;      // phase-1 split: K half, M (site) half
  const int64_t b0 = (int64_t)blockIdx.x * SB_MS;

  // block [d0, d1): at most 64 sites, a multiple of 8 unless it ends at n, and as long
  // as the in-block units c[d1-1] - c[d0] fit the LDS stage (at least 8 sites)
  auto block_end = [&](int d0) {
    const int c0 = c[d0];
    int d1 = min(d0 + SB_T, n);
    while (d1 - d0 > 8 && c[d1 - 1] - c0 > SB_UB) d1 = d0 + ((d1 - d0 - 1) >> 3) * 8;
    return d1;
  };
  auto fetch_p1 = [&](typename F::P1& f, int dblk, int k0) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int d = dblk + 32 * mh + 16 * mt + l16;
      if constexpr (sizeof(WT) == 2) {
        if (d < n) {
          const bf16_t* prow = (const bf16_t*)P + (int64_t)d * ldh + k0 + 4 * g;
          f.a[mt][0] = *(const uint2*)prow;
          f.a[mt][1] = *(const uint2*)(prow + 16);
        } else {
          f.a[mt][0] = f.a[mt][1] = make_uint2(0, 0);
        }
      } else {
        f.a[mt] = (d < n) ? ((const float*)P)[(int64_t)d * ldh + k0 + g] : 0.f;
      }
    }
  };
  auto use_p1 = [&](const typename F::P1& f, int k0, int c0, floatx4_t(&acc)[2]) {
    if constexpr (sizeof(WT) == 2) {
      const float* srow = st + l16 * LDA + k0 + 4 * g;
      const float4 ra = *(const float4*)srow;
      const float4 rb = *(const float4*)(srow + 16);
      float r[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kk = k0 + 4 * g + (e & 3) + ((e >> 2) << 4);
        r[e] = (kk < c0) ? fmaxf(r[e], 0.f) : 0.f;
      }
      bf16x8_t hi, mid, lo;
      split3(r, hi, mid, lo);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const bf16x8_t a = __builtin_bit_cast(
            bf16x8_t, make_uint4(f.a[mt][0].x, f.a[mt][0].y, f.a[mt][1].x, f.a[mt][1].y));
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hi, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, mid, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lo, acc[mt], 0, 0, 0);
      }
    } else {
      const int k = k0 + g;
      const float r = (k < c0) ? fmaxf(st[l16 * LDA + k], 0.f) : 0.f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[mt], r, acc[mt], 0, 0, 0);
    }
  };
  auto fetch_p3 = [&](typename F::P3& f, int dblk, int k0) {
    const int unit = k0 + l16;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int dd = dblk + 32 * ks + 8 * g;
      const bool ok = unit < h && dd + 8 <= ldn;
      if constexpr (sizeof(WT) == 2) {
        f.a[ks] = ok ? *(const uint4*)((const bf16_t*)Pt + (int64_t)unit * ldn + dd) : make_uint4(0, 0, 0, 0);
      } else {
        const float* p = (const float*)Pt + (int64_t)unit * ldn + dd;
        f.a[ks][0] = ok ? *(const uint4*)p : make_uint4(0, 0, 0, 0);
        f.a[ks][1] = ok ? *(const uint4*)(p + 4) : make_uint4(0, 0, 0, 0);
      }
    }
  };
  // state rows (units) k0+4g..+3 of sample l16 += tile x block spins; units < c1 untouched
  auto use_p3 = [&](const typename F::P3& f, int k0, int c1, const bf16x8_t(&sv)[2]) {
    float* cp = st + l16 * LDA + k0 + 4 * g;
    const float4 cur = *(const float4*)cp;
    floatx4_t acc = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      if constexpr (sizeof(WT) == 2) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, f.a[ks]), sv[ks], acc, 0, 0, 0);
      } else {
        const float4 w0 = __builtin_bit_cast(float4, f.a[ks][0]);
        const float4 w1 = __builtin_bit_cast(float4, f.a[ks][1]);
        const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        bf16x8_t hi, mid, lo;
        split3(w, hi, mid, lo);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, sv[ks], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mid, sv[ks], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, sv[ks], acc, 0, 0, 0);
      }
    }
    if (k0 + 4 * g >= c1) {
      *(float4*)cp = make_float4(acc[0], acc[1], acc[2], acc[3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (k0 + 4 * g + e >= c1) cp[e] = acc[e];
    }
  };

  for (int i = t; i < SB_MS * LDA; i += 256) {
    const int k = i % LDA;
    st[i] = (k < h) ? b1[k] : 0.f;
  }
  float lp_part = 0.f;
  // phase-1 fragment ring: slot p holds this wave's chunk it with it = p (mod PD1);
  // the first PD1 chunks of a block are fetched during the previous block
  typename F::P1 fr[PD1];
  auto chunks_of = [&](int cc0) {  // this wave's chunks kh, kh+2, ... below cc0
    const int nch = (cc0 + KC - 1) / KC;
    return (nch > kh) ? (nch - kh + 1) / 2 : 0;
  };
  {
    const int cnt = chunks_of(c[0]);
#pragma unroll
    for (int p = 0; p < PD1; ++p)
      if (p < cnt) fetch_p1(fr[p], 0, (kh + 2 * p) * KC);
  }
  __syncthreads();

  // bounds of the current block; those of the next block are loaded during the current one
  int d1 = block_end(0), c0 = c[0], c1 = c[d1 - 1];
  for (int d0 = 0; d0 < n;) {
    const int Tb = d1 - d0;
    const int U = c1 - c0;
    const bool fastpb = U <= SB_UB;

    // ---------------- staging: loads now, LDS stores after phase 1 (no wait here)
    const int cbv = (t < Tb) ? c[d0 + t] : 0;
    float pbv[SB_T * SB_UB / 256];
#pragma unroll
    for (int q = 0; q < SB_T * SB_UB / 256; ++q) {
      const int i = t + 256 * q;
      pbv[q] = (fastpb && i < Tb * U) ? to_f32(P[(int64_t)(d0 + i / U) * ldh + c0 + i % U]) : 0.f;
    }
    {
      const int s = t >> 4, q4 = t & 15;  // 16 samples x 16 groups of 4 sites
      if (4 * q4 < Tb) {
        const float4 u4 = site_uniforms(seed, step, tag, (uint64_t)(b0 + s + offset), (uint32_t)((d0 >> 2) + q4));
        const float uv[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float u = uv[e];
          // s = +1 iff u < sigma(z) iff z > log(u) - log(1-u); u = 0 gives -inf (always +1)
          thr[s * SB_T + 4 * q4 + e] = __logf(u) - log1pf(-u);
        }
      }
    }

    // ---------------- phase 1: Zp = relu(A[:, :c0]) P[block, :c0]^T, fragments PD1 chunks ahead
    {
      floatx4_t acc[2];
      acc[0] = acc[1] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
      const int cnt = chunks_of(c0);
      for (int base = 0; base < cnt; base += PD1) {
#pragma unroll
        for (int p = 0; p < PD1; ++p) {
          const int it = base + p;
          if (it < cnt) {
            use_p1(fr[p], (kh + 2 * it) * KC, c0, acc);
            if (it + PD1 < cnt) fetch_p1(fr[p], d0, (kh + 2 * (it + PD1)) * KC);
          }
        }
      }
      // C layout: lane l holds rows (sites) 4*(l/16)+e, column (sample) l%16
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 32 * mh + 16 * mt + 4 * g + e;
          red[(kh * SB_T + j) * SB_MS + l16] = acc[mt][e];
        }
    }
    // staged values of this block
    if (t < Tb) cb[t] = cbv;
    if (t == 0) cb[Tb] = c1;
#pragma unroll
    for (int q = 0; q < SB_T * SB_UB / 256; ++q) {
      const int i = t + 256 * q;
      if (fastpb && i < Tb * U) pb[(i / U) * SB_UB + i % U] = pbv[q];
    }
    // fragments for later: the first PD3 phase-3 tiles of this block and the first PD1
    // phase-1 chunks of the next block; their loads overlap the serial phase
    typename F::P3 gr[PD3];
    const int p3base = (c1 & ~15) + 16 * wv;
    const int ntile = (p3base < h) ? (h - p3base + 63) / 64 : 0;
#pragma unroll
    for (int p = 0; p < PD3; ++p)
      if (p < ntile) fetch_p3(gr[p], d0, p3base + 64 * p);
    int d1n = n, c0n = 0, c1n = 0;
    if (d1 < n) {
      c0n = c[d1];
      d1n = block_end(d1);
      c1n = c[d1n - 1];
      const int cntn = chunks_of(c0n);
#pragma unroll
      for (int p = 0; p < PD1; ++p)
        if (p < cntn) fetch_p1(fr[p], d1, (kh + 2 * p) * KC);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = t + 256 * q;
      const int j = idx >> 4, s = idx & 15;
      if (j < Tb) zp[s * SB_T + j] = red[j * SB_MS + s] + red[(SB_T + j) * SB_MS + s] + b2[d0 + j];
    }
    __syncthreads();

    // ---------------- phase 2: units completing inside the block (wave w: samples 4w..4w+3)
    {
      const int s = 4 * wv + g;
      float* as = st + s * LDA;
      if (fastpb) {
        // lane (s, l16) owns sites l16 + 16m and in-block units c0 + l16 + 16mm in registers
        float zr[4], th[4], ar[2];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int j = l16 + 16 * m;
          zr[m] = (j < Tb) ? zp[s * SB_T + j] : 0.f;
          th[m] = (j < Tb) ? thr[s * SB_T + j] : 0.f;
        }
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
          const int u = c0 + l16 + 16 * mm;
          ar[mm] = (u < c1) ? as[u] : 0.f;
        }
        // run starts: site j starts a run when c[d0+j] differs from its predecessor
        const int cbl = (lane < Tb) ? cb[lane] : c1;
        const int cbp = (lane >= 1 && lane <= Tb) ? cb[lane - 1] : -1;
        const uint64_t starts = __ballot(lane < Tb && cbl != cbp);
        uint32_t dec = 0;
        int i = 0;
        while (i < Tb) {
          const uint64_t later = (i < 63) ? (starts >> (i + 1)) : 0ull;
          const int ie = later ? min(Tb, i + 1 + (int)__builtin_ctzll(later)) : Tb;
          const int cr = __builtin_amdgcn_readlane(cbl, i);
          const int cn = (ie < Tb) ? __builtin_amdgcn_readlane(cbl, ie) : c1;
          // decide every site of the run at once
          uint64_t bm[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int j = l16 + 16 * m;
            const bool inrun = (j >= i) && (j < ie);
            const bool up = zr[m] > th[m];
            if (inrun) {
              if (up) dec |= 1u << m;
              else zr[m] = -zr[m];
            }
            bm[m] = __ballot(inrun && up);
          }
          if (cr < c1) {
            // this lane's sample: bit j = spin of site j is +1 (sites of the run only)
            const uint64_t sm = ((bm[0] >> (16 * g)) & 0xFFFFull) | (((bm[1] >> (16 * g)) & 0xFFFFull) << 16) |
                                (((bm[2] >> (16 * g)) & 0xFFFFull) << 32) | (((bm[3] >> (16 * g)) & 0xFFFFull) << 48);
            // in-block units not yet complete receive the run's spins
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) {
              const int u = c0 + l16 + 16 * mm;
              if (u >= cr && u < c1) {
                float a0 = ar[mm], a1 = 0.f;
                for (int jb = i; jb < ie; jb += 8) {
                  // eight sites at a time: all LDS reads issued before the FMAs
                  float w8[8], s8[8];
#pragma unroll
                  for (int q = 0; q < 8; ++q) {
                    const int j = jb + q;
                    s8[q] = ((sm >> (j & 63)) & 1ull) ? 1.f : -1.f;
                    w8[q] = (j < ie) ? pb[j * SB_UB + (u - c0)] : 0.f;
                  }
#pragma unroll
                  for (int q = 0; q < 8; q += 2) {
                    a0 = fmaf(s8[q], w8[q], a0);
                    a1 = fmaf(s8[q + 1], w8[q + 1], a1);
                  }
                }
                ar[mm] = a0 + a1;
              }
            }
            // units completing after the run feed every pending site of the block
            for (int u = cr; u < cn; ++u) {
              const int rel = u - c0;
              const float v = (rel >= 16) ? ar[1] : ar[0];
              const float r = fmaxf(__shfl(v, (lane & 48) | (rel & 15)), 0.f);
#pragma unroll
              for (int m = 0; m < 4; ++m) {
                const int j = l16 + 16 * m;
                if (j >= ie && j < Tb) zr[m] = fmaf(pb[j * SB_UB + rel], r, zr[m]);
              }
            }
          }
          i = ie;
        }
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
          const int u = c0 + l16 + 16 * mm;
          if (u < c1) as[u] = ar[mm];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int j = l16 + 16 * m;
          if (j < Tb) {
            sbk[s * SB_T + j] = ((dec >> m) & 1u) ? (int8_t)1 : (int8_t)-1;
            lp_part += log_sigmoid(zr[m]);  // zr holds s_d z_d
          }
        }
      } else {
        // many units complete inside the block: work through LDS, weights from global
        float* zs = zp + s * SB_T;
        float* ts = thr + s * SB_T;
        int8_t* ss = sbk + s * SB_T;
        int i = 0;
        while (i < Tb) {
          const int cr = cb[i];
          int ie = i + 1;
          while (ie < Tb && cb[ie] == cr) ++ie;
          const int cn = cb[ie];
          for (int j = i + l16; j < ie; j += 16) {
            const float z = zs[j];
            const bool up = z > ts[j];
            ss[j] = up ? (int8_t)1 : (int8_t)-1;
            ts[j] = up ? z : -z;
          }
          if (cr < c1) {
            wave_sync_lds();
            for (int u = cr + l16; u < c1; u += 16) {
              float a = as[u];
              for (int j = i; j < ie; ++j) a = fmaf((float)ss[j], to_f32(P[(int64_t)(d0 + j) * ldh + u]), a);
              as[u] = a;
            }
            if (cn > cr) {
              wave_sync_lds();
              for (int j = ie + l16; j < Tb; j += 16) {
                float z = zs[j];
                for (int u = cr; u < cn; ++u)
                  z = fmaf(to_f32(P[(int64_t)(d0 + j) * ldh + u]), fmaxf(as[u], 0.f), z);
                zs[j] = z;
              }
            }
            wave_sync_lds();
          }
          i = ie;
        }
        wave_sync_lds();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int j = l16 + 16 * m;
          if (j < Tb) lp_part += log_sigmoid(ts[j]);
        }
      }
    }
    __syncthreads();

    // ---------------- spins of the block to global memory
    {
      const int s = t >> 4, q4 = t & 15;
      if (4 * q4 < Tb && b0 + s < B) {
        uint32_t word = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (4 * q4 + e < Tb) word |= ((uint32_t)(uint8_t)sbk[s * SB_T + 4 * q4 + e]) << (8 * e);
        *(uint32_t*)(S + (b0 + s) * lds + d0 + 4 * q4) = word;
      }
    }

    // ---------------- phase 3: A[:, c1:] += S_block P[block, c1:], fragments PD3 tiles ahead
    {
      bf16x8_t sv[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int j = 32 * ks + 8 * g + e;
          const int8_t v = (j < Tb) ? sbk[l16 * SB_T + j] : (int8_t)0;
          sv[ks][e] = __builtin_bit_cast(__bf16, (bf16_t)(v == 0 ? 0 : (v > 0 ? 0x3F80 : 0xBF80)));
        }
      for (int base = 0; base < ntile; base += PD3) {
#pragma unroll
        for (int p = 0; p < PD3; ++p) {
          const int i = base + p;
          if (i < ntile) {
            use_p3(gr[p], p3base + 64 * i, c1, sv);
            if (i + PD3 < ntile) fetch_p3(gr[p], d0, p3base + 64 * (i + PD3));
          }
        }
      }
    }
    __syncthreads();
    d0 = d1;
    d1 = d1n;
    c0 = c0n;
    c1 = c1n;
  }

  // log pi: sum the 16 per-thread partials of each sample (one 16-lane DPP row)
  float v = lp_part;
  v += VQMC_DPP(v, 0xB1);
  v += VQMC_DPP(v, 0x4E);
  v += VQMC_DPP(v, 0x141);
  v += VQMC_DPP(v, 0x140);
  const int s = t >> 4;
  if ((t & 15) == 0 && b0 + s < B) {
    if (logp) logp[b0 + s] = v;
    for (int64_t col = round_up(n, 4); col < lds; col += 4) *(uint32_t*)(S + (b0 + s) * lds + col) = 0u;
  }
}

bool sample_blocked_supported(int n, int h) { return sb_smem_bytes(h) <= 160 * 1024; }

template <typename WT>
static hipError_t launch_blocked_t(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                                   uint32_t tag, int8_t* S, float* logp, hipStream_t st) {
  const size_t smem = sb_smem_bytes(m.h);
  hipError_t e = hipFuncSetAttribute((const void*)sample_blocked_kernel<WT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((B + SB_MS - 1) / SB_MS);
  sample_blocked_kernel<WT><<<grid, 256, smem, st>>>((const WT*)m.P, (const WT*)m.Pt, round_up(m.h, kPad),
                                                     round_up(m.n, kPad), m.b1, m.b2, m.c, m.n, m.h,
                                                     sb_lda(m.h), B, seed, step, offset, tag, S,
                                                     round_up(m.n, kPad), logp);
  return hipGetLastError();
}

hipError_t launch_sample_blocked(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                                 uint32_t tag, int8_t* S, float* logp, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return launch_blocked_t<bf16_t>(m, B, seed, step, offset, tag, S, logp, st);
  return launch_blocked_t<float>(m, B, seed, step, offset, tag, S, logp, st);
}

}  // namespace vqmc
