// Pipelined incremental sampler (Algorithm 1 of the paper, with the per-site forward pass
// replaced by an incremental update of the hidden pre-activations).
//
// Notation: packed weights P[d][k] (k < c[d]: W2[d][k]; k >= c[d]: W1[k][d]), state
// A[s][k] = b1[k] + sum_{sites d' received so far} s_d' P[d'][k] of each sample s.  Site d is
//   z_d = b2[d] + sum_{k < c[d]} P[d][k] relu(A[k]),  s_d = +1 iff u < sigma(z_d),
// and unit k receives s_d P[d][k] from every site d < m(k).
//
// Sites are processed in 64-site blocks b = [64b, 64b + 64).  Unit k completes (receives
// its last input) inside block floor(m(k) / 64); with f_b = c[min(64b + 63, n - 1)] the
// units completing in block b are [f_{b-1}, f_b) (f_{-1} = 0).  Only those units make the
// block serial; everything else is a product:
//   logits   z of block b+1 = b2 + relu(A[:, :f_b]) P[block b+1, :f_b]^T        (MFMA)
//   push     A[:, k] += S_block P[block, k] for the units completing after the block
//                                                                                (MFMA)
//   serial   for each unit u in [f_{b-1}, f_b) in order:
//              a_u = A_u + sum_{sites j of the block feeding u} s_j P[j][u]
//              z_j += P[j][u] relu(a_u) for the sites j of the block that use u
//            and s_j = +1 iff z_j > logit(u_j) once every unit site j uses has been added.
// The serial sweep needs no per-site bookkeeping: the W1 half of a unit's column (sites
// feeding it) is always decided when the unit is reached, and the W2 half (sites using it)
// never is, so with the two halves stored apart (the band, see vqmc_band) the sweep reads
// the sign of every site's current logit margin and multiplies by the W1 half, and adds the
// W2 half to every logit; undecided sites meet zero W1 weights and decided ones zero W2
// weights.
//
// Workgroup = 8 samples, 4 waves.  Wave 0 runs the serial sweep of block b with lane
// (sample s, group g) holding sites 8g..8g+7 of sample s in registers; a unit's dot product
// is an 8-lane DPP reduction.  Waves 1-3 meanwhile push block b-1's spins into the units
// completing after block b, compute the part of block b+1's logits that only needs units
// complete before block b, draw block b+1's uniforms, and write out block b-1's spins and
// log-probabilities.  After the sweep all four waves push block b's spins into the units
// of block b+1's sweep and add block b's completed units to block b+1's logits.
//
// Arithmetic: FP32 state and logits.  BF16 weights: the products run on
// v_mfma_f32_16x16x32_bf16, exact for the +-1 spins of the push and with every FP32
// activation split into three BF16 terms (hi + mid + lo is exact) for the logits.  FP32
// weights: v_mfma_f32_16x16x4_f32 for the logits, three-term BF16 split of the weights for
// the push.  The sweep is plain FP32 FMA.  The draw u < sigma(z) is z > logit(u).
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int SP_MS = 8;           // samples per workgroup
constexpr int SP_T = 64;           // sites per block
constexpr int SP_REC = VQMC_BAND_REC;
constexpr int SP_PDS = 6;          // serial band records in flight
constexpr float SP_SCALE = 0x1p100f;

__host__ __device__ inline int sp_lda(int h) { return (int)round_up(h, 32) + 4; }

__host__ inline size_t sp_smem_bytes(int h) {
  const size_t st = (size_t)SP_MS * sp_lda(h) * 4;
  const size_t blk = (size_t)SP_MS * SP_T * 4;        // one [8][64] float buffer
  return st + 2 * blk /*zp*/ + 2 * blk /*th*/ + 3 * blk /*red*/ + 2 * blk /*zs*/ + 2 * SP_MS * SP_T /*sb*/;
}

// exact 3-term BF16 split of 8 floats
__device__ inline void sp_split3(const float r[8], bf16x8_t& hi, bf16x8_t& mid, bf16x8_t& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const bf16_t a = f32_to_bf16(r[e]);
    const float r1 = r[e] - bf16_to_f32(a);
    const bf16_t b = f32_to_bf16(r1);
    const float r2 = r1 - bf16_to_f32(b);
    hi[e] = __builtin_bit_cast(__bf16, a);
    mid[e] = __builtin_bit_cast(__bf16, b);
    lo[e] = __builtin_bit_cast(__bf16, f32_to_bf16(r2));
  }
}

// A-operand fragments of the products, fetched ahead of their use.
//  Z: logits, one K chunk at unit k0, the 4 site tiles of a block (rows = sites)
//     BF16: units k0+8g..k0+8g+7 of site row 16t+i     FP32: unit k0+g
//  U: push, one 16-unit tile (rows = units), both 32-site halves of a block
template <typename WT>
struct SpFrag;
template <>
struct SpFrag<bf16_t> {
  static constexpr int KC = 32;
  typedef uint4 Z1;
  struct Z { uint4 a[4]; };
  struct U { uint4 a[2]; };
};
template <>
struct SpFrag<float> {
  static constexpr int KC = 4;
  typedef float Z1;
  struct Z { float a[4]; };
  struct U { uint4 a[2][2]; };
};

template <typename WT>
__global__ __launch_bounds__(256) void sample_pipe_kernel(
    const WT* __restrict__ P, const WT* __restrict__ Pt, const float* __restrict__ band, int64_t ldh,
    int64_t ldn, const float* __restrict__ b1, const float* __restrict__ b2, const int32_t* __restrict__ c,
    int n, int h, int LDA, int64_t B, uint64_t seed, uint64_t step, int64_t offset, uint32_t tag,
    int8_t* __restrict__ S, int64_t lds, float* __restrict__ logp) {
  using F = SpFrag<WT>;
  constexpr int KC = F::KC;
  constexpr int BLK = SP_MS * SP_T;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float* st = (float*)smem;        // [8][LDA]  state A; final pre-activation once complete
  float* zp = st + SP_MS * LDA;    // [2][8][64] logits of a block before its sweep
  float* th = zp + 2 * BLK;        // [2][8][64] -logit(u) * 2^100
  float* red = th + 2 * BLK;       // [3][64][8] helpers' partial logits of the next block
  float* zs = red + 3 * BLK;       // [2][8][64] s_d z_d of a swept block
  int8_t* sb = (int8_t*)(zs + 2 * BLK);  // [2][8][64] spins of a swept block (0 past n)

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int64_t b0 = (int64_t)blockIdx.x * SP_MS;
  const int nb = (n + SP_T - 1) / SP_T;
  auto fend = [&](int b) { return c[min(SP_T * b + SP_T - 1, n - 1)]; };

  // ---- fragment loaders
  auto fetch_z = [&](typename F::Z& f, int dblk, int k0) {
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      // rows past n load row n-1: their logits are never read back
      const int d = min(dblk + 16 * tt + l16, n - 1);
      if constexpr (sizeof(WT) == 2) {
        f.a[tt] = *(const uint4*)((const bf16_t*)P + (int64_t)d * ldh + k0 + 8 * g4);
      } else {
        f.a[tt] = ((const float*)P)[(int64_t)d * ldh + k0 + g4];
      }
    }
  };
  // activation operand of a K chunk at k0: relu(A[l16][k]) for k in [lo, hi), else 0
  //   BF16: units k0+8g..k0+8g+7 split into three BF16 terms     FP32: unit k0+g
  struct Act {
    bf16x8_t xh, xm, xl;
    float r;
  };
  auto act = [&](int k0, int lo, int hi) {
    Act x;
    if constexpr (sizeof(WT) == 2) {
      float r[8];
      const float* srow = st + l16 * LDA + k0 + 8 * g4;
      if (l16 < SP_MS) {
        const float4 ra = *(const float4*)srow, rb = *(const float4*)(srow + 4);
        r[0] = ra.x; r[1] = ra.y; r[2] = ra.z; r[3] = ra.w;
        r[4] = rb.x; r[5] = rb.y; r[6] = rb.z; r[7] = rb.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = 0.f;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * g4 + e;
        r[e] = (k >= lo && k < hi) ? fmaxf(r[e], 0.f) : 0.f;
      }
      sp_split3(r, x.xh, x.xm, x.xl);
      x.r = 0.f;
    } else {
      const int k = k0 + g4;
      x.r = (l16 < SP_MS && k >= lo && k < hi) ? fmaxf(st[l16 * LDA + k], 0.f) : 0.f;
    }
    return x;
  };
  // one site tile: acc += P[tile rows, chunk] x activation
  auto mfma_z = [&](const Act& x, auto a, floatx4_t acc) {
    if constexpr (sizeof(WT) == 2) {
      const bf16x8_t w = __builtin_bit_cast(bf16x8_t, a);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x.xh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x.xm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x.xl, acc, 0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x.r, acc, 0, 0, 0);
    }
    return acc;
  };
  auto fetch_u = [&](typename F::U& f, int dblk, int k0) {
    // rows past h load row h-1: those state rows are never written back
    const int unit = min(k0 + l16, h - 1);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int dd = dblk + 32 * ks + 8 * g4;  // dblk + 64 <= ldn (blocks are 64-aligned)
      if constexpr (sizeof(WT) == 2) {
        f.a[ks] = *(const uint4*)((const bf16_t*)Pt + (int64_t)unit * ldn + dd);
      } else {
        const float* p = (const float*)Pt + (int64_t)unit * ldn + dd;
        f.a[ks][0] = *(const uint4*)p;
        f.a[ks][1] = *(const uint4*)(p + 4);
      }
    }
  };
  // state rows (units) k0+4g..+3 of sample l16 += tile x block spins, rows outside [lo, hi) kept
  auto use_u = [&](const typename F::U& f, int k0, int lo, int hi, const bf16x8_t (&sv)[2]) {
    float* cp = st + l16 * LDA + k0 + 4 * g4;
    floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
    if (l16 < SP_MS) {
      const float4 cur = *(const float4*)cp;
      acc = (floatx4_t){cur.x, cur.y, cur.z, cur.w};
    }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      if constexpr (sizeof(WT) == 2) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, f.a[ks]), sv[ks], acc, 0, 0, 0);
      } else {
        const float4 w0 = __builtin_bit_cast(float4, f.a[ks][0]);
        const float4 w1 = __builtin_bit_cast(float4, f.a[ks][1]);
        const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        bf16x8_t wh, wm, wl;
        sp_split3(w, wh, wm, wl);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, sv[ks], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm, sv[ks], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, sv[ks], acc, 0, 0, 0);
      }
    }
    if (l16 < SP_MS) {
      const int k = k0 + 4 * g4;
      if (k >= lo && k + 3 < hi) {
        *(float4*)cp = make_float4(acc[0], acc[1], acc[2], acc[3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k + e >= lo && k + e < hi) cp[e] = acc[e];
      }
    }
  };
  // spins of a swept block as the B operand of the push (+-1 / 0 in BF16), sample column l16
  auto spin_operand = [&](const int8_t* sblk, bf16x8_t (&sv)[2]) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      uint2 raw = make_uint2(0, 0);
      if (l16 < SP_MS) raw = *(const uint2*)(sblk + l16 * SP_T + 32 * ks + 8 * g4);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int8_t v = (int8_t)(((e < 4 ? raw.x : raw.y) >> (8 * (e & 3))) & 0xFF);
        sv[ks][e] = __builtin_bit_cast(__bf16, (bf16_t)(v == 0 ? 0 : (v > 0 ? 0x3F80 : 0xBF80)));
      }
    }
  };
  // -logit(u) * 2^100 for a block: thread tt < 128 draws sites 4(tt&15)..+3 of sample tt>>4
  auto thresholds = [&](int blk, float* dst, int tt) {
    const int s = tt >> 4, q4 = tt & 15;
    const int d = SP_T * blk + 4 * q4;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (d < n) {
      const float4 u4 = site_uniforms(seed, step, tag, (uint64_t)(b0 + s + offset), (uint32_t)(d >> 2));
      const float uv[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // s = +1 iff u < sigma(z) iff z > log(u) - log(1-u); u = 0 gives -inf (always +1)
        const float lg = __logf(uv[e]) - log1pf(-uv[e]);
        v[e] = (d + e < n) ? -lg * SP_SCALE : 0.f;
      }
    }
    *(float4*)(dst + s * SP_T + 4 * q4) = make_float4(v[0], v[1], v[2], v[3]);
  };

  // ---- prologue: state = b1, block 0 logits = b2, block 0 thresholds
  for (int i = t; i < SP_MS * LDA; i += 256) {
    const int k = i % LDA;
    st[i] = (k < h) ? b1[k] : 0.f;
  }
  for (int i = t; i < BLK; i += 256) {
    const int j = i % SP_T;
    zp[i] = (j < n) ? b2[j] : 0.f;
  }
  if (t < 128) thresholds(0, th, t);

  // serial lane roles (wave 0): sample ss, sites 8sg..8sg+7 of the block
  const int ss = lane >> 3, sg = lane & 7;
  float4 rw1a[SP_PDS], rw1b[SP_PDS], rw2a[SP_PDS], rw2b[SP_PDS];
  float rns[SP_PDS];
  auto fetch_rec = [&](int p, int u) {
    const float* r = band + (int64_t)u * SP_REC;
    rw1a[p] = *(const float4*)(r + 8 * sg);
    rw1b[p] = *(const float4*)(r + 8 * sg + 4);
    rw2a[p] = *(const float4*)(r + 64 + 8 * sg);
    rw2b[p] = *(const float4*)(r + 64 + 8 * sg + 4);
    rns[p] = r[128 + (lane & 3)];  // the four copies keep this a per-lane (vector) load
  };
  if (wv == 0) {
#pragma unroll
    for (int p = 0; p < SP_PDS; ++p) fetch_rec(p, min(p, h - 1));
  }
  float lp_part = 0.f;  // wave 1: log pi partial of sample lane>>3, sites 8(lane&7)..
  __syncthreads();

  // spins out + log pi partial of a swept block (wave 1)
  auto emit = [&](int blk, int buf) {
    const int s = lane >> 3, q = lane & 7;
    const int dblk = SP_T * blk;
    const uint2 w = *(const uint2*)(sb + buf * BLK + s * SP_T + 8 * q);
    if (b0 + s < B) *(uint2*)(S + (b0 + s) * lds + dblk + 8 * q) = w;
    const float* zrow = zs + buf * BLK + s * SP_T + 8 * q;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (dblk + 8 * q + e < n) lp_part += log_sigmoid(zrow[e]);
  };

  int fprev = 0, fcur = fend(0);
  for (int b = 0; b < nb; ++b) {
    const int d0 = SP_T * b, Tb = min(SP_T, n - d0);
    const bool has_next = b + 1 < nb;
    const int fnext = has_next ? fend(b + 1) : h;
    const int cur = b & 1, nxt = cur ^ 1;

    if (wv == 0) {
      // ================= serial sweep of block b over units [fprev, fcur)
      float zr[8], tz[8];
      {
        const float* zrow = zp + cur * BLK + ss * SP_T + 8 * sg;
        const float* trow = th + cur * BLK + ss * SP_T + 8 * sg;
        const float4 z0 = *(const float4*)zrow, z1 = *(const float4*)(zrow + 4);
        const float4 t0 = *(const float4*)trow, t1 = *(const float4*)(trow + 4);
        zr[0] = z0.x; zr[1] = z0.y; zr[2] = z0.z; zr[3] = z0.w;
        zr[4] = z1.x; zr[5] = z1.y; zr[6] = z1.z; zr[7] = z1.w;
        tz[0] = t0.x; tz[1] = t0.y; tz[2] = t0.z; tz[3] = t0.w;
        tz[4] = t1.x; tz[5] = t1.y; tz[6] = t1.z; tz[7] = t1.w;
      }
      float* arow = st + ss * LDA;
      float a0n = arow[fprev];
      for (int ub = fprev - fprev % SP_PDS; ub < fcur; ub += SP_PDS) {
#pragma unroll
        for (int p = 0; p < SP_PDS; ++p) {
          const int u = ub + p;
          if (u >= fprev && u < fcur) {
            const float a0 = a0n;
            a0n = arow[u + 1];
            const float w1[8] = {rw1a[p].x, rw1a[p].y, rw1a[p].z, rw1a[p].w,
                                 rw1b[p].x, rw1b[p].y, rw1b[p].z, rw1b[p].w};
            const float w2[8] = {rw2a[p].x, rw2a[p].y, rw2a[p].z, rw2a[p].w,
                                 rw2b[p].x, rw2b[p].y, rw2b[p].z, rw2b[p].w};
            // c_e = 1 if site e is (or would be) drawn +1 now, else 0; w1 holds 2 W1
            float acc = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float ce = __builtin_amdgcn_fmed3f(fmaf(zr[e], SP_SCALE, tz[e]), 0.f, 1.f);
              acc = fmaf(ce, w1[e], acc);
            }
            acc += VQMC_DPP(acc, 0xB1);   // quad_perm [1,0,3,2]
            acc += VQMC_DPP(acc, 0x4E);   // quad_perm [2,3,0,1]
            acc += VQMC_DPP(acc, 0x141);  // row_half_mirror: 8-lane total in every lane
            const float a = (acc + rns[p]) + a0;
            const float r = fmaxf(a, 0.f);
#pragma unroll
            for (int e = 0; e < 8; ++e) zr[e] = fmaf(w2[e], r, zr[e]);
            arow[u] = a;
          }
          // Every step reloads its slot, so the number of loads in flight is the same on
          // every path and each use waits only for its own slot.  A slot that was used
          // takes unit u + PDS; a slot skipped before the range already holds u + PDS and
          // one skipped after it holds u, which the next block needs: both reload what
          // they hold.  The barrier keeps the loads after the slot's last use, so they go
          // straight into the slot's registers.
          __builtin_amdgcn_sched_barrier(0);
          fetch_rec(p, min(u < fcur ? u + SP_PDS : u, h - 1));
        }
      }
      // decisions, spins and s*z of the block
      uint32_t lo = 0, hi = 0;
      float zsv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = 8 * sg + e;
        const float ce = __builtin_amdgcn_fmed3f(fmaf(zr[e], SP_SCALE, tz[e]), 0.f, 1.f);
        const bool up = ce > 0.5f;
        const uint32_t byte = (j < Tb) ? (up ? 0x01u : 0xFFu) : 0u;
        if (e < 4) lo |= byte << (8 * e);
        else hi |= byte << (8 * (e - 4));
        zsv[e] = up ? zr[e] : -zr[e];
      }
      *(uint2*)(sb + cur * BLK + ss * SP_T + 8 * sg) = make_uint2(lo, hi);
      float* zsr = zs + cur * BLK + ss * SP_T + 8 * sg;
      *(float4*)zsr = make_float4(zsv[0], zsv[1], zsv[2], zsv[3]);
      *(float4*)(zsr + 4) = make_float4(zsv[4], zsv[5], zsv[6], zsv[7]);
    } else {
      // ================= helpers (waves 1-3)
      const int hw = wv - 1;
      // push of block b-1's spins into units [fcur, h): 16-unit tiles hw, hw+3, ...
      // Ring loads are issued on every path (indices clamped to valid memory) so that each
      // use waits only for its own fragment.
      constexpr int PDU = 4;
      typename F::U fu[PDU];
      const int ubase = fcur & ~15;
      const int nut = (b >= 1 && ubase < h) ? (h - ubase + 15) / 16 : 0;
      const int cntu = (nut > hw) ? (nut - hw + 2) / 3 : 0;
      const int dprev = max(d0 - SP_T, 0);
      auto tile_u = [&](int it) { return ubase + 16 * (hw + 3 * min(it, max(cntu - 1, 0))); };
#pragma unroll
      for (int p = 0; p < PDU; ++p) fetch_u(fu[p], dprev, tile_u(p));
      // early logits of block b+1 over units [0, fprev): K chunks hw, hw+3, ...
      constexpr int PDZ = (sizeof(WT) == 2) ? 4 : 8;
      typename F::Z fz[PDZ];
      const int nzc = has_next ? (fprev + KC - 1) / KC : 0;
      const int cntz = (nzc > hw) ? (nzc - hw + 2) / 3 : 0;
      auto chunk_z = [&](int it) { return cntz ? KC * (hw + 3 * min(it, cntz - 1)) : 0; };
#pragma unroll
      for (int p = 0; p < PDZ; ++p) fetch_z(fz[p], d0 + SP_T, chunk_z(p));

      // VALU work while the fragments load
      if (hw == 0) {
        if (b >= 1) emit(b - 1, nxt);
      } else if (has_next) {
        thresholds(b + 1, th + nxt * BLK, (hw - 1) * 64 + lane);
      }

      if (cntu) {
        bf16x8_t sv[2];
        spin_operand(sb + nxt * BLK, sv);
        for (int base = 0; base < cntu; base += PDU) {
#pragma unroll
          for (int p = 0; p < PDU; ++p) {
            const int it = base + p;
            if (it < cntu) use_u(fu[p], ubase + 16 * (hw + 3 * it), fcur, h, sv);
            __builtin_amdgcn_sched_barrier(0);
            fetch_u(fu[p], dprev, tile_u(it + PDU));
          }
        }
      }
      if (has_next) {
        floatx4_t acc[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) acc[tt] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
        for (int base = 0; base < cntz; base += PDZ) {
#pragma unroll
          for (int p = 0; p < PDZ; ++p) {
            const int it = base + p;
            if (it < cntz) {
              const Act x = act(KC * (hw + 3 * it), 0, fprev);
#pragma unroll
              for (int tt = 0; tt < 4; ++tt) acc[tt] = mfma_z(x, fz[p].a[tt], acc[tt]);
            }
            __builtin_amdgcn_sched_barrier(0);
            fetch_z(fz[p], d0 + SP_T, chunk_z(it + PDZ));
          }
        }
        // C layout: lane holds rows (sites) 16tt + 4g4 + e, column (sample) l16
        if (l16 < SP_MS) {
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[(hw * SP_T + 16 * tt + 4 * g4 + e) * SP_MS + l16] = acc[tt][e];
        }
      }
    }
    __syncthreads();

    // ================= tail (all waves): block b+1's sweep needs block b's spins in its
    // units and block b's completed units in its logits
    if (has_next) {
      const int d0n = d0 + SP_T, Tbn = min(SP_T, n - d0n);
      // push block b's spins into units [fcur, fnext): tiles wv, wv+4, ...
      {
        const int ub0 = fcur & ~15;
        bf16x8_t sv[2];
        bool have_sv = false;
        for (int k0 = ub0 + 16 * wv; k0 < fnext; k0 += 64) {
          if (!have_sv) {
            spin_operand(sb + cur * BLK, sv);
            have_sv = true;
          }
          typename F::U f;
          fetch_u(f, d0, k0);
          use_u(f, k0, fcur, fnext, sv);
        }
      }
      // logits of block b+1, site tile wv: + units [fprev, fcur) + helpers' partials + b2
      {
        floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = fprev & ~(KC - 1); k0 < fcur; k0 += KC) {
          const int d = min(d0n + 16 * wv + l16, n - 1);  // rows past n: never read back
          typename F::Z1 a;
          if constexpr (sizeof(WT) == 2) {
            a = *(const uint4*)((const bf16_t*)P + (int64_t)d * ldh + k0 + 8 * g4);
          } else {
            a = ((const float*)P)[(int64_t)d * ldh + k0 + g4];
          }
          const Act x = act(k0, fprev, fcur);
          acc = mfma_z(x, a, acc);
        }
        if (l16 < SP_MS) {
          float* zrow = zp + nxt * BLK + l16 * SP_T;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int j = 16 * wv + 4 * g4 + e;
            float v = 0.f;
            if (j < Tbn) {
              const float r0 = red[(0 * SP_T + j) * SP_MS + l16];
              const float r1 = red[(1 * SP_T + j) * SP_MS + l16];
              const float r2 = red[(2 * SP_T + j) * SP_MS + l16];
              v = b2[d0n + j] + ((r0 + r1) + r2) + acc[e];
            }
            zrow[j] = v;
          }
        }
      }
    }
    __syncthreads();
    fprev = fcur;
    fcur = fnext;
  }

  // last block's spins and log pi, then the 8-lane log pi sum of each sample
  if (wv == 1) {
    emit(nb - 1, (nb - 1) & 1);
    float v = lp_part;
    v += VQMC_DPP(v, 0xB1);
    v += VQMC_DPP(v, 0x4E);
    v += VQMC_DPP(v, 0x141);
    const int s = lane >> 3;
    if ((lane & 7) == 0 && b0 + s < B && logp) logp[b0 + s] = v;
  }
}

// Band records (see vqmc_band): one wave per unit k.
template <typename WT>
__global__ __launch_bounds__(256) void band_kernel(const WT* __restrict__ Pt, int64_t ldn, const int32_t* __restrict__ c,
                                                   int n, int h, float* __restrict__ band) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6), j = threadIdx.x & 63;
  if (k >= h) return;
  // m(k) = first site d with k < c[d] (exists: c[n-1] = h); block of the sweep = m(k) / 64
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] > k) hi = mid;
    else lo = mid + 1;
  }
  const int d = (lo / SP_T) * SP_T + j;
  float w = 0.f;
  bool feeds = false;
  if (d < n) {
    w = to_f32(Pt[(int64_t)k * ldn + d]);
    feeds = k >= c[d];
  }
  float* r = band + (int64_t)k * SP_REC;
  r[j] = feeds ? 2.f * w : 0.f;
  r[64 + j] = feeds ? 0.f : w;
  // minus the W1 half's sum (fixed butterfly order, identical in every lane)
  float s = feeds ? w : 0.f;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o);
  if (j < 4) r[128 + j] = -s;
}

size_t band_floats(int h) { return (size_t)h * SP_REC; }

hipError_t launch_band(const vqmc_made& m, float* band, hipStream_t st) {
  const unsigned grid = (unsigned)((m.h + 3) / 4);
  const int64_t ldn = round_up(m.n, kPad);
  if (m.wdtype == VQMC_BF16)
    band_kernel<bf16_t><<<grid, 256, 0, st>>>((const bf16_t*)m.Pt, ldn, m.c, m.n, m.h, band);
  else
    band_kernel<float><<<grid, 256, 0, st>>>((const float*)m.Pt, ldn, m.c, m.n, m.h, band);
  return hipGetLastError();
}

bool sample_pipe_supported(int n, int h) { return sp_smem_bytes(h) <= 160 * 1024; }

template <typename WT>
static hipError_t launch_pipe_t(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                                uint32_t tag, int8_t* S, float* logp, hipStream_t st) {
  const size_t smem = sp_smem_bytes(m.h);
  hipError_t e = hipFuncSetAttribute((const void*)sample_pipe_kernel<WT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((B + SP_MS - 1) / SP_MS);
  sample_pipe_kernel<WT><<<grid, 256, smem, st>>>((const WT*)m.P, (const WT*)m.Pt, m.band, round_up(m.h, kPad),
                                                  round_up(m.n, kPad), m.b1, m.b2, m.c, m.n, m.h, sp_lda(m.h), B,
                                                  seed, step, offset, tag, S, round_up(m.n, kPad), logp);
  return hipGetLastError();
}

hipError_t launch_sample_pipe(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                              uint32_t tag, int8_t* S, float* logp, hipStream_t st) {
  if (m.wdtype == VQMC_BF16) return launch_pipe_t<bf16_t>(m, B, seed, step, offset, tag, S, logp, st);
  return launch_pipe_t<float>(m, B, seed, step, offset, tag, S, logp, st);
}

}  // namespace vqmc
