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
//   logits   z of block b+1 over the units complete before block b:
//            b2 + relu(A[:, :f_{b-1}]) P[block b+1, :f_{b-1}]^T                  (MFMA)
//   push     A[:, k] += S_{block b-1} P[block b-1, k] for the units k >= f_b      (MFMA)
//   sweep    for each unit u in [f_{b-1}, f_b) in order:
//              a_u = A_u + sum_{j in block b-1} s_j P[j][u]
//                        + sum_{sites j of block b feeding u} s_j P[j][u]
//              z_j += P[j][u] relu(a_u) for the sites j of block b that use u, and for
//                     every site j of block b+1
//            and s_j = +1 iff z_j > logit(u_j) once every unit site j uses has been added.
// The sweep needs no per-site bookkeeping: the W1 half of a unit's column (sites
// feeding it) is always decided when the unit is reached, and the W2 half (sites using it)
// never is, so with the two halves stored apart (the band, see vqmc_band) the sweep reads
// the sign of every site's current logit margin and multiplies by the W1 half, and adds the
// W2 half to every logit; undecided sites meet zero W1 weights and decided ones zero W2
// weights.  The band also holds each unit's weights to the block before (all feeding it)
// and the block after (all using it), so the sweep itself finishes both products that
// depend on the block it has just drawn, and one barrier per block suffices.
//
// Workgroup = 8 samples, 12 waves.  Waves 0-1 sweep block b, four samples each, lane
// (sample s, group g) holding sites 4g..4g+3 of sample s (and of the next block) in
// registers; a unit's dot product is a 16-lane DPP reduction.  The ten helper waves 2-11
// meanwhile push block b-1's spins into the units completing after block b (all helpers),
// compute the part of block b+1's logits that only needs units complete before block b
// (helpers 4-9), draw block b+1's uniforms (helpers 0-1) and write out block b-1's spins and
// log-probabilities (helpers 2-3).  Three waves per SIMD let the helpers' memory latency overlap (issue
// priority: sweep, then the logit helpers, then the rest); the two
// roles run separate loops with one barrier per block each.
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
constexpr int SP_PDS = 4;          // band records in flight in the sweep
constexpr float SP_SCALE = 0x1p100f;

__host__ __device__ inline int sp_lda(int h) { return (int)round_up(h, 32) + 4; }
// row stride of the BF16 split planes: a multiple of 8 elements, so 8-unit reads are 16-byte aligned
__host__ __device__ inline int sp_plda(int h) { return (int)round_up(h, 32) + 8; }

constexpr int SP_NSW = 2;          // sweep waves (four samples each)
constexpr int SP_RS = SP_T + 4;    // row stride of the helpers' partial logits: samples on distinct banks
constexpr int SP_NHW = 10;         // helper waves
// First helper that takes logit tiles: with the activation planes in LDS (cheap logit tiles)
// helpers 0-3 keep to their other work; without them every helper shares the logit tiles.
__host__ __device__ constexpr int sp_zh0(bool planes) { return planes ? 4 : 0; }
__host__ __device__ constexpr int sp_nz(bool planes) { return SP_NHW - sp_zh0(planes); }  // partial-logit slots
constexpr int SP_THREADS = 64 * (SP_NSW + SP_NHW);

__host__ inline size_t sp_smem_bytes(int n, int h, bool planes) {
  const size_t st = (size_t)(SP_MS + 1) * sp_lda(h) * 4;   // + a spare row of zeros
  const size_t blk = (size_t)SP_MS * SP_T * 4;        // one [8][64] float buffer
  const size_t nb = (size_t)(n + SP_T - 1) / SP_T;
  return st + 2 * sp_nz(planes) * (size_t)SP_MS * SP_RS * 4 /*red*/ + 2 * blk /*th*/ + 2 * blk /*zs*/ + 2 * SP_MS * SP_T /*sb*/ +
         2 * SP_MS * SP_T * 2 /*sbf*/ +
         round_up((int64_t)(nb + 1) * 4, 16) /*fb*/ + (planes ? (3 * (size_t)SP_MS + 1) * sp_plda(h) * 2 : 0);
}
constexpr size_t SP_LDS_MAX = 160 * 1024;
// BF16 weights keep the three-term split of every completed activation in LDS when it fits
__host__ inline bool sp_planes(int n, int h, int wdtype) {
  return wdtype == VQMC_BF16 && sp_smem_bytes(n, h, true) <= SP_LDS_MAX;
}

// The sampler's tables (the band buffer): the h unit records of the sweep, then the
// weight fragments of the helpers' products laid out in the order the MFMA lanes read
// them, so that every fragment load is one contiguous 1 KB row per instruction.
//  logit tiles: for every 64-site block q, NZT = 1 + ceil(h / KC) tiles.  Tile 0 holds b2
//    of the block (BF16: hi, mid, lo of its exact three-term split in units 0-2; FP32: b2
//    in unit 0), tile t >= 1 the weights P[64q + site][KC (t-1) + unit] (zero past n).
//    BF16: [4 site tiles][64 lanes][8 units], lane = (unit group g, site i) = 16 g + i.
//    FP32: [4 site tiles][64 lanes] floats, unit = lane / 16.
//  push tiles: for every 64-site block q, NUT = ceil(h / 16) tiles; tile t holds
//    P[64q + site][16 t + unit] (zero past n and h), [2 site halves][64 lanes][8 sites]
//    with lane = 16 g + unit and sites 32 half + 8 g .. + 7.
struct SpTables {
  int64_t z, u, pm, bytes;  // byte offsets of the logit tiles, push tiles, masked P^T; total size
  int nzt, nut, zt, ut;  // tiles per block and bytes per tile
};
__host__ __device__ inline SpTables sp_tables(int n, int h, int wdtype) {
  SpTables t;
  const int nb = (n + SP_T - 1) / SP_T;
  const bool bf = wdtype == VQMC_BF16;
  const int kc = bf ? 32 : 4;
  t.nzt = 1 + (h + kc - 1) / kc;
  t.nut = (h + 15) / 16;
  t.zt = bf ? 4096 : 1024;
  t.ut = bf ? 2048 : 4096;
  t.z = round_up((int64_t)h * VQMC_BAND_REC * 4, 256);
  t.u = t.z + (int64_t)nb * t.nzt * t.zt;
  t.pm = round_up(t.u + (int64_t)nb * t.nut * t.ut, 256);
  // BF16: then the backward's masked copy of P^T, h x ld(n) (unit k feeds site d: k < c[d])
  t.bytes = bf ? t.pm + (int64_t)h * round_up(n, 64) * 2 : t.pm;
  return t;
}

// Exact 3-term BF16 split of 8 floats by truncation: hi keeps the top 8 significant bits
// of x, mid the top 8 of the exact remainder x - hi, and lo = x - hi - mid has at most 8
// significant bits left, so hi + mid + lo = x with every term a BF16 value (normal range).
// Two terms' upper halves are packed into one dword with v_perm_b32.
__device__ inline void sp_split3(const float r[8], bf16x8_t& hi, bf16x8_t& mid, bf16x8_t& lo) {
  uint32_t h[4], m[4], l[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint32_t x0 = __float_as_uint(r[2 * p]), x1 = __float_as_uint(r[2 * p + 1]);
    const uint32_t h0 = x0 & 0xFFFF0000u, h1 = x1 & 0xFFFF0000u;
    const float r0 = r[2 * p] - __uint_as_float(h0), r1 = r[2 * p + 1] - __uint_as_float(h1);
    const uint32_t m0 = __float_as_uint(r0) & 0xFFFF0000u, m1 = __float_as_uint(r1) & 0xFFFF0000u;
    const float q0 = r0 - __uint_as_float(m0), q1 = r1 - __uint_as_float(m1);
    // bytes 2,3 of the first operand to the low half, bytes 2,3 of the second to the high
    h[p] = __builtin_amdgcn_perm(x1, x0, 0x07060302u);
    m[p] = __builtin_amdgcn_perm(__float_as_uint(r1), __float_as_uint(r0), 0x07060302u);
    l[p] = __builtin_amdgcn_perm(__float_as_uint(q1), __float_as_uint(q0), 0x07060302u);
    (void)h1;
    (void)m1;
  }
  hi = __builtin_bit_cast(bf16x8_t, make_uint4(h[0], h[1], h[2], h[3]));
  mid = __builtin_bit_cast(bf16x8_t, make_uint4(m[0], m[1], m[2], m[3]));
  lo = __builtin_bit_cast(bf16x8_t, make_uint4(l[0], l[1], l[2], l[3]));
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
  struct Z { uint4 a[4]; };
  struct U { uint4 a[2]; };
};
template <>
struct SpFrag<float> {
  static constexpr int KC = 4;
  struct Z { float a[4]; };
  struct U { uint4 a[2][2]; };
};

// Raw buffer loads of one table tile: base and size in scalar registers, lane offset in a
// vector register.
typedef __amdgpu_buffer_rsrc_t sp_rsrc_t;
__device__ inline sp_rsrc_t sp_rsrc(const uint8_t* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, bytes, 0x00020000);
}
// voff: the lane's byte offset (vector register), soff: the tile's (scalar register)
__device__ inline uint4 sp_ld16(sp_rsrc_t r, int voff, uint32_t soff = 0) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, (int)soff, 0));
}
__device__ inline float sp_ld4(sp_rsrc_t r, int voff, uint32_t soff = 0) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, (int)soff, 0));
}

// one band record of the sweep lane's 4 sites
struct SpRec {
  float4 w1;  // 2 W1, this block
  float4 w2;  // W2, this block
  float4 p1;  // 2 W1, previous block
  float4 n2;  // W2, next block
  float ns;   // minus the sum of the W1 halves
};

// TIMING: each wave also counts its cycles (s_memtime) between the per-block barriers.
// cyc[(g * 12 + w) * 3] = cycles wave w of sample group g spent from leaving one block's barrier
// to arriving at the next one's, summed over the blocks; [.. + 1] = cycles from the first
// departure to the last; [.. + 2] = the same span in ticks of the 100 MHz constant clock.
template <typename WT, bool PLANES, bool TIMING>
__global__ __launch_bounds__(SP_THREADS) void sample_pipe_kernel(
    const uint8_t* __restrict__ ztab, const uint8_t* __restrict__ utab, int nzt, int nut,
    const float* __restrict__ band, const float* __restrict__ b1, const float* __restrict__ b2,
    const int32_t* __restrict__ c,
    int n, int h, int LDA, int64_t B, uint64_t seed, uint64_t step, int64_t offset, uint32_t tag,
    int8_t* __restrict__ S, int64_t lds, float* __restrict__ logp, float* __restrict__ Zs, WT* __restrict__ Rt,
    int64_t ldB, uint64_t* __restrict__ cyc) {
  using F = SpFrag<WT>;
  constexpr int KC = F::KC;
  constexpr int BLK = SP_MS * SP_T;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float* st = (float*)smem;        // [8][LDA]  state A; final pre-activation once complete
                                   // row 8: zeros, the rows of the products' unused columns
  constexpr int RB = SP_MS * SP_RS;
  constexpr int SP_ZH0 = sp_zh0(PLANES), SP_NZ = sp_nz(PLANES);
  float* red = st + (SP_MS + 1) * LDA;  // [2][SP_NZ][8][68] logit helpers' partial logits of a block (+ b2)
  float* th = red + 2 * SP_NZ * RB;    // [2][8][64] -logit(u) * 2^100
  float* zs = th + 2 * BLK;        // [2][8][64] s_d z_d of a swept block
  int8_t* sb = (int8_t*)(zs + 2 * BLK);  // [2][8][64] spins of a swept block (0 past n)

  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index, uniform
  const int l16 = lane & 15, g4 = lane >> 4;
  const int64_t b0 = (int64_t)blockIdx.x * SP_MS;
  const int nb = (n + SP_T - 1) / SP_T;
  uint64_t tm_dep = 0, tm_t0 = 0, tm_busy = 0, tm_r0 = 0;
  auto tm_start = [&]() {
    if constexpr (TIMING) {
      tm_r0 = __builtin_amdgcn_s_memrealtime();
      tm_t0 = tm_dep = __builtin_amdgcn_s_memtime();
    }
  };
  auto block_barrier = [&]() {
    if constexpr (TIMING) tm_busy += __builtin_amdgcn_s_memtime() - tm_dep;
    lds_barrier();
    if constexpr (TIMING) tm_dep = __builtin_amdgcn_s_memtime();
  };
  auto tm_store = [&]() {
    if constexpr (TIMING) {
      if (lane == 0) {
        const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
        uint64_t* o = cyc + ((int64_t)blockIdx.x * (SP_NSW + SP_NHW) + wv) * 3;
        o[0] = tm_busy;
        o[1] = tm_dep - tm_t0;
        o[2] = r1 - tm_r0;
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
        // s = +1 iff u < sigma(z) iff z > log(u) - log(1-u); u = 0 gives -inf (always +1).
        // 1 - u is exact for the 24-bit dyadic u.
        const float lg = __logf(uv[e]) - __logf(1.f - uv[e]);
        v[e] = (d + e < n) ? -lg * SP_SCALE : 0.f;
      }
    }
    *(float4*)(dst + s * SP_T + 4 * q4) = make_float4(v[0], v[1], v[2], v[3]);
  };

  // ---- prologue: state = b1, block 0's logits = b2, block 0's thresholds, block bounds
  // [2][8][64] the same spins in BF16 (+1, -1, 0): the B operand of the push products as is
  bf16_t* sbf = (bf16_t*)(sb + 2 * BLK);
  int* fb = (int*)(sbf + 2 * BLK);  // fb[b + 1] = f_b, fb[0] = 0
  // the bounds are the same for every lane: read them into scalar registers so that all
  // loop control and addressing derived from them stays scalar
  auto fbs = [&](int i) { return __builtin_amdgcn_readfirstlane(fb[i]); };
  // [3][8][PLDA] BF16: hi, mid, lo of relu(A) of every completed unit, then a row of zeros
  // (PLANES only)
  bf16_t* pl = (bf16_t*)((uint8_t*)fb + round_up((int64_t)(nb + 1) * 4, 16));
  const int PLDA = sp_plda(h);
  for (int i = t; i < (SP_MS + 1) * LDA; i += SP_THREADS) {
    const int k = i % LDA;
    st[i] = (k < h && i < SP_MS * LDA) ? b1[k] : 0.f;
  }
  if constexpr (PLANES) {
    for (int i = t; i < PLDA; i += SP_THREADS) pl[3 * SP_MS * PLDA + i] = 0;
  }
  for (int i = t; i < SP_NZ * RB; i += SP_THREADS) {  // block 0's logits: b2 in the first slot
    const int j = i % SP_RS;
    red[i] = (i < RB && j < SP_T && j < n) ? b2[j] : 0.f;
  }
  for (int i = t; i <= nb; i += SP_THREADS) fb[i] = (i == 0) ? 0 : c[min(SP_T * i - 1, n - 1)];
  if (t < 128) thresholds(0, th, t);

  if (wv < SP_NSW) {
    // ================= sweep waves: samples 4wv..4wv+3, lane = (sample, 4-site group)
    // issue priority: the sweep (the serial chain of each block) first, then the logit helpers
    // (the longest helper work per block), then the rest
    __builtin_amdgcn_s_setprio(3);
    const int ss = 4 * wv + (lane >> 4), g = lane & 15;
    SpRec ring[SP_PDS];
    auto fetch_rec = [&](SpRec& r, int u) {
      const float* q = band + (int64_t)u * SP_REC + 4 * g;
      r.w1 = *(const float4*)q;
      r.w2 = *(const float4*)(q + 64);
      r.p1 = *(const float4*)(q + 128);
      r.n2 = *(const float4*)(q + 192);
      // the four copies keep this a per-lane (vector) load
      r.ns = band[(int64_t)u * SP_REC + 256 + (lane & 3)];
    };
#pragma unroll
    for (int p = 0; p < SP_PDS; ++p) fetch_rec(ring[p], min(p, h - 1));
    float zn[4], cp[4];  // next block's logits from this block's units; previous block's draws
#pragma unroll
    for (int e = 0; e < 4; ++e) zn[e] = cp[e] = 0.f;
    float* arow = st + ss * LDA;
    __syncthreads();
    tm_start();
    for (int b = 0; b < nb; ++b) {
      const int d0 = SP_T * b, Tb = min(SP_T, n - d0);
      const int fprev = fbs(b), fcur = fbs(b + 1);
      const int cur = b & 1;
      float zr[4], tz[4];
      {
        const float* r0 = red + cur * SP_NZ * RB + ss * SP_RS + 4 * g;
        float4 acc4 = *(const float4*)r0;
#pragma unroll
        for (int q = 1; q < SP_NZ; ++q) {
          const float4 x = *(const float4*)(r0 + q * RB);
          acc4.x += x.x; acc4.y += x.y; acc4.z += x.z; acc4.w += x.w;
        }
        const float4 t4 = *(const float4*)(th + cur * BLK + ss * SP_T + 4 * g);
        zr[0] = acc4.x + zn[0]; zr[1] = acc4.y + zn[1]; zr[2] = acc4.z + zn[2]; zr[3] = acc4.w + zn[3];
        tz[0] = t4.x; tz[1] = t4.y; tz[2] = t4.z; tz[3] = t4.w;
#pragma unroll
        for (int e = 0; e < 4; ++e) zn[e] = 0.f;
      }
      float a0n = arow[fprev];
      for (int ub = fprev - fprev % SP_PDS; ub < fcur; ub += SP_PDS) {
#pragma unroll
        for (int p = 0; p < SP_PDS; ++p) {
          const int u = ub + p;
          if (u >= fprev && u < fcur) {
            const SpRec& r = ring[p];
            const float a0 = a0n;
            a0n = arow[u + 1];
            const float w1[4] = {r.w1.x, r.w1.y, r.w1.z, r.w1.w};
            const float w2[4] = {r.w2.x, r.w2.y, r.w2.z, r.w2.w};
            const float p1[4] = {r.p1.x, r.p1.y, r.p1.z, r.p1.w};
            const float n2[4] = {r.n2.x, r.n2.y, r.n2.z, r.n2.w};
            // c_e = 1 if site e is (or would be) drawn +1 now, else 0; w1 and p1 hold 2 W1
            float acc0 = 0.f, acc1 = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float ce = __builtin_amdgcn_fmed3f(fmaf(zr[e], SP_SCALE, tz[e]), 0.f, 1.f);
              acc0 = fmaf(ce, w1[e], acc0);
              acc1 = fmaf(cp[e], p1[e], acc1);
            }
            float acc = acc0 + acc1;
            acc += VQMC_DPP(acc, 0xB1);   // quad_perm [1,0,3,2]
            acc += VQMC_DPP(acc, 0x4E);   // quad_perm [2,3,0,1]
            acc += VQMC_DPP(acc, 0x141);  // row_half_mirror
            acc += VQMC_DPP(acc, 0x140);  // row_mirror: 16-lane total in every lane
            const float a = (acc + r.ns) + a0;
            const float rl = fmaxf(a, 0.f);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              zr[e] = fmaf(w2[e], rl, zr[e]);
              zn[e] = fmaf(n2[e], rl, zn[e]);
            }
            arow[u] = a;
            if constexpr (PLANES) {
              // exact three-term split of relu(a) by truncation (see sp_split3)
              const uint32_t x = __float_as_uint(rl);
              const float r1 = rl - __uint_as_float(x & 0xFFFF0000u);
              const uint32_t y = __float_as_uint(r1);
              const float r2 = r1 - __uint_as_float(y & 0xFFFF0000u);
              bf16_t* q = pl + ss * PLDA + u;
              q[0] = (bf16_t)(x >> 16);
              q[SP_MS * PLDA] = (bf16_t)(y >> 16);
              q[2 * SP_MS * PLDA] = (bf16_t)(__float_as_uint(r2) >> 16);
            }
          }
          // Every step reloads its slot, so the number of loads in flight is the same on
          // every path and each use waits only for its own slot.  A slot that was used
          // takes unit u + PDS; a slot skipped before the range already holds u + PDS and
          // one skipped after it holds u, which the next block needs: both reload what
          // they hold.  The barrier keeps the loads after the slot's last use, so they go
          // straight into the slot's registers.
          __builtin_amdgcn_sched_barrier(0);
          fetch_rec(ring[p], min(u < fcur ? u + SP_PDS : u, h - 1));
        }
      }
      // decisions, spins and s*z of the block
      uint32_t word = 0, bw[2] = {0u, 0u};
      float zsv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * g + e;
        const float ce = __builtin_amdgcn_fmed3f(fmaf(zr[e], SP_SCALE, tz[e]), 0.f, 1.f);
        const bool up = ce > 0.5f;
        word |= ((j < Tb) ? (up ? 0x01u : 0xFFu) : 0u) << (8 * e);
        bw[e >> 1] |= ((j < Tb) ? (up ? 0x3F80u : 0xBF80u) : 0u) << (16 * (e & 1));
        zsv[e] = (j < Tb) ? (up ? zr[e] : -zr[e]) : 0.f;
        cp[e] = (j < Tb && up) ? 1.f : 0.f;
      }
      *(uint32_t*)(sb + cur * BLK + ss * SP_T + 4 * g) = word;
      *(uint2*)(sbf + cur * BLK + ss * SP_T + 4 * g) = make_uint2(bw[0], bw[1]);
      *(float4*)(zs + cur * BLK + ss * SP_T + 4 * g) = make_float4(zsv[0], zsv[1], zsv[2], zsv[3]);
      block_barrier();
    }
    tm_store();
  } else {
    // ================= helper waves
    const int hw = wv - SP_NSW;
    if (hw >= SP_ZH0) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(0);
    float lp_part = 0.f;  // waves hw 2-3: log pi partial of sample 4(hw-2) + lane/16
    // spins, s*z and log pi partial of a swept block: helper hw in {2, 3}, lane =
    // (sample 4(hw-2) + lane/16, sites 4(lane%16)..+3)
    auto emit = [&](int blk, int buf) {
      const int s = 4 * (hw - 2) + (lane >> 4), q = lane & 15;
      const int dblk = SP_T * blk;
      const uint32_t w = *(const uint32_t*)(sb + buf * BLK + s * SP_T + 4 * q);
      if (b0 + s < B) *(uint32_t*)(S + (b0 + s) * lds + dblk + 4 * q) = w;
      const float4 z4 = *(const float4*)(zs + buf * BLK + s * SP_T + 4 * q);
      const float zv[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (dblk + 4 * q + e < n) lp_part += log_sigmoid(zv[e]);
      // s*z is read again only by the backward, after the energies: a streaming store
      if (Zs && b0 + s < B) store_nt(Zs + (b0 + s) * lds + dblk + 4 * q, __builtin_bit_cast(uint4, z4));
    };
    // ---- work items.  Push tiles: block b pushes block b-1's spins into the 16-unit tiles
    // hw, hw + SP_NHW, ... of the units [f_b & ~15, h).  Logit tiles: block b adds tiles
    // hw - SP_ZH0, hw - SP_ZH0 + SP_NZ, ... of block b+1 to its logits (helpers from SP_ZH0 on;
    // each writes its partial logits to its own slot): tile 0 is b2, tile t >= 1 the K chunk t-1 of the units
    // [0, f_{b-1}).  An item is (block, index);
    // block nb marks "past the last item".  Their weight fragments do not depend on the
    // draws, so each kind has a ring of PD slots that runs ahead through the items of later
    // blocks: a slot holds one of the PD oldest items not yet used, and a used slot takes
    // the next item of its cursor.  Each pass over a ring reloads every slot (an unused slot
    // reloads the item it holds), so the loads in flight after any slot's load are the same
    // on every path and each use waits for its own fragment only.
    struct It { int bb, i; };
    const int ntu = (h + 15) / 16;
    auto next_u = [&](It c) {
      c.i += SP_NHW;
      while (c.i >= ntu) {
        if (++c.bb >= nb) return It{nb, 0};
        c.i = (fbs(c.bb + 1) >> 4) + hw;
      }
      return c;
    };
    // logit tiles go to the helpers from SP_ZH0 on (the first ones draw the thresholds and
    // write out the swept block); the others hold no logit item
    const int zh = hw - SP_ZH0;
    auto next_z = [&](It c, int& lim) {  // lim: chunk count of the cursor's block
      if (zh < 0) return It{nb, 0};
      c.i += SP_NHW - SP_ZH0;
      while (c.i >= lim) {
        if (++c.bb + 1 >= nb) return It{nb, 0};
        lim = 1 + (fbs(c.bb) + KC - 1) / KC;  // the bias tile and the chunks of [0, f_{bb-1})
        c.i = zh;
      }
      return c;
    };
    // Fragments come from the tables: one contiguous row of 64 lanes per load, zeros baked
    // in past the last site and unit.
    constexpr int ES = sizeof(WT);
    constexpr int ZT = (ES == 2) ? 4096 : 1024, UT = (ES == 2) ? 2048 : 4096;
    // Buffer loads: one resource per table (under 4 GB, checked at launch); the tile's byte
    // offset is a scalar operand and the lane's offset a fixed vector one.
    const sp_rsrc_t rz = sp_rsrc(ztab, (int)(uint32_t)((int64_t)nb * nzt * ZT));
    const sp_rsrc_t ru = sp_rsrc(utab, (int)(uint32_t)((int64_t)nb * nut * UT));
    auto load_z = [&](typename F::Z& f, It c) {  // logit tile i of block bb+1
      const uint32_t so = c.bb < nb ? ((uint32_t)(c.bb + 1) * (uint32_t)nzt + (uint32_t)c.i) * ZT : 0u;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        if constexpr (ES == 2) f.a[tt] = sp_ld16(rz, tt * 1024 + lane * 16, so);
        else f.a[tt] = sp_ld4(rz, tt * 256 + lane * 4, so);
      }
    };
    auto load_u = [&](typename F::U& f, It c) {  // push tile i of block bb-1
      const uint32_t so = c.bb < nb ? ((uint32_t)(c.bb - 1) * (uint32_t)nut + (uint32_t)c.i) * UT : 0u;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        if constexpr (ES == 2) {
          f.a[ks] = sp_ld16(ru, ks * 1024 + lane * 16, so);
        } else {
          f.a[ks][0] = sp_ld16(ru, ks * 2048 + lane * 32, so);
          f.a[ks][1] = sp_ld16(ru, ks * 2048 + lane * 32 + 16, so);
        }
      }
    };
    // Products on 16x16 MFMA tiles whose columns are samples: columns 8-15 have no sample.
    // In the push they multiply zero spins and read and write the zero row 8 of the state.
    const int srow = (l16 < SP_MS) ? l16 : SP_MS;
    float* const st_push = st + srow * LDA + 4 * g4;  // + k0: units k0+4g4..+3
    // spins of block b-1 as the push's B operand (+-1 / 0 in BF16), sample column l16
    auto spin_operand = [&](const bf16_t* sblk, bf16x8_t (&sv)[2]) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        uint4 raw = make_uint4(0u, 0u, 0u, 0u);
        if (l16 < SP_MS) raw = *(const uint4*)(sblk + l16 * SP_T + 32 * ks + 8 * g4);
        sv[ks] = __builtin_bit_cast(bf16x8_t, raw);
      }
    };
    // state rows k0+4g4..+3 += tile x block spins; rows below lo belong to the sweep
    auto push_mfma = [&](const typename F::U& f, floatx4_t acc, const bf16x8_t (&sv)[2]) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        if constexpr (ES == 2) {
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
      return acc;
    };
    auto push_store = [&](float* cp, int k0, int lo, floatx4_t acc) {
      if (k0 >= lo) {
        *(float4*)cp = make_float4(acc[0], acc[1], acc[2], acc[3]);
      } else {  // the tile holding f_b: only the units from f_b on
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k0 + 4 * g4 + e >= lo) cp[e] = acc[e];
        // (keeps the last masked store from being merged with the full-tile store above,
        // which would split that one into two)
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // logits' B operand.  BF16 weights: each product pairs the three BF16 terms of the
    // activations in one MFMA's 16 columns: columns 0-7 take hi (first product) and lo
    // (second) of sample l16, columns 8-15 mid of sample l16-8 and zeros; the two halves
    // are added when the block's partial logits are written.
    const bf16_t* pl1 = pl + l16 * PLDA + 8 * g4;                              // [hi; mid]
    const bf16_t* pl2 = pl + (l16 < SP_MS ? 2 * SP_MS + l16 : 3 * SP_MS) * PLDA + 8 * g4;  // [lo; 0]
    const float* st_z = st + (ES == 2 ? (l16 & 7) : srow) * LDA + (ES == 2 ? 8 * g4 : g4);
    const bool lowcol = l16 < SP_MS;
    // tile 0 (b2) times ones in its first units: BF16 units 0-2 hold hi, mid, lo of b2, whose
    // sum is exact in the FP32 accumulator; FP32 unit 0 holds b2
    auto bias_mfma = [&](const typename F::Z& f, floatx4_t (&acc)[4]) {
      const bool on = g4 == 0 && lowcol;
      if constexpr (ES == 2) {
        const uint32_t o2 = on ? 0x3F803F80u : 0u, o1 = on ? 0x3F80u : 0u;
        const bf16x8_t ones = __builtin_bit_cast(bf16x8_t, make_uint4(o2, o1, 0u, 0u));
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
          acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, f.a[tt]), ones, acc[tt], 0, 0, 0);
      } else {
        const float one = on ? 1.f : 0.f;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[tt], one, acc[tt], 0, 0, 0);
      }
    };

    // the B operand of the bias tile for BF16: ones in units 0-2 of the low columns
    const uint4 ones_u = (g4 == 0 && lowcol) ? make_uint4(0x3F803F80u, 0x3F80u, 0u, 0u) : make_uint4(0u, 0u, 0u, 0u);

    // Ring depths: every pass reloads every slot, so a deeper ring costs loads and issue on each
    // pass; with BF16 weights two slots of each kind (about one block of prefetch) are fastest
    // (three: 3 % slower, one: 5-20 % slower); FP32 weights (smaller logit tiles): two push and
    // three logit slots (1.4 % faster than three and six).
    constexpr int PDU = 2;
    constexpr int PDZ = (ES == 2) ? 2 : 3;
    typename F::U fu[PDU];
    typename F::Z fz[PDZ];
    It su[PDU], sz[PDZ];  // item held by each slot
    __syncthreads();      // the block bounds fb[] are written by every thread
    tm_start();
    int zlim = 0;
    It cu = next_u(It{0, ntu});
    It cz = next_z(It{-1, 0}, zlim);
#pragma unroll
    for (int p = 0; p < PDU; ++p) {
      su[p] = cu;
      load_u(fu[p], cu);
      cu = next_u(cu);
    }
#pragma unroll
    for (int p = 0; p < PDZ; ++p) {
      sz[p] = cz;
      load_z(fz[p], cz);
      cz = next_z(cz, zlim);
    }
    for (int b = 0; b < nb; ++b) {
      const int d0 = SP_T * b;
      const bool has_next = b + 1 < nb;
      const int fprev = fbs(b), fcur = fbs(b + 1);
      const int nxt = (b & 1) ^ 1;

      // VALU work first: the ring's fragments for this block were issued a block ago
      if (hw < 2) {
        if (has_next) thresholds(b + 1, th + nxt * BLK, hw * 64 + lane);
      } else if (hw < 4) {
        if (b >= 1) emit(b - 1, nxt);
      }

      // push of block b-1's spins into units [fcur, h)
      auto any_u = [&]() {
        bool a = false;
#pragma unroll
        for (int p = 0; p < PDU; ++p) a |= su[p].bb == b;
        return a;
      };
      if (any_u()) {
        bf16x8_t sv[2];
        spin_operand(sbf + nxt * BLK, sv);
        do {
          // the state of every slot's tile first (a slot of a later block reads rows no
          // one writes during this block), then each used tile's product and store
          floatx4_t cur[PDU];
#pragma unroll
          for (int p = 0; p < PDU; ++p) {
            const float4 v = *(const float4*)(st_push + 16 * su[p].i);
            cur[p] = (floatx4_t){v.x, v.y, v.z, v.w};
          }
#pragma unroll
          for (int p = 0; p < PDU; ++p) {
            if (su[p].bb == b) {
              const int k0 = 16 * su[p].i;
              push_store(st_push + k0, k0, fcur, push_mfma(fu[p], cur[p], sv));
              su[p] = cu;
              cu = next_u(cu);
            }
            __builtin_amdgcn_sched_barrier(0);
            load_u(fu[p], su[p]);
          }
        } while (any_u());
      }

      // block b+1's logits over the units complete before block b, [0, fprev) (the units of
      // block b are added by the sweep)
      if (has_next && zh >= 0) {
        floatx4_t acc[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) acc[tt] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
        auto any_z = [&]() {
          bool a = false;
#pragma unroll
          for (int p = 0; p < PDZ; ++p) a |= sz[p].bb == b;
          return a;
        };
        while (any_z()) {
          if constexpr (PLANES) {
            // each slot's activations are read one slot ahead (units not complete yet are
            // masked below)
            auto read_pl = [&](int p, uint4& a1, uint4& a2) {
              const int kq = KC * max(sz[p].i - 1, 0);
              a1 = *(const uint4*)(pl1 + kq);
              a2 = *(const uint4*)(pl2 + kq);
            };
            uint4 y1, y2;
            read_pl(0, y1, y2);
#pragma unroll
            for (int p = 0; p < PDZ; ++p) {
              uint4 x1[1] = {y1}, x2[1] = {y2};
              if (p + 1 < PDZ) read_pl(p + 1, y1, y2);
              if (sz[p].bb == b) {
                // the bias tile runs the same two products as a chunk, on (ones, zeros), so
                // that both kinds of item accumulate in the same registers
                if (sz[p].i == 0) {
                  x1[0] = ones_u;
                  x2[0] = make_uint4(0u, 0u, 0u, 0u);
                } else {
                  const int k0 = KC * (sz[p].i - 1);
                  if (k0 + KC > fprev) {  // the chunk holding f_{b-1}: units from there are the sweep's
                    bf16_t* e1 = (bf16_t*)&x1[0];
                    bf16_t* e2 = (bf16_t*)&x2[0];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                      const bool keep = k0 + 8 * g4 + e < fprev;
                      e1[e] = keep ? e1[e] : (bf16_t)0;
                      e2[e] = keep ? e2[e] : (bf16_t)0;
                    }
                  }
                }
                const bf16x8_t xa = __builtin_bit_cast(bf16x8_t, x1[0]);
                const bf16x8_t xb = __builtin_bit_cast(bf16x8_t, x2[0]);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                  const bf16x8_t w = __builtin_bit_cast(bf16x8_t, fz[p].a[tt]);
                  acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xa, acc[tt], 0, 0, 0);
                  acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xb, acc[tt], 0, 0, 0);
                }
                sz[p] = cz;
                cz = next_z(cz, zlim);
              }
              __builtin_amdgcn_sched_barrier(0);
              load_z(fz[p], sz[p]);
            }
          } else if constexpr (ES == 2) {
#pragma unroll
            for (int p = 0; p < PDZ; ++p) {
              if (sz[p].bb == b && sz[p].i == 0) {
                bias_mfma(fz[p], acc);
                sz[p] = cz;
                cz = next_z(cz, zlim);
              } else if (sz[p].bb == b) {
                const int k0 = KC * (sz[p].i - 1);
                const float4 ra = *(const float4*)(st_z + k0), rb = *(const float4*)(st_z + k0 + 4);
                float rr[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) rr[e] = (k0 + 8 * g4 + e < fprev) ? fmaxf(rr[e], 0.f) : 0.f;
                bf16x8_t xh, xm, xl;
                sp_split3(rr, xh, xm, xl);
                const uint4 uh = __builtin_bit_cast(uint4, xh), um = __builtin_bit_cast(uint4, xm),
                            ul = __builtin_bit_cast(uint4, xl);
                const uint4 u1 = lowcol ? uh : um;
                const uint4 u2 = lowcol ? ul : make_uint4(0, 0, 0, 0);
                const bf16x8_t xa = __builtin_bit_cast(bf16x8_t, u1);
                const bf16x8_t xb = __builtin_bit_cast(bf16x8_t, u2);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                  const bf16x8_t w = __builtin_bit_cast(bf16x8_t, fz[p].a[tt]);
                  acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xa, acc[tt], 0, 0, 0);
                  acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xb, acc[tt], 0, 0, 0);
                }
                sz[p] = cz;
                cz = next_z(cz, zlim);
              }
              __builtin_amdgcn_sched_barrier(0);
              load_z(fz[p], sz[p]);
            }
          } else {
#pragma unroll
            for (int p = 0; p < PDZ; ++p) {
              if (sz[p].bb == b && sz[p].i == 0) {
                bias_mfma(fz[p], acc);
                sz[p] = cz;
                cz = next_z(cz, zlim);
              } else if (sz[p].bb == b) {
                const int k0 = KC * (sz[p].i - 1);
                const float rr = (k0 + g4 < fprev) ? fmaxf(st_z[k0], 0.f) : 0.f;
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
                  acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fz[p].a[tt], rr, acc[tt], 0, 0, 0);
                sz[p] = cz;
                cz = next_z(cz, zlim);
              }
              __builtin_amdgcn_sched_barrier(0);
              load_z(fz[p], sz[p]);
            }
          }
        }
        // C layout: lane holds rows (sites) 16tt + 4g4 + e, column l16
        if constexpr (ES == 2) {
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[tt][e] += VQMC_DPP(acc[tt][e], 0x128);  // row_ror:8
        }
        if (lowcol) {
          float* dst = red + nxt * SP_NZ * RB + zh * RB + l16 * SP_RS + 4 * g4;
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
            *(float4*)(dst + 16 * tt) = make_float4(acc[tt][0], acc[tt][1], acc[tt][2], acc[tt][3]);
        }
      }
      block_barrier();
    }
    tm_store();
    // last block's spins and log pi, then the 16-lane log pi sum of each sample
    if (hw == 2 || hw == 3) {
      emit(nb - 1, (nb - 1) & 1);
      float v = lp_part;
      v += VQMC_DPP(v, 0xB1);
      v += VQMC_DPP(v, 0x4E);
      v += VQMC_DPP(v, 0x141);
      v += VQMC_DPP(v, 0x140);
      const int s = 4 * (hw - 2) + (lane >> 4);
      if ((lane & 15) == 0 && b0 + s < B && logp) logp[b0 + s] = v;
    }
  }
  // every unit is complete once both loops are done: the hidden activations relu(A) of
  // the forward pass, batch-contiguous (Rt[k][b], zero for b >= B up to ldB)
  __syncthreads();
  if (Rt) {
    const int64_t bend = (blockIdx.x + 1 == gridDim.x) ? ldB : b0 + SP_MS;
    for (int k = t; k < h; k += SP_THREADS) {
      WT v[SP_MS];
#pragma unroll
      for (int s = 0; s < SP_MS; ++s) {
        const float a = (b0 + s < B) ? fmaxf(st[s * LDA + k], 0.f) : 0.f;
        if constexpr (sizeof(WT) == 2) v[s] = f32_to_bf16(a);
        else v[s] = a;
      }
      WT* out = Rt + (int64_t)k * ldB + b0;
      if constexpr (sizeof(WT) == 2) {
        *(uint4*)out = *(const uint4*)v;
      } else {
        *(uint4*)out = *(const uint4*)v;
        *(uint4*)(out + 4) = *(const uint4*)(v + 4);
      }
      for (int64_t bb = b0 + SP_MS; bb < bend; ++bb) Rt[(int64_t)k * ldB + bb] = (WT)0;
    }
  }
}

// Band records (see vqmc_band): one wave per unit k, lane j = site j of a block.
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
  const int q = lo / SP_T;
  float* r = band + (int64_t)k * SP_REC;
  // this block: W1 (sites feeding k) doubled, W2 (sites using k)
  const int d = q * SP_T + j;
  float w = 0.f;
  bool feeds = false;
  if (d < n) {
    w = to_f32(Pt[(int64_t)k * ldn + d]);
    feeds = k >= c[d];
  }
  r[j] = feeds ? 2.f * w : 0.f;
  r[64 + j] = feeds ? 0.f : w;
  // previous block: every site feeds k
  const int dp = (q - 1) * SP_T + j;
  const float wp = (q > 0) ? to_f32(Pt[(int64_t)k * ldn + dp]) : 0.f;
  r[128 + j] = 2.f * wp;
  // next block: every site uses k
  const int dn = (q + 1) * SP_T + j;
  r[192 + j] = (dn < n) ? to_f32(Pt[(int64_t)k * ldn + dn]) : 0.f;
  // minus the W1 halves' sum (fixed butterfly order, identical in every lane)
  float s = (feeds ? w : 0.f) + wp;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o);
  if (j < 4) r[256 + j] = -s;
}

size_t band_floats(int h) { return (size_t)h * SP_REC; }


// Logit tiles (layout: see SpTables), one thread per lane row of a site tile.
template <typename WT>
__global__ __launch_bounds__(256) void ztile_kernel(const WT* __restrict__ P, int64_t ldh, const float* __restrict__ b2,
                                                    int n, int nb, int nzt, uint8_t* __restrict__ zt) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = (int)(gid & 63), tt = (int)((gid >> 6) & 3);
  const int64_t tile = gid >> 8;  // q * nzt + t
  if (tile >= (int64_t)nb * nzt) return;
  const int q = (int)(tile / nzt), t = (int)(tile % nzt);
  const int i = lane & 15, g = lane >> 4;
  const int d = SP_T * q + 16 * tt + i;
  if constexpr (sizeof(WT) == 2) {
    uint32_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (d < n) {
      if (t == 0) {
        if (g == 0) {  // exact three-term split of b2 by truncation
          const float x = b2[d];
          const float hi = __uint_as_float(__float_as_uint(x) & 0xFFFF0000u);
          const float r = x - hi;
          const float mid = __uint_as_float(__float_as_uint(r) & 0xFFFF0000u);
          const float lo = r - mid;
          v[0] = __float_as_uint(hi) >> 16;
          v[1] = __float_as_uint(mid) >> 16;
          v[2] = __float_as_uint(lo) >> 16;
        }
      } else {  // eight consecutive units of row d (inside the padded row: 32 t <= ldh)
        const uint4 r = *(const uint4*)(P + (int64_t)d * ldh + 32 * (t - 1) + 8 * g);
        *(uint4*)(zt + tile * 4096 + tt * 1024 + lane * 16) = r;
        return;
      }
    }
    *(uint4*)(zt + tile * 4096 + tt * 1024 + lane * 16) =
        make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
  } else {
    float v = 0.f;
    if (d < n) v = (t == 0) ? (g == 0 ? b2[d] : 0.f) : P[(int64_t)d * ldh + 4 * (t - 1) + g];
    *(float*)(zt + tile * 1024 + tt * 256 + lane * 4) = v;
  }
}

// Push tiles (layout: see SpTables), one thread per lane row of a site half.
template <typename WT>
__global__ __launch_bounds__(256) void utile_kernel(const WT* __restrict__ Pt, int64_t ldn, int h, int nb, int nut,
                                                    uint8_t* __restrict__ ut) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = (int)(gid & 63), ks = (int)((gid >> 6) & 1);
  const int64_t tile = gid >> 7;  // q * nut + t
  if (tile >= (int64_t)nb * nut) return;
  const int q = (int)(tile / nut), t = (int)(tile % nut);
  const int k = 16 * t + (lane & 15), d0 = SP_T * q + 32 * ks + 8 * (lane >> 4);
  // eight consecutive sites of row k (inside the padded row: d0 + 8 <= 64 nb <= ldn)
  const WT* row = Pt + (int64_t)k * ldn + d0;
  const uint4 z = make_uint4(0, 0, 0, 0);
  if constexpr (sizeof(WT) == 2) {
    *(uint4*)(ut + tile * 2048 + ks * 1024 + lane * 16) = (k < h) ? *(const uint4*)row : z;
  } else {
    uint8_t* o = ut + tile * 4096 + ks * 2048 + lane * 32;
    *(uint4*)o = (k < h) ? *(const uint4*)row : z;
    *(uint4*)(o + 16) = (k < h) ? *(const uint4*)(row + 4) : z;
  }
}

hipError_t launch_band(const vqmc_made& m, float* band, hipStream_t st, bool tiles) {
  const unsigned grid = (unsigned)((m.h + 3) / 4);
  const int64_t ldn = round_up(m.n, kPad);
  if (m.wdtype == VQMC_BF16)
    band_kernel<bf16_t><<<grid, 256, 0, st>>>((const bf16_t*)m.Pt, ldn, m.c, m.n, m.h, band);
  else
    band_kernel<float><<<grid, 256, 0, st>>>((const float*)m.Pt, ldn, m.c, m.n, m.h, band);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !tiles) return e;
  const SpTables tb = sp_tables(m.n, m.h, m.wdtype);
  const int nb = (m.n + SP_T - 1) / SP_T;
  const int64_t ldh = round_up(m.h, kPad);
  uint8_t* tab = (uint8_t*)band;
  const unsigned gz = (unsigned)(((int64_t)nb * tb.nzt * 256 + 255) / 256);
  const unsigned gu = (unsigned)(((int64_t)nb * tb.nut * 128 + 255) / 256);
  if (m.wdtype == VQMC_BF16) {
    ztile_kernel<bf16_t><<<gz, 256, 0, st>>>((const bf16_t*)m.P, ldh, m.b2, m.n, nb, tb.nzt, tab + tb.z);
    utile_kernel<bf16_t><<<gu, 256, 0, st>>>((const bf16_t*)m.Pt, ldn, m.h, nb, tb.nut, tab + tb.u);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_mask_w2t(m, (bf16_t*)(tab + tb.pm), st);
  } else {
    ztile_kernel<float><<<gz, 256, 0, st>>>((const float*)m.P, ldh, m.b2, m.n, nb, tb.nzt, tab + tb.z);
    utile_kernel<float><<<gu, 256, 0, st>>>((const float*)m.Pt, ldn, m.h, nb, tb.nut, tab + tb.u);
  }
  return hipGetLastError();
}

bool sample_pipe_supported(int n, int h) { return sp_smem_bytes(n, h, false) <= SP_LDS_MAX; }

size_t sample_tables_bytes(int n, int h, int wdtype) { return (size_t)sp_tables(n, h, wdtype).bytes; }

void sample_tables_layout(int n, int h, int wdtype, int64_t* z, int64_t* u, int64_t* pm, int* nzt, int* nut) {
  const SpTables t = sp_tables(n, h, wdtype);
  *z = t.z;
  *u = t.u;
  *pm = t.pm;
  *nzt = t.nzt;
  *nut = t.nut;
}

template <typename WT, bool PLANES, bool TIMING = false>
static hipError_t launch_pipe_t(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                                uint32_t tag, int8_t* S, float* logp, float* Zs, void* Rt, int64_t ldB,
                                hipStream_t st, uint64_t* cyc = nullptr) {
  const size_t smem = sp_smem_bytes(m.n, m.h, PLANES);
  hipError_t e = hipFuncSetAttribute((const void*)sample_pipe_kernel<WT, PLANES, TIMING>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((B + SP_MS - 1) / SP_MS);
  const SpTables tb = sp_tables(m.n, m.h, m.wdtype);
  // the helpers address each table through one buffer resource with 32-bit offsets
  const int64_t nbk = (m.n + SP_T - 1) / SP_T;
  if (nbk * tb.nzt * tb.zt >= (INT64_C(1) << 32) || nbk * tb.nut * tb.ut >= (INT64_C(1) << 32))
    return hipErrorInvalidValue;
  const uint8_t* tab = (const uint8_t*)m.band;
  sample_pipe_kernel<WT, PLANES, TIMING><<<grid, SP_THREADS, smem, st>>>(
      tab + tb.z, tab + tb.u, tb.nzt, tb.nut, m.band, m.b1, m.b2, m.c, m.n, m.h,
      sp_lda(m.h), B, seed, step, offset, tag, S, round_up(m.n, kPad), logp, Zs, (WT*)Rt, ldB, cyc);
  return hipGetLastError();
}

hipError_t launch_sample_pipe(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int64_t offset,
                              uint32_t tag, int8_t* S, float* logp, hipStream_t st, float* Zs, void* Rt) {
  const int64_t ldB = round_up(B, kPad);
  if (m.wdtype == VQMC_BF16) {
    if (sp_planes(m.n, m.h, m.wdtype))
      return launch_pipe_t<bf16_t, true>(m, B, seed, step, offset, tag, S, logp, Zs, Rt, ldB, st);
    return launch_pipe_t<bf16_t, false>(m, B, seed, step, offset, tag, S, logp, Zs, Rt, ldB, st);
  }
  return launch_pipe_t<float, false>(m, B, seed, step, offset, tag, S, logp, Zs, Rt, ldB, st);
}

int sample_pipe_waves() { return SP_NSW + SP_NHW; }

hipError_t launch_sample_pipe_cycles(const vqmc_made& m, int64_t B, uint64_t seed, uint64_t step, int8_t* S,
                                     float* logp, uint64_t* cycles, hipStream_t st) {
  const int64_t ldB = round_up(B, kPad);
  if (m.wdtype == VQMC_BF16) {
    if (sp_planes(m.n, m.h, m.wdtype))
      return launch_pipe_t<bf16_t, true, true>(m, B, seed, step, 0, 0, S, logp, nullptr, nullptr, ldB, st, cycles);
    return launch_pipe_t<bf16_t, false, true>(m, B, seed, step, 0, 0, S, logp, nullptr, nullptr, ldB, st, cycles);
  }
  return launch_pipe_t<float, false, true>(m, B, seed, step, 0, 0, S, logp, nullptr, nullptr, ldB, st, cycles);
}

}  // namespace vqmc
