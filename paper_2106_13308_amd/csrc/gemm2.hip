// BF16 products of the backward pass fed by direct-to-LDS loads (gfx950).
//
// After the incremental sampler has produced relu(A) (Rt) and the logits, the score
// gradient (Sec. 2.1: g = sum_b c_b grad log pi(s_b)) needs three masked products of the
// MADE (Sec. 2.3 MADE layer), all "NT" (both operands K-contiguous):
//   D[b][k]  = [A[b][k] > 0] sum_{d : c[d] > k} G[b][d] P[d][k]   (dF/dA; K = sites)
//   dP[d][k] = sum_b G[b][d] R[b][k]          if k < c[d]          (dF/dW2; K = batch)
//            = sum_b S[b][d] D[b][k]          otherwise            (dF/dW1)
// The first product's mask is a property of the weight operand, so it runs on a masked
// copy of P^T (W1 entries zeroed); the second's masks select output elements.
//
// Engine: a BM x BN tile per workgroup of WGM x WGN waves (each BM/WGM x BN/WGN as 16x16 MFMA
// blocks, v_mfma_f32_16x16x32_bf16, FP32 accumulation; eight or sixteen waves, two or four per
// SIMD, so one wave's loads and barrier waits overlap the others' products).  K advances 64 elements (one 128-byte
// row segment) per stage; three (or four) stages rotate through separate LDS buffers.  Each
// stage is brought in by global_load_lds_dwordx4 (16 bytes per lane straight into LDS, no
// registers): a wave instruction fills 8 rows, lane l the 16-byte chunk l % 8 of row l / 8, from
// a per-lane byte offset fixed for the whole run plus the stage's column (scalar).  Chunk c of
// row r is stored at position c ^ (r % 8), so the 16 rows an MFMA operand read touches spread
// over the LDS banks.  A wave waits for its own loads of a stage (vmcnt) before the stage's
// barrier; after the barrier every wave's loads of that stage have landed.  The next stage to
// fetch is issued right after the barrier, into the buffer every wave finished reading before it.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

typedef __attribute__((address_space(3))) void g2_lds_t;

// s_waitcnt with vmcnt = N and no wait on the other counters (gfx9 encoding)
template <int N>
__device__ inline void g2_wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int BM, int BN, int WGM, int WGN>
struct G2 {
  static constexpr int NW = WGM * WGN;                          // waves: WGM x WGN grid
  static constexpr int FM = BM / (16 * WGM), FN = BN / (16 * WGN);  // 16x16 blocks per wave
  static constexpr int AI = BM / (8 * NW), BI = BN / (8 * NW);  // load instructions per wave per stage
  static constexpr int NLD = AI + BI;
  static_assert(AI * 8 * NW == BM && BI * 8 * NW == BN, "tile rows must split evenly over the waves");

  // operands: rows row0 + r (clamped to rows - 1: rows past the end are loaded but their
  // results are never stored), K columns [k, k + 64) of a row-major bf16 matrix whose
  // leading dimension is a multiple of 64 with zero padding
  struct Op {
    const bf16_t* X;
    int64_t ld;
    int row0, rows;
  };

  // byte offsets of this lane's 16-byte chunks from column 0 of the operands (fixed for a run)
  struct Lanes {
    uint32_t a[AI], b[BI];
  };
  __device__ static Lanes lanes(const Op& a, const Op& b, int wv, int lane) {
    Lanes L;
    const int rl = 8 * wv + (lane >> 3), p = lane & 7;
#pragma unroll
    for (int j = 0; j < AI; ++j) {
      const int r = 8 * NW * j + rl;
      const int gr = min(a.row0 + r, a.rows - 1);
      L.a[j] = (uint32_t)(((int64_t)gr * a.ld + 8 * (p ^ (r & 7))) * 2);
    }
#pragma unroll
    for (int j = 0; j < BI; ++j) {
      const int r = 8 * NW * j + rl;
      const int gr = min(b.row0 + r, b.rows - 1);
      L.b[j] = (uint32_t)(((int64_t)gr * b.ld + 8 * (p ^ (r & 7))) * 2);
    }
    return L;
  }
  __device__ static void issue(const Op& a, const Op& b, const Lanes& L, int k, uint4* As, uint4* Bs, int wv) {
    const uint8_t* ab = (const uint8_t*)(a.X + k);
    const uint8_t* bb = (const uint8_t*)(b.X + k);
#pragma unroll
    for (int j = 0; j < AI; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(ab + L.a[j]), (g2_lds_t*)(As + (8 * NW * j + 8 * wv) * 8), 16,
                                       0, 0);
#pragma unroll
    for (int j = 0; j < BI; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(bb + L.b[j]), (g2_lds_t*)(Bs + (8 * NW * j + 8 * wv) * 8), 16,
                                       0, 0);
  }

  __device__ static void compute(const uint4* As, const uint4* Bs, int wm, int wn, int lane,
                                 floatx4_t (&acc)[FM][FN]) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int c = 4 * ks + (lane >> 4);
      bf16x8_t a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int r = wm + 16 * i + (lane & 15);
        a[i] = __builtin_bit_cast(bf16x8_t, As[r * 8 + (c ^ (r & 7))]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int r = wn + 16 * j + (lane & 15);
        b[j] = __builtin_bit_cast(bf16x8_t, Bs[r * 8 + (c ^ (r & 7))]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }

  // acc = A[rows] x B[rows]^T over K stages [kbeg, kbeg + 64 nst); buffers: three A, three B
  __device__ static void run(const Op& a, const Op& b, int kbeg, int nst, uint4* A0, uint4* A1, uint4* A2,
                             uint4* B0, uint4* B1, uint4* B2, floatx4_t (&acc)[FM][FN]) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv / WGN) * (BM / WGM), wn = (wv % WGN) * (BN / WGN);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    if (nst <= 0) return;
    // every step issues one stage (past the end: the last stage again, never read), so the
    // count of loads in flight is the same on every path
    auto kof = [&](int s) { return kbeg + 64 * min(s, nst - 1); };
    const Lanes L = lanes(a, b, wv, lane);
    issue(a, b, L, kof(0), A0, B0, wv);
    issue(a, b, L, kof(1), A1, B1, wv);
    int i = 0;
    for (; i + 3 <= nst; i += 3) {
      g2_wait_vm<NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 2), A2, B2, wv);
      compute(A0, B0, wm, wn, lane, acc);
      g2_wait_vm<NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 3), A0, B0, wv);
      compute(A1, B1, wm, wn, lane, acc);
      g2_wait_vm<NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 4), A1, B1, wv);
      compute(A2, B2, wm, wn, lane, acc);
    }
    if (i < nst) {
      g2_wait_vm<NLD>();
      __builtin_amdgcn_s_barrier();
      compute(A0, B0, wm, wn, lane, acc);
    }
    if (i + 1 < nst) {
      g2_wait_vm<0>();
      __builtin_amdgcn_s_barrier();
      compute(A1, B1, wm, wn, lane, acc);
    }
    // drain the loads still in flight before the buffers are reused
    g2_wait_vm<0>();
    __builtin_amdgcn_s_barrier();
  }

  // run with four rotating stages: three in flight while one is multiplied
  __device__ static void run4(const Op& a, const Op& b, int kbeg, int nst, uint4* A0, uint4* A1, uint4* A2,
                              uint4* A3, uint4* B0, uint4* B1, uint4* B2, uint4* B3, floatx4_t (&acc)[FM][FN]) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv / WGN) * (BM / WGM), wn = (wv % WGN) * (BN / WGN);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    if (nst <= 0) return;
    auto kof = [&](int s) { return kbeg + 64 * min(s, nst - 1); };
    const Lanes L = lanes(a, b, wv, lane);
    issue(a, b, L, kof(0), A0, B0, wv);
    issue(a, b, L, kof(1), A1, B1, wv);
    issue(a, b, L, kof(2), A2, B2, wv);
    int i = 0;
    for (; i + 4 <= nst; i += 4) {
      g2_wait_vm<2 * NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 3), A3, B3, wv);
      compute(A0, B0, wm, wn, lane, acc);
      g2_wait_vm<2 * NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 4), A0, B0, wv);
      compute(A1, B1, wm, wn, lane, acc);
      g2_wait_vm<2 * NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 5), A1, B1, wv);
      compute(A2, B2, wm, wn, lane, acc);
      g2_wait_vm<2 * NLD>();
      __builtin_amdgcn_s_barrier();
      issue(a, b, L, kof(i + 6), A2, B2, wv);
      compute(A3, B3, wm, wn, lane, acc);
    }
    // stages i, i + 1, i + 2 are in flight in A0/B0, A1/B1, A2/B2
    if (i < nst) {
      g2_wait_vm<2 * NLD>();
      __builtin_amdgcn_s_barrier();
      compute(A0, B0, wm, wn, lane, acc);
    }
    if (i + 1 < nst) {
      g2_wait_vm<NLD>();
      __builtin_amdgcn_s_barrier();
      compute(A1, B1, wm, wn, lane, acc);
    }
    if (i + 2 < nst) {
      g2_wait_vm<0>();
      __builtin_amdgcn_s_barrier();
      compute(A2, B2, wm, wn, lane, acc);
    }
    g2_wait_vm<0>();
    __builtin_amdgcn_s_barrier();
  }
};

// ---------------------------------------------------------------- masked copy of P^T
// Pm[k][d] = P[d][k] where unit k feeds site d (k < c[d]), 0 elsewhere (and for d >= n).
// Workgroup index -> (row tile, column tile) such that the column tiles of one row tile run back to
// back on one XCD: workgroups are dealt round-robin to the 8 XCDs, each with its own L2, so the
// row tile's operand is then fetched into one L2 instead of eight.  Launch 8 * ceil(nrow / 8) * ncol
// workgroups; r >= nrow marks a surplus one.
__device__ inline void xcd_tile(int w, int nrow, int ncol, int& r, int& c) {
  const int x = w & 7, j = w >> 3;
  r = x + 8 * (j / ncol);
  c = j % ncol;
  (void)nrow;
}
__host__ inline unsigned xcd_grid(int nrow, int ncol) { return (unsigned)(8 * ((nrow + 7) / 8) * ncol); }

__global__ __launch_bounds__(256) void mask_w2t_kernel(const bf16_t* __restrict__ Pt, int64_t ldn,
                                                        const int32_t* __restrict__ c, int n, int h,
                                                        bf16_t* __restrict__ Pm) {
  // block (x, k): row k, eight-element vectors 256x .. 256x + 255
  const int k = blockIdx.y;
  const int d0 = (blockIdx.x * 256 + threadIdx.x) * 8;
  if (d0 >= ldn) return;
  uint4 v = *(const uint4*)(Pt + (int64_t)k * ldn + d0);
  int cd[8];
  if (d0 + 8 <= n) {
    const int4 c0 = *(const int4*)(c + d0), c1 = *(const int4*)(c + d0 + 4);
    cd[0] = c0.x; cd[1] = c0.y; cd[2] = c0.z; cd[3] = c0.w;
    cd[4] = c1.x; cd[5] = c1.y; cd[6] = c1.z; cd[7] = c1.w;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) cd[q] = (d0 + q < n) ? c[d0 + q] : 0;
  }
  bf16_t* e = (bf16_t*)&v;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (cd[q] <= k) e[q] = 0;  // also every site >= n (cd = 0)
  *(uint4*)(Pm + (int64_t)k * ldn + d0) = v;
}

// ---------------------------------------------------------------- hidden adjoint
// D = [A > 0] (G Pm^T); writes Dt (h x ldB) and db1 partials (per 64-sample tile).
// Unit tile n0 only sees sites d >= count_le(c, n0) (earlier sites do not use it).
constexpr int HB_BM = 64, HB_BN = 128, HB_WGM = 2, HB_WGN = 4;
__global__ __launch_bounds__(64 * HB_WGM * HB_WGN) void bwd_hidden2_kernel(const bf16_t* __restrict__ G, int64_t ldn,
                                                           const bf16_t* __restrict__ Pm,
                                                           const int32_t* __restrict__ c, int n, int h, int64_t B,
                                                           const bf16_t* __restrict__ Rt, bf16_t* __restrict__ Dt,
                                                           int64_t ldB, float* __restrict__ db1_part, int64_t ldh) {
  using E = G2<HB_BM, HB_BN, HB_WGM, HB_WGN>;
  __shared__ __attribute__((aligned(16))) uint4 A0[HB_BM * 8], A1[HB_BM * 8], A2[HB_BM * 8];
  __shared__ __attribute__((aligned(16))) uint4 B0[HB_BN * 8], B1[HB_BN * 8], B2[HB_BN * 8];
  __shared__ float colacc[HB_WGM][HB_BN];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv / HB_WGN) * (HB_BM / HB_WGM), wn = (wv % HB_WGN) * (HB_BN / HB_WGN);
  int mt, nt;
  const int nmt = (int)((B + HB_BM - 1) / HB_BM);  // = ldB / HB_BM: padding rows of Dt are written too
  xcd_tile(blockIdx.x, nmt, (h + HB_BN - 1) / HB_BN, mt, nt);
  if (mt >= nmt) return;
  const int64_t m0 = (int64_t)mt * HB_BM;  // samples
  const int n0 = nt * HB_BN;               // units
  // first site using unit n0 (c non-decreasing)
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] <= n0) lo = mid + 1;
    else hi = mid;
  }
  const int kbeg = (lo / 64) * 64;
  const int nst = (int)((ldn - kbeg) / 64);
  const E::Op a{G, ldn, (int)m0, (int)B};
  const E::Op b{Pm, ldn, n0, h};
  floatx4_t acc[E::FM][E::FN];
  E::run(a, b, kbeg, nst, A0, A1, A2, B0, B1, B2, acc);
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
        bf16_t rv[4], dv[4];
        *(uint2*)rv = *(const uint2*)(Rt + (int64_t)k * ldB + bb);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float dl = (bf16_to_f32(rv[e]) > 0.f && bb + e < B) ? acc[i][j][e] : 0.f;
          cs[j] += dl;
          dv[e] = f32_to_bf16(dl);
        }
        *(uint2*)(Dt + (int64_t)k * ldB + bb) = *(const uint2*)dv;
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
    for (int j = 0; j < E::FN; ++j) colacc[wv / HB_WGN][wn + j * 16 + lane] = cs[j];
  }
  __syncthreads();
  if (t < HB_BN) {
    const int k = n0 + t;
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < HB_WGM; ++q) v += colacc[q][t];
    if (k < ldh) db1_part[(int64_t)mt * ldh + k] = v;
  }
}

// ---------------------------------------------------------------- weight gradient
// Both halves in one launch: a tile runs the lower product (Gt x Rt) if any of its
// elements has k < c[d], the upper one (St x Dt) if any has k >= c[d], and stores each
// element from the product of its half.
constexpr int WB_BM = 128, WB_BN = 128, WB_WGM = 4, WB_WGN = 4;
__global__ __launch_bounds__(64 * WB_WGM * WB_WGN) void bwd_weight2_kernel(const bf16_t* __restrict__ Gt, const bf16_t* __restrict__ Rt,
                                                           const bf16_t* __restrict__ St, const bf16_t* __restrict__ Dt,
                                                           int64_t ldB, const int32_t* __restrict__ c, int n, int h,
                                                           float* __restrict__ dP,
                                                           const float* __restrict__ db1_part, int np1, int64_t ldh,
                                                           const float* __restrict__ db2_part, int np2, int64_t ldn,
                                                           float* __restrict__ db1, float* __restrict__ db2) {
  // the bias gradients first: thread i of the launch sums the partials of db2[i] (i < n) or of
  // db1[i - n] (the grid has more than n + h threads)
  {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) db2[i] = sum_parts(db2_part, np2, ldn, i);
    else if (i < n + h) db1[i - n] = sum_parts(db1_part, np1, ldh, i - n);
  }
  using E = G2<WB_BM, WB_BN, WB_WGM, WB_WGN>;
  __shared__ __attribute__((aligned(16))) uint4 A0[WB_BM * 8], A1[WB_BM * 8], A2[WB_BM * 8], A3[WB_BM * 8];
  __shared__ __attribute__((aligned(16))) uint4 B0[WB_BN * 8], B1[WB_BN * 8], B2[WB_BN * 8], B3[WB_BN * 8];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv / WB_WGN) * (WB_BM / WB_WGM), wn = (wv % WB_WGN) * (WB_BN / WB_WGN);
  int dt, kt;
  xcd_tile(blockIdx.x, (n + WB_BM - 1) / WB_BM, (h + WB_BN - 1) / WB_BN, dt, kt);
  if (dt * WB_BM >= n) return;
  const int d0 = dt * WB_BM;   // sites
  const int k0 = kt * WB_BN;   // units
  const int dlast = min(d0 + WB_BM - 1, n - 1), klast = min(k0 + WB_BN - 1, h - 1);
  const bool lower = k0 < c[dlast];
  const bool upper = klast >= c[d0];
  const int nst = (int)(ldB / 64);
  floatx4_t acc[E::FM][E::FN];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (half == 0 ? !lower : !upper) continue;
    const E::Op a{half == 0 ? Gt : St, ldB, d0, n};
    const E::Op b{half == 0 ? Rt : Dt, ldB, k0, h};
    E::run4(a, b, 0, nst, A0, A1, A2, A3, B0, B1, B2, B3, acc);
#pragma unroll
    for (int i = 0; i < E::FM; ++i)
#pragma unroll
      for (int j = 0; j < E::FN; ++j) {
        const int k = k0 + wn + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int d = d0 + wm + i * 16 + 4 * (lane >> 4) + e;
          if (d < n && k < h && ((k < c[d]) == (half == 0))) dP[(int64_t)d * h + k] = acc[i][j][e];
        }
      }
  }
}

size_t mask_w2t_bytes(int n, int h) { return (size_t)h * round_up(n, kPad) * sizeof(bf16_t); }

hipError_t launch_mask_w2t(const vqmc_made& m, bf16_t* Pm, hipStream_t st) {
  const int64_t ldn = round_up(m.n, kPad);
  mask_w2t_kernel<<<dim3((unsigned)((ldn / 8 + 255) / 256), (unsigned)m.h), 256, 0, st>>>((const bf16_t*)m.Pt, ldn,
                                                                                         m.c, m.n, m.h, Pm);
  return hipGetLastError();
}

hipError_t launch_bwd_hidden2(const vqmc_made& m, int64_t B, const bf16_t* G, const bf16_t* Pm, const bf16_t* Rt,
                              bf16_t* Dt, float* db1_part, hipStream_t st) {
  const int64_t ldn = round_up(m.n, kPad), ldB = round_up(B, kPad), ldh = round_up(m.h, kPad);
  bwd_hidden2_kernel<<<xcd_grid((int)(ldB / HB_BM), (m.h + HB_BN - 1) / HB_BN), 64 * HB_WGM * HB_WGN, 0, st>>>(
      G, ldn, Pm, m.c, m.n, m.h, B, Rt, Dt, ldB, db1_part, ldh);
  return hipGetLastError();
}

hipError_t launch_backward_products2(const vqmc_made& m, int64_t B, const bf16_t* G, const bf16_t* Gt,
                                     const bf16_t* St, const bf16_t* Rt, bf16_t* Dt, bf16_t* Pm,
                                     float* db1_part, int np1, const float* db2_part, int np2, float* dP, float* db1,
                                     float* db2, hipStream_t st, bool pm_ready) {
  const int64_t ldn = round_up(m.n, kPad), ldB = round_up(B, kPad), ldh = round_up(m.h, kPad);
  hipError_t e = pm_ready ? hipSuccess : launch_mask_w2t(m, Pm, st);
  if (e != hipSuccess) return e;
  bwd_hidden2_kernel<<<xcd_grid((int)(ldB / HB_BM), (m.h + HB_BN - 1) / HB_BN), 64 * HB_WGM * HB_WGN, 0, st>>>(
      G, ldn, Pm, m.c, m.n, m.h, B, Rt, Dt, ldB, db1_part, ldh);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned wgrid = xcd_grid((m.n + WB_BM - 1) / WB_BM, (m.h + WB_BN - 1) / WB_BN);
  if ((int64_t)wgrid * 64 * WB_WGM * WB_WGN < (int64_t)m.n + m.h) return hipErrorInvalidValue;  // never: >= 64 n threads
  bwd_weight2_kernel<<<wgrid, 64 * WB_WGM * WB_WGN, 0, st>>>(Gt, Rt, St, Dt, ldB, m.c, m.n, m.h, dP, db1_part, np1,
                                                             ldh, db2_part, np2, ldn, db1, db2);
  return hipGetLastError();
}

}  // namespace vqmc
