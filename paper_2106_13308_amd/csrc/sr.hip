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
// BF16 factors (sr_gram_mfma_kernel): the sites with one value of c form a segment j (c is
// non-decreasing, so segments are runs of sites; gamma_j is their c).  Then
//   sum_d GG'_d (1 + Q_{c[d]}) = sum_j X_j (.) (1 + Q_{gamma_j}),  X_j = sum_{d in j} GG'_d,
// and the sites with c[d] <= k are the segments with gamma_j <= k, so the ss' prefix of the
// second sweep advances a segment at a time.  X_j and the ss' advances are products over the
// segment's sites (MFMA on a copy of G and S in which every segment starts a 16-site chunk);
// what stays elementwise is one multiply-add per segment (X_j (.) F) and, per unit, the RR'
// advance and the DD' term: about 2 #segments + 3 h operations per entry instead of
// 3 (n + h).  One sweep in the order of the keys (segment gamma_j before unit gamma_j) serves
// both sums.
//
// FP32 factors (sr_gram_kernel): elementwise FP32 work; every Gram entry carries its own
// running prefix.  Each workgroup owns a 64 x 64 tile (tiles on or above the diagonal
// only; K is symmetric) of one work item, a range of one sweep; the factor rows are
// batch-contiguous (X[j][b], ld(B) columns) and reach the tile through LDS panels of rows.  A combine pass adds the items' partial sums in a fixed
// order and mirrors the upper tiles.
#include <algorithm>

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

// Work items (blockIdx.y): a sweep and a range [begin, end) of its outer rows.  The
// longer sweep is split in two; its second half rebuilds the prefix from row 0, which
// costs at most the prefix length again.  Each item writes its own partial sum.
constexpr int GR_ITEMS = 3;
struct GramItems {
  int part[GR_ITEMS], begin[GR_ITEMS], end[GR_ITEMS];
};

constexpr int GR_PR = 32;  // rows per LDS panel

// Rows [r0, min(r0 + GR_PR, nrows)) of X, columns [c0, c0 + 64) and [c1, c1 + 64), into
// panel[row][0..63] and panel[row][64..127] as float: eight threads per row, 16 values each.
template <typename T>
__device__ inline void load_panel(const T* __restrict__ X, int64_t ldb, int r0, int nrows, int64_t c0, int64_t c1,
                                  float (*panel)[2 * GR_T]) {
  const int r = threadIdx.x >> 3, seg = threadIdx.x & 7;
  if (r0 + r >= nrows) return;
  const int64_t col = (seg < 4 ? c0 : c1) + 16 * (seg & 3);
  const T* src = X + (int64_t)(r0 + r) * ldb + col;
  float* dst = &panel[r][16 * seg];
  for (int q = 0; q < 4; ++q) {
    float v[4];
    load4<T>(src + 4 * q, v);
    *reinterpret_cast<float4*>(dst + 4 * q) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// part 0: sum_d GG'_d (1 + prefix_{k < c[d]} RR'_k)
// part 1: sum_k DD'_k (1 + prefix_{d : c[d] <= k} ss'_d)
// A 64 x 64 tile per workgroup of four waves, a 4 x 4 block per thread.  Rows of the
// prefix factor and of the outer factor are staged through two LDS panels of GR_PR rows
// (both 64-sample column ranges of the tile), refilled when the sweep runs past them; the
// staircase order is the same for every thread, so the refills are uniform.  The prefix
// accumulator starts at 1, so an outer row costs one multiply and one multiply-add per
// entry.
template <typename T>
__global__ __launch_bounds__(256) void sr_gram_kernel(const T* __restrict__ Gt, const T* __restrict__ Rt,
                                                      const T* __restrict__ Dt, const T* __restrict__ St,
                                                      int64_t ldb, const int32_t* __restrict__ c,
                                                      const int32_t* __restrict__ cnt, int n, int h, int64_t B,
                                                      int nt, GramItems items, float* __restrict__ parts) {
  __shared__ __align__(16) float pp[GR_PR][2 * GR_T];  // prefix rows
  __shared__ __align__(16) float po[GR_PR][2 * GR_T];  // outer rows
  __shared__ int plim[GR_PR];                          // prefix length of each outer row in po
  int ti, tj;
  upper_tile(blockIdx.x, nt, ti, tj);
  const int item = blockIdx.y;
  const int part = items.part[item];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t c0 = (int64_t)ti * GR_T, c1 = (int64_t)tj * GR_T;
  // part 0: prefix rows R (h), outer rows G (n); part 1: prefix rows S (n), outer rows D (h)
  const T* Xp = part ? St : Rt;
  const T* Xo = part ? Dt : Gt;
  const int np = part ? n : h, no = part ? h : n;
  // prefix rows outer row io sees: k < c[io] (part 0); the sites d with c[d] <= io, a
  // prefix of the sites since c is non-decreasing, cnt[io] of them (part 1)
  const int32_t* lims = part ? cnt : c;
  const int o0 = items.begin[item], o1 = items.end[item];
  float acc[4][4], pre[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = 0.f;
      pre[i][j] = 1.f;
    }
  int ip = 0;                        // next prefix row
  int pbase = -GR_PR, obase = -GR_PR;  // first row held by each panel
  for (int io = o0; io < o1; ++io) {
    if (io >= obase + GR_PR) {
      __syncthreads();
      load_panel<T>(Xo, ldb, io, no, c0, c1, po);
      if (threadIdx.x < GR_PR && io + (int)threadIdx.x < no) plim[threadIdx.x] = lims[io + threadIdx.x];
      obase = io;
      __syncthreads();
    }
    const int lim = __builtin_amdgcn_readfirstlane(plim[io - obase]);
    for (; ip < lim; ++ip) {
      if (ip >= pbase + GR_PR) {
        __syncthreads();
        load_panel<T>(Xp, ldb, ip, np, c0, c1, pp);
        pbase = ip;
        __syncthreads();
      }
      const float4 a = *reinterpret_cast<const float4*>(&pp[ip - pbase][4 * ty]);
      const float4 b = *reinterpret_cast<const float4*>(&pp[ip - pbase][GR_T + 4 * tx]);
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) pre[i][j] = fmaf(av[i], bv[j], pre[i][j]);
    }
    const float4 a = *reinterpret_cast<const float4*>(&po[io - obase][4 * ty]);
    const float4 b = *reinterpret_cast<const float4*>(&po[io - obase][GR_T + 4 * tx]);
    const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i] * bv[j], pre[i][j], acc[i][j]);
  }
  const int64_t br = c0 + 4 * ty, bc = c1 + 4 * tx;
  float* out = parts + (int64_t)item * B * B;
  for (int i = 0; i < 4; ++i) {
    const int64_t r = br + i;
    if (r >= B) break;
    for (int j = 0; j < 4; ++j)
      if (bc + j < B) out[r * B + bc + j] = acc[i][j];
  }
}

// K[b][b'] = sum over the items' partial sums at (lo, hi), the pair ordered so that its
// tile lies on or above the diagonal (where the sweeps wrote it); fixed order.
__global__ void sr_gram_combine_kernel(const float* __restrict__ parts, int nitems, int64_t B,
                                       float* __restrict__ K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * B) return;
  const int64_t r = idx / B, q = idx - r * B;
  const bool upper = (r / GR_T) <= (q / GR_T);
  const int64_t src = upper ? idx : q * B + r;
  float s = parts[src];
  for (int i = 1; i < nitems; ++i) s += parts[(int64_t)i * B * B + src];
  K[idx] = s;
}

// Split of the longer sweep: part 0 costs about 2n + h per entry (outer rows n, prefix h),
// part 1 about 2h + n.  Halving the outer range of the longer one (its halves cost about
// n + h each, the second paying its prefix again) balances the three items.
static GramItems gram_items(int n, int h, int* count) {
  GramItems it{};
  const int big = (n >= h) ? 0 : 1;      // the sweep with the longer outer range
  const int nb = big == 0 ? n : h;       // its outer rows
  const int ns = big == 0 ? h : n;       // its prefix rows = the other sweep's outer rows
  int k = 0;
  if (nb > ns && nb >= 2) {
    it.part[k] = big, it.begin[k] = 0, it.end[k] = nb / 2, ++k;
    it.part[k] = big, it.begin[k] = nb / 2, it.end[k] = nb, ++k;
  } else {
    it.part[k] = big, it.begin[k] = 0, it.end[k] = nb, ++k;
  }
  it.part[k] = 1 - big, it.begin[k] = 0, it.end[k] = ns, ++k;
  *count = k;
  return it;
}

// cnt[k] = #{d : c[d] <= k}, the number of sites feeding hidden unit k's W1 column and
// below (c non-decreasing: an upper bound by bisection).
__global__ void sr_limits_kernel(const int32_t* __restrict__ c, int n, int h, int32_t* __restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= h) return;
  int lo = 0, hi = n;  // first d with c[d] > k lies in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] <= k)
      lo = mid + 1;
    else
      hi = mid;
  }
  cnt[k] = lo;
}

// ---------------------------------------------------------------- BF16: segments on MFMA
// Segment table of c (one workgroup): seg_start[j] (first site), seg_gamma[j] = c of the
// segment, seg_choff[j] = first 16-site chunk (SG_C sites) of segment j in the padded copy
// (seg_choff[nseg] = chunks in all), tab[0] = nseg.  Then sr_seg_inv_kernel: inv[p] = site at
// padded position p, or -1.
constexpr int SG_T = 1024;
constexpr int SG_C = 16;  // sites per chunk of the padded copies (the K of one MFMA)
// exclusive prefix sum over the workgroup: within each wave by shuffles, then the waves' totals
// through LDS (sh: SG_T / 64 ints); total = the workgroup's sum
__device__ inline int block_excl_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < SG_T / 64; ++q) {
    const int sq = sh[q];
    off += (q < wv) ? sq : 0;
    tot += sq;
  }
  total = tot;
  __syncthreads();
  return off + x - v;
}

__global__ __launch_bounds__(SG_T) void sr_seg_prep_kernel(const int32_t* __restrict__ c, int n,
                                                           int32_t* __restrict__ seg_start,
                                                           int32_t* __restrict__ seg_gamma,
                                                           int32_t* __restrict__ seg_choff, int32_t* __restrict__ tab) {
  __shared__ int sh[SG_T / 64];
  const int t = threadIdx.x;
  int base = 0;
  for (int d0 = 0; d0 < n; d0 += SG_T) {
    const int d = d0 + t;
    const int st = (d < n && (d == 0 || c[d] != c[d - 1])) ? 1 : 0;
    int tot;
    const int ex = block_excl_scan(st, sh, tot);
    if (st) seg_start[base + ex] = d;
    base += tot;
  }
  const int nseg = base;
  __syncthreads();
  base = 0;
  for (int j0 = 0; j0 < nseg; j0 += SG_T) {
    const int j = j0 + t;
    int ch = 0;
    if (j < nseg) {
      const int len = ((j + 1 < nseg) ? seg_start[j + 1] : n) - seg_start[j];
      ch = (len + SG_C - 1) / SG_C;
      seg_gamma[j] = c[seg_start[j]];
    }
    int tot;
    const int ex = block_excl_scan(ch, sh, tot);
    if (j < nseg) seg_choff[j] = base + ex;
    base += tot;
  }
  if (t == 0) {
    seg_choff[nseg] = base;
    tab[0] = nseg;
  }
}

// Thread j < nseg writes the padded positions of segment j and the descriptors of its chunks;
// thread i writes -1 at position i when i lies past the last segment's chunks (up to npos).
// Chunk descriptor: the segment's gamma on its first chunk, else SG_NOTFIRST; | SG_LAST on
// its last chunk.
constexpr int32_t SG_NOTFIRST = (1 << 30) - 1, SG_LAST = 1 << 30;
__global__ void sr_seg_inv_kernel(const int32_t* __restrict__ seg_start, const int32_t* __restrict__ seg_gamma,
                                  const int32_t* __restrict__ seg_choff, const int32_t* __restrict__ tab, int n,
                                  int64_t npos, int32_t* __restrict__ inv, int32_t* __restrict__ cinfo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nseg = tab[0];
  const int64_t used = (int64_t)seg_choff[nseg] * SG_C;
  if (i >= used && i < npos) inv[i] = -1;
  if (i < nseg) {
    const int j = (int)i;
    const int s0 = seg_start[j], len = ((j + 1 < nseg) ? seg_start[j + 1] : n) - s0;
    const int q0 = seg_choff[j], q1 = seg_choff[j + 1];
    const int64_t p0 = (int64_t)q0 * SG_C, p1 = (int64_t)q1 * SG_C;
    for (int64_t p = p0; p < p1; ++p) inv[p] = (p - p0 < len) ? s0 + (int)(p - p0) : -1;
    for (int q = q0; q < q1; ++q) cinfo[q] = (q == q0 ? seg_gamma[j] : SG_NOTFIRST) | (q + 1 == q1 ? SG_LAST : 0);
  }
}

// Segment-padded copies, chunk-major (the SG_C positions of chunk q of sample b at
// (q B + b) SG_C, so that one MFMA operand's 16 samples are 512 contiguous bytes):
// Gs = G[b][inv[p]], Ss = s_b,inv[p] (BF16 +-1), 0 where inv[p] < 0.
__device__ inline int64_t seg_pos(int64_t b, int64_t p, int64_t B) { return ((p / SG_C) * B + b) * SG_C + p % SG_C; }
// The same copies by tiles of 16 samples x 64 chunks: the sites the tile's chunks hold (a run of
// at most 64 SG_C of them, the segments being runs) are staged in LDS for the 16 samples, and
// each chunk's 16 samples are written as one contiguous 512-byte run.  Workgroups past the last
// chunk return.
constexpr int SGP_S = 16, SGP_Q = 64, SGP_SPAN = SGP_Q * SG_C;
__global__ __launch_bounds__(256) void sr_seg_pack_tile_kernel(const bf16_t* __restrict__ G,
                                                               const int8_t* __restrict__ S, int64_t ldn,
                                                               const int32_t* __restrict__ inv,
                                                               const int32_t* __restrict__ seg_choff,
                                                               const int32_t* __restrict__ tab, int64_t B,
                                                               bf16_t* __restrict__ Gs, bf16_t* __restrict__ Ss) {
  __shared__ __align__(16) bf16_t gl[SGP_S][SGP_SPAN + 16];
  __shared__ __align__(16) int8_t sl[SGP_S][SGP_SPAN + 32];
  const int t = threadIdx.x;
  const int nch = seg_choff[tab[0]];
  const int q0 = blockIdx.x * SGP_Q;
  if (q0 >= nch) return;
  const int q1 = min(q0 + SGP_Q, nch);
  const int64_t b0 = (int64_t)blockIdx.y * SGP_S;
  // sites of the tile: from the first position (a chunk's first position always holds a site) to
  // the last valid one (a chunk holds at least one site)
  const int s_lo = inv[(int64_t)q0 * SG_C];
  int p = q1 * SG_C - 1;
  while (inv[p] < 0) --p;
  const int s_hi = inv[p];  // s_hi - s_lo < SGP_SPAN
  // 16-byte pieces from 16-byte boundaries (rows of ld(n) elements: the last piece stays inside)
  const int ga = s_lo & ~7, sa = s_lo & ~15;
  const int gpieces = (s_hi - ga) / 8 + 1, spieces = (s_hi - sa) / 16 + 1;
  for (int e = t; e < SGP_S * gpieces; e += 256) {
    const int r = e / gpieces, k = e - r * gpieces;
    const int64_t b = b0 + r;
    *(uint4*)&gl[r][8 * k] = (b < B) ? *(const uint4*)(G + b * ldn + ga + 8 * k) : make_uint4(0, 0, 0, 0);
  }
  for (int e = t; e < SGP_S * spieces; e += 256) {
    const int r = e / spieces, k = e - r * spieces;
    const int64_t b = b0 + r;
    *(uint4*)&sl[r][16 * k] = (b < B) ? *(const uint4*)(S + b * ldn + sa + 16 * k) : make_uint4(0, 0, 0, 0);
  }
  __syncthreads();
  // thread t: chunk q0 + (t / 32) + 8 i, sample t / 2 % 16, half t % 2 (eight positions)
  const int r = (t >> 1) & (SGP_S - 1), h = t & 1;
  const int64_t b = b0 + r;
  for (int q = q0 + (t >> 5); q < q1; q += 8) {
    const int64_t pp = (int64_t)q * SG_C + 8 * h;
    bf16_t gv[8], sv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int d = inv[pp + e];
      gv[e] = d >= 0 ? gl[r][d - ga] : (bf16_t)0;
      const int sg = d >= 0 ? sl[r][d - sa] : 0;
      sv[e] = sg > 0 ? (bf16_t)0x3F80 : (sg < 0 ? (bf16_t)0xBF80 : (bf16_t)0);
    }
    if (b < B) {
      *(uint4*)(Gs + seg_pos(b, pp, B)) = *(const uint4*)gv;
      *(uint4*)(Ss + seg_pos(b, pp, B)) = *(const uint4*)sv;
    }
  }
}

// One 64 x 64 tile of K (on or above the diagonal) per workgroup of four waves, each wave a
// 32 x 32 quadrant as 2 x 2 MFMA blocks (v_mfma_f32_16x16x16_bf16, one 16-site chunk per
// product; lane (lr, lg) holds the entries (4 lg + e, lr) of each block).  F = 1 + the RR'
// prefix, F2 = 1 + the ss' prefix, acc = K.  The chunks of the padded copies stream through a
// ring of GM_RING register sets (loaded GM_RING chunks ahead); the units' R and D rows come
// through LDS panels of GM_PR units.  Workgroups are dealt round-robin to the 8 XCDs; each
// XCD takes a contiguous run of the tile order, so that its tiles share row tiles in its L2.
constexpr int GM_PR = 64;
constexpr int GM_RING = 4;
struct GmFrag {
  uint2 ga[2], gb[2], sa[2], sb[2];
  int32_t info;  // the chunk's descriptor (same in every lane)
};
typedef __attribute__((ext_vector_type(4))) short gm_bf16x4_t;

__global__ __launch_bounds__(256) void sr_gram_mfma_kernel(const bf16_t* __restrict__ Gs, const bf16_t* __restrict__ Ss,
                                                           int64_t ldk, const bf16_t* __restrict__ Rt,
                                                           const bf16_t* __restrict__ Dt, int64_t ldb,
                                                           const int32_t* __restrict__ cinfo,
                                                           const int32_t* __restrict__ seg_choff,
                                                           const int32_t* __restrict__ tab, int h, int64_t B, int nt,
                                                           float* __restrict__ K) {
  __shared__ __align__(16) float pr[GM_PR][2 * GR_T];
  __shared__ __align__(16) float pd[GM_PR][2 * GR_T];
  int ti, tj;
  {
    const int w = blockIdx.x, G = gridDim.x, x = w & 7, q = G >> 3, r = G & 7;
    upper_tile(x * q + min(x, r) + (w >> 3), nt, ti, tj);
  }
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int64_t b0 = (int64_t)ti * GR_T, b1 = (int64_t)tj * GR_T;
  int64_t ra[2], rb[2];  // fragment rows, clamped (results of rows >= B are never stored)
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    ra[i] = min(b0 + wm + 16 * i + lr, B - 1) * SG_C + 4 * lg;
    rb[i] = min(b1 + wn + 16 * i + lr, B - 1) * SG_C + 4 * lg;
  }
  floatx4_t acc[2][2], F[2][2], F2[2][2], X[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
      F[i][j] = (floatx4_t){1.f, 1.f, 1.f, 1.f};
      F2[i][j] = (floatx4_t){1.f, 1.f, 1.f, 1.f};
      X[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    }
  const int nseg = __builtin_amdgcn_readfirstlane(tab[0]);
  const int nch = __builtin_amdgcn_readfirstlane(seg_choff[nseg]);
  int unit = 0;                             // units [0, unit) are in F and acc
  int pbase = -GM_PR;

  auto load = [&](GmFrag& f, int q) {
    const int qc = min(q, max(nch - 1, 0));
    const int64_t ko = (int64_t)qc * B * SG_C;
    f.info = cinfo[qc];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      f.ga[i] = *(const uint2*)(Gs + ra[i] + ko);
      f.gb[i] = *(const uint2*)(Gs + rb[i] + ko);
      f.sa[i] = *(const uint2*)(Ss + ra[i] + ko);
      f.sb[i] = *(const uint2*)(Ss + rb[i] + ko);
    }
  };
  // unit u: F += RR'_u, acc += DD'_u (.) F2 (F2 holds the segments with gamma <= u)
  auto units_to = [&](int uend) {
    for (; unit < uend; ++unit) {
      if (unit >= pbase + GM_PR) {
        __syncthreads();
#pragma unroll
        for (int half = 0; half < GM_PR / 32; ++half) {
          const int r = 32 * half + (t >> 3), seg8 = t & 7;  // 8 threads per row, 16 samples each
          if (unit + r < h) {
            const int64_t col = (seg8 < 4 ? b0 : b1) + 16 * (seg8 & 3);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              float v[4];
              load4<bf16_t>(Rt + (int64_t)(unit + r) * ldb + col + 4 * q, v);
              *(float4*)&pr[r][16 * seg8 + 4 * q] = make_float4(v[0], v[1], v[2], v[3]);
              load4<bf16_t>(Dt + (int64_t)(unit + r) * ldb + col + 4 * q, v);
              *(float4*)&pd[r][16 * seg8 + 4 * q] = make_float4(v[0], v[1], v[2], v[3]);
            }
          }
        }
        pbase = unit;
        __syncthreads();
      }
      const float* r = pr[unit - pbase];
      const float* d = pd[unit - pbase];
      float4 r4[2], d4[2];
      float rc[2], dc[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        r4[i] = *(const float4*)(r + wm + 16 * i + 4 * lg);
        d4[i] = *(const float4*)(d + wm + 16 * i + 4 * lg);
        rc[i] = r[GR_T + wn + 16 * i + lr];
        dc[i] = d[GR_T + wn + 16 * i + lr];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float ri[4] = {r4[i].x, r4[i].y, r4[i].z, r4[i].w};
          const float di[4] = {d4[i].x, d4[i].y, d4[i].z, d4[i].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            F[i][j][e] = fmaf(ri[e], rc[j], F[i][j][e]);
            acc[i][j][e] = fmaf(di[e] * dc[j], F2[i][j][e], acc[i][j][e]);
          }
        }
    }
  };
  // chunk q (of segment seg): before its first chunk, the units below its gamma; then the
  // products; after its last chunk, X (.) F into acc
  auto step = [&](const GmFrag& f, int q) {
    (void)q;
    const int info = __builtin_amdgcn_readfirstlane(f.info);
    const int gamma = info & SG_NOTFIRST;
    if (gamma != SG_NOTFIRST) {
      units_to(min(gamma, h));
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) X[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        X[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(gm_bf16x4_t, f.ga[i]),
                                                             __builtin_bit_cast(gm_bf16x4_t, f.gb[j]), X[i][j], 0, 0, 0);
        F2[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(gm_bf16x4_t, f.sa[i]),
                                                              __builtin_bit_cast(gm_bf16x4_t, f.sb[j]), F2[i][j], 0, 0, 0);
      }
    if (info & SG_LAST) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[i][j][e] = fmaf(X[i][j][e], F[i][j][e], acc[i][j][e]);
    }
  };
  GmFrag f[GM_RING];
#pragma unroll
  for (int p = 0; p < GM_RING; ++p) load(f[p], p);
  int q = 0;
  for (; q + GM_RING <= nch; q += GM_RING) {
#pragma unroll
    for (int p = 0; p < GM_RING; ++p) {
      step(f[p], q + p);
      load(f[p], q + p + GM_RING);
    }
  }
#pragma unroll
  for (int p = 0; p < GM_RING - 1; ++p)
    if (q + p < nch) step(f[p], q + p);
  units_to(h);

  // K[row][col] and its mirror; on a diagonal tile only the entries with row <= col
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = b0 + wm + 16 * i + 4 * lg + e, col = b1 + wn + 16 * j + lr;
        if (row < B && col < B && (ti < tj || row <= col)) {
          K[row * B + col] = acc[i][j][e];
          K[col * B + row] = acc[i][j][e];
        }
      }
}

// BF16 scratch: the segment table and the padded copies
struct SegLayout {
  int64_t kpmax, ldk;  // chunks at most; row length of the padded copies
  size_t start, gamma, choff, tab, inv, cinfo, gs, ss, total;
};
static SegLayout seg_layout(int n, int h, int64_t B) {
  SegLayout L;
  L.kpmax = (n + SG_C - 1) / SG_C + min(n, h + 1);
  L.ldk = L.kpmax * SG_C;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up((int64_t)bytes, 256);
    return o;
  };
  L.start = take((size_t)n * 4);
  L.gamma = take((size_t)n * 4);
  L.choff = take((size_t)(n + 1) * 4);
  L.tab = take(16);
  L.inv = take((size_t)L.ldk * 4);
  L.cinfo = take((size_t)L.kpmax * 4);
  L.gs = take((size_t)B * L.ldk * 2);
  L.ss = take((size_t)B * L.ldk * 2);
  L.total = off;
  return L;
}

size_t sr_gram_parts_bytes(int n, int h, int64_t B, int dtype) {
  if (dtype == VQMC_BF16) return seg_layout(n, h, B).total;
  return (size_t)GR_ITEMS * B * B * 4 + (size_t)round_up((int64_t)h * 4, 256);
}

static hipError_t launch_sr_gram_mfma(const bf16_t* G, const int8_t* S, int64_t ldn, const bf16_t* Rt,
                                      const bf16_t* Dt, int64_t ldb, const int32_t* c, int n, int h, int64_t B,
                                      void* scratch, float* K, hipStream_t st) {
  const SegLayout L = seg_layout(n, h, B);
  uint8_t* w = (uint8_t*)scratch;
  int32_t* start = (int32_t*)(w + L.start);
  int32_t* gamma = (int32_t*)(w + L.gamma);
  int32_t* choff = (int32_t*)(w + L.choff);
  int32_t* tab = (int32_t*)(w + L.tab);
  int32_t* inv = (int32_t*)(w + L.inv);
  int32_t* cinfo = (int32_t*)(w + L.cinfo);
  bf16_t* Gs = (bf16_t*)(w + L.gs);
  bf16_t* Ss = (bf16_t*)(w + L.ss);
  sr_seg_prep_kernel<<<1, SG_T, 0, st>>>(c, n, start, gamma, choff, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t ninv = std::max<int64_t>(n, L.ldk);
  sr_seg_inv_kernel<<<(unsigned)((ninv + 255) / 256), 256, 0, st>>>(start, gamma, choff, tab, n, L.ldk, inv, cinfo);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 pgrid((unsigned)((L.kpmax + SGP_Q - 1) / SGP_Q), (unsigned)((B + SGP_S - 1) / SGP_S));
  sr_seg_pack_tile_kernel<<<pgrid, 256, 0, st>>>(G, S, ldn, inv, choff, tab, B, Gs, Ss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nt = (int)((B + GR_T - 1) / GR_T);
  const int64_t pairs = (int64_t)nt * (nt + 1) / 2;
  sr_gram_mfma_kernel<<<(unsigned)pairs, 256, 0, st>>>(Gs, Ss, L.ldk, Rt, Dt, ldb, cinfo, choff, tab, h, B, nt, K);
  return hipGetLastError();
}

hipError_t launch_sr_gram_sweeps(int dtype, const void* Gt, const void* Rt, const void* Dt, const void* St,
                                 int64_t ldb, const int32_t* c, int n, int h, int64_t B, float* parts, float* K,
                                 hipStream_t st, const void* G, const int8_t* S, int64_t ldn) {
  if (dtype == VQMC_BF16)
    return launch_sr_gram_mfma((const bf16_t*)G, S, ldn, (const bf16_t*)Rt, (const bf16_t*)Dt, ldb, c, n, h, B,
                               parts, K, st);
  int32_t* cnt = (int32_t*)(parts + (int64_t)GR_ITEMS * B * B);
  sr_limits_kernel<<<(unsigned)((h + 255) / 256), 256, 0, st>>>(c, n, h, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nt = (int)((B + GR_T - 1) / GR_T);
  const int64_t pairs = (int64_t)nt * (nt + 1) / 2;
  if (pairs > 0x7FFFFFFF) return hipErrorInvalidValue;
  int nitems = 0;
  const GramItems items = gram_items(n, h, &nitems);
  const dim3 grid((unsigned)pairs, (unsigned)nitems);
  sr_gram_kernel<float><<<grid, 256, 0, st>>>((const float*)Gt, (const float*)Rt, (const float*)Dt,
                                              (const float*)St, ldb, c, cnt, n, h, B, nt, items, parts);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = B * B;
  sr_gram_combine_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(parts, nitems, B, K);
  return hipGetLastError();
}

}  // namespace vqmc
