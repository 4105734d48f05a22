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
// This is elementwise FP32 work, not a contraction: every Gram entry carries its own
// running prefix.  Each workgroup owns a 64 x 64 tile (tiles on or above the diagonal
// only; K is symmetric) of one work item, a range of one sweep; the factor rows are
// batch-contiguous (X[j][b], ld(B) columns) and reach the tile through LDS panels of rows.  A combine pass adds the items' partial sums in a fixed
// order and mirrors the upper tiles.
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

size_t sr_gram_parts_bytes(int64_t B, int h) {
  return (size_t)GR_ITEMS * B * B * 4 + (size_t)round_up((int64_t)h * 4, 256);
}

hipError_t launch_sr_gram_sweeps(int dtype, const void* Gt, const void* Rt, const void* Dt, const void* St,
                                 int64_t ldb, const int32_t* c, int n, int h, int64_t B, float* parts, float* K,
                                 hipStream_t st) {
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
  if (dtype == VQMC_BF16)
    sr_gram_kernel<bf16_t><<<grid, 256, 0, st>>>((const bf16_t*)Gt, (const bf16_t*)Rt, (const bf16_t*)Dt,
                                                 (const bf16_t*)St, ldb, c, cnt, n, h, B, nt, items, parts);
  else
    sr_gram_kernel<float><<<grid, 256, 0, st>>>((const float*)Gt, (const float*)Rt, (const float*)Dt,
                                                (const float*)St, ldb, c, cnt, n, h, B, nt, items, parts);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = B * B;
  sr_gram_combine_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(parts, nitems, B, K);
  return hipGetLastError();
}

}  // namespace vqmc
