// The B x B solve of stochastic reconfiguration on the device (Sec. 2.1: natural gradient
// with the Fisher information of the per-sample scores; Sec. 5.1: SR with a ridge lambda).
// In sample space the SR direction for the batch gradient g = O^T c is x = O^T y with
//
//     (K + lambda B I) y = B c,      K = O O^T   (symmetric positive semi-definite),
//
// so the only dense linear algebra is this B x B system.  It is solved in FP64 by a blocked
// right-looking Cholesky factorisation L L^T = K + shift I (64 x 64 blocks, the matrix padded
// to a multiple of 64 with identity rows), the forward substitution L w = rhs folded into the
// factorisation, and a blocked back substitution L^T y = w.
//
// Launches per block column j (nb = padded B / 64 of them):
//   chol_trsm_kernel    nb - j - 1 workgroups of one wave: workgroup i - 1 solves its block row
//                       L_{j+i,j} = A_{j+i,j} L_jj^-T and updates w_{j+i} -= L_{j+i,j} w_j;
//   chol_update_kernel  one workgroup per block (i, k), j < k <= i: A_ik -= L_ij L_kj^T; the one
//                       on block (j + 1, j + 1) then factors it with one wave, a row per lane in
//                       registers, with the forward substitution of w_{j+1}, and stores L and w
//                       (the first diagonal block: chol_factor_kernel).
// and, from the last block column to the first,
//   chol_back_kernel    max(j, 1) workgroups: each solves L_jj^T y_j = w_j (workgroup 0
//                       stores y_j), workgroup i < j updates w_i -= L_ji^T y_j.
// The work is O(B^3 / 3) FP64 multiply-adds, a few milliseconds of vector FP64 at most for
// the batch sizes of the paper; the launches are latency-bound, not flop-bound.
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

constexpr int CB = 64;  // block edge

// A = K + shift I on the B x B part, identity on the padding; w = scale * rhs (0 on padding).
__global__ void chol_init_kernel(const float* __restrict__ K, int64_t B, int64_t ld, double shift,
                                 const float* __restrict__ rhs, double scale, double* __restrict__ A,
                                 double* __restrict__ w) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ld * ld) return;
  const int64_t r = idx / ld, c = idx - r * ld;
  double v;
  if (r < B && c < B) v = (double)K[r * B + c] + (r == c ? shift : 0.0);
  else v = (r == c) ? 1.0 : 0.0;
  A[idx] = v;
  if (idx < ld) w[idx] = (idx < B) ? scale * (double)rhs[idx] : 0.0;
}

// The panel runs on one wave per workgroup.  Lane r holds row r of the 64 x 64 diagonal block
// in registers and the block is factored right-looking, one column after another: column c's
// diagonal entry comes from lane c, the lanes below scale their entry and write it to row c of
// Lt (so that Lt[c][r] = L[r][c]), every lane reads the entries below c back as broadcasts and
// updates its entries right of c.  The column loops are unrolled, so a row stays in registers,
// and one wave needs no barriers: the only chain is the sequence of columns.  The block-row
// solve X L^T = A_ij runs the same way, a row of X per lane, reading L from Lt.
constexpr int CL = CB + 2;  // LDS row stride (doubles): 16-byte aligned rows
// groups of eight LDS reads in flight ahead of the multiply-adds of the column loops (depths of one to
// four give the same time within 1 %)
constexpr int CHOL_PF = 2;

// 1 / sqrt(d): the hardware estimate refined by two Newton steps r <- r (3 - d r^2) / 2, each
// roughly doubling the correct bits of the estimate (about 23 of them), so the result is accurate
// to a few ulp of double precision; NaN for d < 0, +inf for d = 0.
__device__ inline double chol_rsqrt(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * fma(-0.5 * d, r * r, 1.5);
  r = r * fma(-0.5 * d, r * r, 1.5);
  return r;
}

__device__ inline double chol_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// A[r0 .. r0 + 64)[c0 .. c0 + 64) into T (row-major, stride CL), one wave: two rows per 16-byte
// load instruction, all 32 loads issued before the first store to LDS (one memory round trip)
__device__ inline void chol_load_tile(const double* __restrict__ A, int64_t ld, int64_t r0, int64_t c0,
                                      double (*T)[CL]) {
  const int l = threadIdx.x, rh = l >> 5, cq = 2 * (l & 31);
  double2 v[CB / 2];
#pragma unroll
  for (int i = 0; i < CB / 2; ++i) v[i] = *(const double2*)(A + (r0 + 2 * i + rh) * ld + c0 + cq);
#pragma unroll
  for (int i = 0; i < CB / 2; ++i) *(double2*)&T[2 * i + rh][cq] = v[i];
}

// x[c2] -= xc * row[c2] for c2 in (c, CB): the row read from LDS in groups of eight, PF groups
// ahead of the multiply-adds (a ring of PF + 1 groups in registers), with compiler memory barriers
// between the groups so that the reads of later groups are not hoisted further (their registers
// would not fit).
template <int PF>
__device__ __attribute__((always_inline)) inline void chol_axpy_tail(double (&x)[CB], int c, double xc, const double* row) {
  constexpr int G = 8;
  double v[PF + 1][G];
#pragma unroll
  for (int q = 0; q < PF; ++q)
#pragma unroll
    for (int e = 0; e < G; ++e) v[q][e] = (c + 1 + G * q + e < CB) ? row[c + 1 + G * q + e] : 0.0;
#pragma unroll
  for (int q = 0; c + 1 + G * q < CB; ++q) {
    const int g0 = c + 1 + G * q, gn = g0 + G * PF;
#pragma unroll
    for (int e = 0; e < G; ++e)
      if (gn + e < CB) v[(q + PF) % (PF + 1)][e] = row[gn + e];
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < G; ++e)
      if (g0 + e < CB) x[g0 + e] = fma(-xc, v[q % (PF + 1)][e], x[g0 + e]);
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Diagonal block of column j, one wave: the block in T (row-major, stride CL), L_jj back into A
// (lower triangle) and w_j' = L_jj^-1 w_j into w.  Lt: scratch for the columns of L.
__device__ __attribute__((always_inline)) inline void chol_factor_wave(const double (*T)[CL], double (*Lt)[CL],
                                                                      double* __restrict__ A, int64_t ld,
                                                                      int64_t j0, double* __restrict__ w) {
  const int l = threadIdx.x;
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = T[l][c];
  double wv = w[j0 + l];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const double d = chol_bcast(x[c], c);
    const double rs = chol_rsqrt(d);              // NaN if the block is not positive definite
    x[c] = (l == c) ? d * rs : ((l > c) ? x[c] * rs : 0.0);
    Lt[c][l] = x[c];
    const double wc = chol_bcast(wv, c) * rs;     // w'_c
    if (l == c) wv = wc;
    else if (l > c) wv = fma(-x[c], wc, wv);
    chol_axpy_tail<CHOL_PF>(x, c, x[c], Lt[c]);
  }
  // rows coalesced from Lt
#pragma unroll 8
  for (int r = 0; r < CB; ++r)
    if (l <= r) A[(j0 + r) * ld + j0 + l] = Lt[l][r];
  w[j0 + l] = wv;
}

// The first diagonal block (the later ones are factored by chol_update_kernel).
__global__ __launch_bounds__(CB) void chol_factor_kernel(double* __restrict__ A, int64_t ld, int j,
                                                         double* __restrict__ w) {
  __shared__ __align__(16) double T[CB][CL];
  __shared__ __align__(16) double Lt[CB][CL];
  const int64_t j0 = (int64_t)j * CB;
  chol_load_tile(A, ld, j0, j0, T);
  chol_factor_wave(T, Lt, A, ld, j0, w);
}

// Block row i of column j (workgroup i - 1, i > j): X L_jj^T = A_ij, a row of X per lane, with L_jj
// read back from A into Lt; then w_i -= X w_j'.
__global__ __launch_bounds__(CB) void chol_trsm_kernel(double* __restrict__ A, int64_t ld, int j,
                                                       double* __restrict__ w) {
  __shared__ __align__(16) double T[CB][CL];   // A_ij; X on the way out
  __shared__ __align__(16) double Lt[CB][CL];  // Lt[c][r] = L[r][c]
  __shared__ double rdl[CB];                   // 1 / L[c][c]
  __shared__ double wl[CB];                    // w_j'
  const int l = threadIdx.x;
  const int64_t j0 = (int64_t)j * CB, i0 = j0 + (int64_t)(blockIdx.x + 1) * CB;
  chol_load_tile(A, ld, j0, j0, T);
#pragma unroll 8
  for (int c = 0; c < CB; ++c) Lt[c][l] = (l >= c) ? T[l][c] : 0.0;
  rdl[l] = 1.0 / T[l][l];
  wl[l] = w[j0 + l];
  chol_load_tile(A, ld, i0, j0, T);
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = T[l][c];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    x[c] *= rdl[c];
    chol_axpy_tail<CHOL_PF>(x, c, x[c], Lt[c]);
  }
  double sdot = 0.0;
#pragma unroll
  for (int c = 0; c < CB; ++c) sdot = fma(x[c], wl[c], sdot);
  w[i0 + l] -= sdot;
#pragma unroll
  for (int c = 0; c < CB; ++c) T[c][l] = x[c];
#pragma unroll 8
  for (int r = 0; r < CB; ++r) A[(i0 + r) * ld + j0 + l] = T[l][r];
}

// Trailing update of block column j: A_ik -= L_ij L_kj^T for j < k <= i (the lower
// triangle of the trailing matrix; blockIdx.x enumerates its blocks row by row).  Workgroup 0
// updates the next diagonal block (j + 1, j + 1), keeps it in LDS and factors it with its first
// wave (chol_factor_wave), so that the next block column starts with its block-row solves.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, int64_t ld, int j,
                                                          double* __restrict__ w) {
  __shared__ __align__(16) double Li[CB][CL];
  __shared__ __align__(16) double Lk[CB][CL];
  int ii = 0, rem = blockIdx.x;
  while (rem > ii) {  // row ii holds ii + 1 blocks
    rem -= ii + 1;
    ++ii;
  }
  const int kk = rem;
  const int64_t j0 = (int64_t)j * CB, i0 = j0 + (int64_t)(ii + 1) * CB, k0 = j0 + (int64_t)(kk + 1) * CB;
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  // both blocks with 16-byte loads and the block being updated, all issued before the first
  // store to LDS (one memory round trip); the two blocks are stored transposed (Li[c][r] =
  // L_ij[r][c]), so that the products read four consecutive rows of a column at once
  const int rq = t >> 5, cq = 2 * (t & 31);  // rows rq + 8 i, columns cq, cq + 1
  double2 vi[CB / 8], vk[CB / 8];
#pragma unroll
  for (int i = 0; i < CB / 8; ++i) {
    vi[i] = *(const double2*)(A + (i0 + rq + 8 * i) * ld + j0 + cq);
    vk[i] = *(const double2*)(A + (k0 + rq + 8 * i) * ld + j0 + cq);
  }
  double av0[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double4 q = *(const double4*)(A + (i0 + 4 * ty + a) * ld + k0 + 4 * tx);
    av0[a][0] = q.x; av0[a][1] = q.y; av0[a][2] = q.z; av0[a][3] = q.w;
  }
#pragma unroll
  for (int i = 0; i < CB / 8; ++i) {
    Li[cq][rq + 8 * i] = vi[i].x;
    Li[cq + 1][rq + 8 * i] = vi[i].y;
    Lk[cq][rq + 8 * i] = vk[i].x;
    Lk[cq + 1][rq + 8 * i] = vk[i].y;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
  for (int c = 0; c < CB; ++c) {
    const double2 a01 = *(const double2*)&Li[c][4 * ty], a23 = *(const double2*)&Li[c][4 * ty + 2];
    const double2 b01 = *(const double2*)&Lk[c][4 * tx], b23 = *(const double2*)&Lk[c][4 * tx + 2];
    const double av[4] = {a01.x, a01.y, a23.x, a23.y}, bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
  }
  double nv[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) nv[a][b] = av0[a][b] - acc[a][b];
  if (blockIdx.x != 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
      *(double4*)(A + (i0 + 4 * ty + a) * ld + k0 + 4 * tx) = make_double4(nv[a][0], nv[a][1], nv[a][2], nv[a][3]);
    return;
  }
  // the next diagonal block: the updated values into LDS (Li is free once every thread has its
  // products), then its factorisation by the first wave
  __syncthreads();
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) Li[4 * ty + a][4 * tx + b] = nv[a][b];
  __syncthreads();
  if (t < CB) chol_factor_wave(Li, Lk, A, ld, i0, w);
}

// Back substitution of block j: L_jj^T y_j = w_j, then workgroup i < j applies
// w_i -= L_ji^T y_j.  Lane c holds column c of L_jj; y is found from the last row up, each new
// y_r passed to the other lanes through LDS (every workgroup solves the block, the same
// arithmetic, so the copies agree bit for bit).
__global__ __launch_bounds__(64) void chol_back_kernel(const double* __restrict__ A, int64_t ld, int j,
                                                       double* __restrict__ w, double* __restrict__ y) {
  __shared__ double yv[CB];
  const int c = threadIdx.x;
  const int64_t j0 = (int64_t)j * CB;
  double lc[CB];  // lc[r] = L[r][c] (used for r >= c)
#pragma unroll
  for (int r = 0; r < CB; ++r) lc[r] = A[(j0 + r) * ld + j0 + c];
  double acc = w[j0 + c];
#pragma unroll
  for (int r = CB - 1; r >= 0; --r) {
    if (c == r) yv[r] = acc / lc[r];
    __syncthreads();
    if (c < r) acc = fma(-lc[r], yv[r], acc);
  }
  if (blockIdx.x == 0) y[j0 + c] = yv[c];
  if (blockIdx.x >= j) return;
  // (L_ji^T y_j)[q] = sum_r L[j0 + r][i0 + q] y_j[r], lane q = c
  const int64_t i0 = (int64_t)blockIdx.x * CB;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < CB; ++r) s = fma(A[(j0 + r) * ld + i0 + c], yv[r], s);
  w[i0 + c] -= s;
}

__global__ void chol_out_kernel(const double* __restrict__ y, int64_t B, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) out[i] = (float)y[i];
}

size_t sr_solve_ws_bytes(int64_t B) {
  const int64_t ld = round_up(B, CB);
  return (size_t)round_up(ld * ld * 8, 256) + 2 * (size_t)round_up(ld * 8, 256);
}

hipError_t launch_sr_solve(const float* K, int64_t B, double shift, const float* rhs, double scale, float* y,
                           void* ws, hipStream_t st) {
  const int64_t ld = round_up(B, CB);
  const int nb = (int)(ld / CB);
  double* A = (double*)ws;
  double* w = (double*)((uint8_t*)ws + round_up(ld * ld * 8, 256));
  double* yd = (double*)((uint8_t*)w + round_up(ld * 8, 256));
  chol_init_kernel<<<(unsigned)((ld * ld + 255) / 256), 256, 0, st>>>(K, B, ld, shift, rhs, scale, A, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  chol_factor_kernel<<<1, CB, 0, st>>>(A, ld, 0, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int j = 0; j < nb; ++j) {
    // block column j: its diagonal block is factored (above, or by the previous update)
    const int m = nb - j - 1;
    if (m > 0) {
      chol_trsm_kernel<<<(unsigned)m, CB, 0, st>>>(A, ld, j, w);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      chol_update_kernel<<<(unsigned)(m * (m + 1) / 2), 256, 0, st>>>(A, ld, j, w);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  for (int j = nb - 1; j >= 0; --j) {
    chol_back_kernel<<<(unsigned)(j > 0 ? j : 1), 64, 0, st>>>(A, ld, j, w, yd);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  chol_out_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(yd, B, y);
  return hipGetLastError();
}

}  // namespace vqmc
