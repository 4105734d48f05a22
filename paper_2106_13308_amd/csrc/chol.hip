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
//   chol_panel_kernel   nb - j workgroups: each factors the diagonal block A_jj, blocked by 16
//                       columns (the same arithmetic in every workgroup, so the copies agree
//                       bit for bit);
//                       workgroup 0 stores L_jj and w_j, workgroup i > 0 solves its block row
//                       L_{j+i,j} = A_{j+i,j} L_jj^-T and updates w_{j+i} -= L_{j+i,j} w_j;
//   chol_update_kernel  one workgroup per block (i, k), j < k <= i: A_ik -= L_ij L_kj^T.
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

// The panel is blocked again inside, by 16 columns (SB): a sub-block's columns are factored one
// after another by the lanes that own its rows (a row per lane, at most 16 dependent updates
// per column, in registers), then everything to its right is brought up to date by a rank-16
// update spread over all 256 threads.  The sequential part of a 64-column panel is thus four
// short chains instead of one long one.
constexpr int SB = 16;

// Lane-per-row solve of the 16 columns [s0, s0 + SB) of one row x against the factored
// diagonal sub-block D (D[q][c], q >= c, of L): x[c] = (x[c] - sum_{c' < c} x[c'] D[c][c']) / D[c][c].
__device__ inline void chol_row_solve16(double (&x)[SB], const double (*L)[CB + 1], int s0) {
#pragma unroll
  for (int c = 0; c < SB; ++c) {
    double v = x[c];
#pragma unroll
    for (int q = 0; q < c; ++q) v = fma(-x[q], L[s0 + c][s0 + q], v);
    x[c] = v / L[s0 + c][s0 + c];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Cholesky of the diagonal block F (lower triangle, in place) with the forward substitution of
// w (in wc) folded in; 256 threads.
__device__ inline void chol_factor_block(double (*F)[CB + 1], double* wc) {
  const int t = threadIdx.x;
  for (int s0 = 0; s0 < CB; s0 += SB) {
    // the diagonal sub-block: one lane per row, its 16 entries factored column by column
    if (t < SB) {
      const int r = s0 + t;
      for (int c = 0; c < SB; ++c) {
        const int cc = s0 + c;
        if (t == c) {
          double v = F[cc][cc];
          for (int q = s0; q < cc; ++q) v = fma(-F[cc][q], F[cc][q], v);
          F[cc][cc] = sqrt(v);  // NaN if the block is not positive definite
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        if (t > c) {
          double v = F[r][cc];
          for (int q = s0; q < cc; ++q) v = fma(-F[r][q], F[cc][q], v);
          F[r][cc] = v / F[cc][cc];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
      }
      // forward substitution of the sub-block's part of w
      for (int c = 0; c < SB; ++c) {
        const int cc = s0 + c;
        if (t == c) {
          double v = wc[cc];
          for (int q = s0; q < cc; ++q) v = fma(-F[cc][q], wc[q], v);
          wc[cc] = v / F[cc][cc];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    // rows below the sub-block: their 16 entries of these columns, a row per thread
    const int r = s0 + SB + t;
    if (t < CB - s0 - SB) {
      double x[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c) x[c] = F[r][s0 + c];
      chol_row_solve16(x, F, s0);
#pragma unroll
      for (int c = 0; c < SB; ++c) F[r][s0 + c] = x[c];
    }
    __syncthreads();
    // rank-16 update of the trailing lower triangle and of the rest of w
    const int m = CB - s0 - SB;
    for (int e = t; e < m * m; e += 256) {
      const int rr = e / m, qq = e - rr * m;
      if (qq <= rr) {
        const int r2 = s0 + SB + rr, q2 = s0 + SB + qq;
        double v = F[r2][q2];
#pragma unroll
        for (int c = 0; c < SB; ++c) v = fma(-F[r2][s0 + c], F[q2][s0 + c], v);
        F[r2][q2] = v;
      }
    }
    if (t < m) {
      const int r2 = s0 + SB + t;
      double v = wc[r2];
#pragma unroll
      for (int c = 0; c < SB; ++c) v = fma(-F[r2][s0 + c], wc[s0 + c], v);
      wc[r2] = v;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ A, int64_t ld, int j,
                                                         double* __restrict__ w) {
  __shared__ double F[CB][CB + 1];
  __shared__ double X[CB][CB + 1];
  __shared__ double wc[CB];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)j * CB;
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    F[r][c] = A[(j0 + r) * ld + j0 + c];
  }
  if (t < CB) wc[t] = w[j0 + t];
  __syncthreads();
  chol_factor_block(F, wc);
  if (blockIdx.x == 0) {
    for (int e = t; e < CB * CB; e += 256) {
      const int r = e >> 6, c = e & (CB - 1);
      if (c <= r) A[(j0 + r) * ld + j0 + c] = F[r][c];
    }
    if (t < CB) w[j0 + t] = wc[t];
    return;
  }
  // block row i0 = j0 + 64 blockIdx.x: X L_jj^T = A_ij, blocked by 16 columns like the factor
  const int64_t i0 = j0 + (int64_t)blockIdx.x * CB;
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    X[r][c] = A[(i0 + r) * ld + j0 + c];
  }
  __syncthreads();
  for (int s0 = 0; s0 < CB; s0 += SB) {
    if (t < CB) {
      double x[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c) x[c] = X[t][s0 + c];
      chol_row_solve16(x, F, s0);
#pragma unroll
      for (int c = 0; c < SB; ++c) X[t][s0 + c] = x[c];
    }
    __syncthreads();
    const int m = CB - s0 - SB;  // X[:, later] -= X[:, sub-block] L[later, sub-block]^T
    for (int e = t; e < CB * m; e += 256) {
      const int r = e / m, q2 = s0 + SB + (e - (e / m) * m);
      double v = X[r][q2];
#pragma unroll
      for (int c = 0; c < SB; ++c) v = fma(-X[r][s0 + c], F[q2][s0 + c], v);
      X[r][q2] = v;
    }
    __syncthreads();
  }
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    A[(i0 + r) * ld + j0 + c] = X[r][c];
  }
  if (t < CB) {
    double s = 0.0;  // (X w_j)[t], w_j the block's substituted values
    for (int c = 0; c < CB; ++c) s = fma(X[t][c], wc[c], s);
    w[i0 + t] -= s;
  }
}

// Trailing update of block column j: A_ik -= L_ij L_kj^T for j < k <= i (the lower
// triangle of the trailing matrix; blockIdx.x enumerates its blocks row by row).
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, int64_t ld, int j) {
  __shared__ double Li[CB][CB + 1];
  __shared__ double Lk[CB][CB + 1];
  int ii = 0, rem = blockIdx.x;
  while (rem > ii) {  // row ii holds ii + 1 blocks
    rem -= ii + 1;
    ++ii;
  }
  const int kk = rem;
  const int64_t j0 = (int64_t)j * CB, i0 = j0 + (int64_t)(ii + 1) * CB, k0 = j0 + (int64_t)(kk + 1) * CB;
  const int t = threadIdx.x;
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    Li[r][c] = A[(i0 + r) * ld + j0 + c];
    Lk[r][c] = A[(k0 + r) * ld + j0 + c];
  }
  __syncthreads();
  const int tx = t & 15, ty = t >> 4;
  double acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int c = 0; c < CB; ++c) {
    double av[4], bv[4];
    for (int a = 0; a < 4; ++a) av[a] = Li[4 * ty + a][c];
    for (int b = 0; b < 4; ++b) bv[b] = Lk[4 * tx + b][c];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) A[(i0 + 4 * ty + a) * ld + k0 + 4 * tx + b] -= acc[a][b];
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
  for (int j = 0; j < nb; ++j) {
    chol_panel_kernel<<<(unsigned)(nb - j), 256, 0, st>>>(A, ld, j, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int m = nb - j - 1;
    if (m > 0) {
      chol_update_kernel<<<(unsigned)(m * (m + 1) / 2), 256, 0, st>>>(A, ld, j);
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
