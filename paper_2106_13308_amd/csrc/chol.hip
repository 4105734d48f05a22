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
//   chol_panel_kernel   nb - j workgroups: each factors the diagonal block A_jj in LDS (the
//                       same arithmetic in every workgroup, so the copies agree bit for bit);
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

// Unblocked right-looking Cholesky of the 64 x 64 block L (lower triangle; LDS, 256 threads)
// together with the forward substitution of w: after step c, column c of L and w[c] are final.
__device__ inline void factor_block(double (*L)[CB + 1], double* w) {
  const int t = threadIdx.x;
  for (int c = 0; c < CB; ++c) {
    const double piv = sqrt(L[c][c]);  // NaN if the block is not positive definite
    const double inv = 1.0 / piv;
    __syncthreads();
    if (t < CB) {
      if (t > c) L[t][c] *= inv;
      else if (t == c) {
        L[c][c] = piv;
        w[c] *= inv;
      }
    }
    __syncthreads();
    for (int e = t; e < CB * CB; e += 256) {
      const int r = e >> 6, q = e & (CB - 1);
      if (q > c && q <= r) L[r][q] -= L[r][c] * L[q][c];
    }
    if (t > c && t < CB) w[t] -= L[t][c] * w[c];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ A, int64_t ld, int j,
                                                         double* __restrict__ w) {
  __shared__ double L[CB][CB + 1];
  __shared__ double X[CB][CB + 1];
  __shared__ double wj[CB];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)j * CB;
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    L[r][c] = (c <= r) ? A[(j0 + r) * ld + j0 + c] : 0.0;
  }
  if (t < CB) wj[t] = w[j0 + t];
  __syncthreads();
  factor_block(L, wj);
  if (blockIdx.x == 0) {
    for (int e = t; e < CB * CB; e += 256) {
      const int r = e >> 6, c = e & (CB - 1);
      if (c <= r) A[(j0 + r) * ld + j0 + c] = L[r][c];
    }
    if (t < CB) w[j0 + t] = wj[t];
    return;
  }
  // block row i0 = j0 + 64 blockIdx.x: X L^T = A_ij, column by column
  const int64_t i0 = j0 + (int64_t)blockIdx.x * CB;
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    X[r][c] = A[(i0 + r) * ld + j0 + c];
  }
  __syncthreads();
  for (int c = 0; c < CB; ++c) {
    if (t < CB) X[t][c] /= L[c][c];
    __syncthreads();
    for (int e = t; e < CB * CB; e += 256) {
      const int r = e >> 6, q = e & (CB - 1);
      if (q > c) X[r][q] -= X[r][c] * L[q][c];
    }
    __syncthreads();
  }
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    A[(i0 + r) * ld + j0 + c] = X[r][c];
  }
  if (t < CB) {
    double s = 0.0;
    for (int c = 0; c < CB; ++c) s += X[t][c] * wj[c];
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

// Back substitution of block j: L_jj^T y_j = w_j (every workgroup solves it in LDS, the same
// arithmetic), then workgroup i < j applies w_i -= L_ji^T y_j.
__global__ __launch_bounds__(256) void chol_back_kernel(const double* __restrict__ A, int64_t ld, int j,
                                                        double* __restrict__ w, double* __restrict__ y) {
  __shared__ double L[CB][CB + 1];
  __shared__ double wj[CB];
  __shared__ double part[4][CB];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)j * CB;
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, c = e & (CB - 1);
    L[r][c] = (c <= r) ? A[(j0 + r) * ld + j0 + c] : 0.0;
  }
  if (t < CB) wj[t] = w[j0 + t];
  __syncthreads();
  for (int c = CB - 1; c >= 0; --c) {
    if (t == 0) wj[c] /= L[c][c];
    __syncthreads();
    if (t < c) wj[t] -= L[c][t] * wj[c];
    __syncthreads();
  }
  if (blockIdx.x == 0 && t < CB) y[j0 + t] = wj[t];
  if (blockIdx.x >= j) return;
  const int64_t i0 = (int64_t)blockIdx.x * CB;
  const int q = t & (CB - 1), g = t >> 6;  // column q of L_ji, rows 16 g .. 16 g + 15
  double s = 0.0;
  for (int r = 16 * g; r < 16 * g + 16; ++r) s += A[(j0 + r) * ld + i0 + q] * wj[r];
  part[g][q] = s;
  __syncthreads();
  if (t < CB) w[i0 + t] -= ((part[0][t] + part[1][t]) + (part[2][t] + part[3][t]));
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
    chol_back_kernel<<<(unsigned)(j > 0 ? j : 1), 256, 0, st>>>(A, ld, j, w, yd);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  chol_out_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(yd, B, y);
  return hipGetLastError();
}

}  // namespace vqmc
