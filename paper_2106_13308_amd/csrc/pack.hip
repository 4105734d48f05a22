// Packing of the MADE weights (Sec. 2.3, MADE layer with binary masks M1, M2).
//
// With sorted degrees the masks are complementary: for 0-based output/input site d,
// unit k feeds output d iff k < c[d] and receives input d iff k >= c[d].  All unmasked
// weights therefore fit one dense n x h matrix P[d][k] = (k < c[d]) ? W2[d][k] : W1[k][d].
#include "common.hpp"
#include "kernels.hpp"

namespace vqmc {

// P32[d][k] from W1 (h x n) and W2 (n x h).  The W1 column read is staged through a
// 32x32 LDS tile so both global reads are coalesced.
__global__ __launch_bounds__(256) void pack_kernel(int n, int h, const float* __restrict__ W1,
                                                    const float* __restrict__ W2,
                                                    const int32_t* __restrict__ c,
                                                    float* __restrict__ P32) {
  __shared__ float tile[32][33];
  const int d0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  // load W1[k0 + r][d0 + tx] into tile[r][tx]
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, d = d0 + tx;
    tile[r][tx] = (k < h && d < n) ? W1[(int64_t)k * n + d] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int d = d0 + r, k = k0 + tx;
    if (d < n && k < h) {
      const float v = (k < c[d]) ? W2[(int64_t)d * h + k] : tile[tx][r];
      P32[(int64_t)d * h + k] = v;
    }
  }
}

__global__ __launch_bounds__(256) void unpack_kernel(int n, int h, const float* __restrict__ P32,
                                                      const int32_t* __restrict__ c,
                                                      float* __restrict__ W1,
                                                      float* __restrict__ W2) {
  __shared__ float tile[32][33];
  const int d0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int d = d0 + r, k = k0 + tx;
    float v = 0.f;
    if (d < n && k < h) {
      v = P32[(int64_t)d * h + k];
      const bool lower = k < c[d];
      W2[(int64_t)d * h + k] = lower ? v : 0.f;
      if (lower) v = 0.f;
    }
    tile[r][tx] = v;  // W1 part (k >= c[d]) in (d, k) order
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, d = d0 + tx;
    if (k < h && d < n) W1[(int64_t)k * n + d] = tile[tx][r];
  }
}

// Working copies: P (n x ldh) and Pt (h x ldn) in float or bf16, zero padded.
template <typename T>
__device__ inline T convert(float x);
template <>
__device__ inline float convert<float>(float x) { return x; }
template <>
__device__ inline bf16_t convert<bf16_t>(float x) { return f32_to_bf16(x); }

template <typename T>
__global__ __launch_bounds__(256) void cast_kernel(int n, int h, int64_t ldh, int64_t ldn,
                                                    const float* __restrict__ P32,
                                                    T* __restrict__ P, T* __restrict__ Pt) {
  __shared__ T tile[32][33];
  const int d0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int d = d0 + r, k = k0 + tx;
    const T v = convert<T>((d < n && k < h) ? P32[(int64_t)d * h + k] : 0.f);
    tile[r][tx] = v;
    if (d < n && k < ldh) P[(int64_t)d * ldh + k] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, d = d0 + tx;
    if (k < h && d < ldn) Pt[(int64_t)k * ldn + d] = tile[tx][r];
  }
}

hipError_t launch_pack(int n, int h, const float* W1, const float* W2, const int32_t* c, float* P32,
                       hipStream_t st) {
  dim3 grid((h + 31) / 32, (n + 31) / 32);
  pack_kernel<<<grid, 256, 0, st>>>(n, h, W1, W2, c, P32);
  return hipGetLastError();
}

hipError_t launch_unpack(int n, int h, const float* P32, const int32_t* c, float* W1, float* W2,
                         hipStream_t st) {
  dim3 grid((h + 31) / 32, (n + 31) / 32);
  unpack_kernel<<<grid, 256, 0, st>>>(n, h, P32, c, W1, W2);
  return hipGetLastError();
}

hipError_t launch_cast(int n, int h, const float* P32, int dtype, void* P, void* Pt, hipStream_t st) {
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad);
  // grid covers the padded extents so that padding is written as zero
  dim3 grid((unsigned)(ldh / 32), (unsigned)(ldn / 32));
  if (dtype == VQMC_BF16)
    cast_kernel<bf16_t><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (bf16_t*)P, (bf16_t*)Pt);
  else
    cast_kernel<float><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (float*)P, (float*)Pt);
  return hipGetLastError();
}

}  // namespace vqmc
