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

// 64 x 64 tile per workgroup: 16-byte reads of P32, 4-element row writes of P, and the
// transpose through LDS written as 8-element rows of Pt.  The grid covers the padded
// extents, so padding is written as zero.
constexpr int CT = 64;
template <typename T>
__global__ __launch_bounds__(256) void cast_kernel(int n, int h, int64_t ldh, int64_t ldn,
                                                    const float* __restrict__ P32,
                                                    T* __restrict__ P, T* __restrict__ Pt) {
  __shared__ T tile[CT][CT + 2];  // odd row stride in dwords for either T: column reads spread
  const int d0 = blockIdx.y * CT, k0 = blockIdx.x * CT;
  const int t = threadIdx.x;
  {
    const int tx = t & 15, ty = t >> 4;  // columns 4 tx .. +3, rows ty + 16 r
    const int k = k0 + 4 * tx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = d0 + ty + 16 * r;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (d < n) {
        if (k + 4 <= h && (h & 3) == 0) {
          const float4 q = *(const float4*)(P32 + (int64_t)d * h + k);
          v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (k + e < h) ? P32[(int64_t)d * h + k + e] : 0.f;
        }
      }
      T o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[e] = convert<T>(v[e]);
        tile[ty + 16 * r][4 * tx + e] = o[e];
      }
      if (d < n) {
        T* dst = P + (int64_t)d * ldh + k;  // k + 4 <= ldh: ldh is a multiple of 64
        if constexpr (sizeof(T) == 2) *(uint2*)dst = *(const uint2*)o;
        else *(float4*)dst = *(const float4*)o;
      }
    }
  }
  __syncthreads();
  {
    const int dx = t & 7, kr = t >> 3;  // sites 8 dx .. +7, units kr + 32 s
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int kk = kr + 32 * s2, k = k0 + kk;
      if (k < h) {
        T o[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = tile[8 * dx + e][kk];
        T* dst = Pt + (int64_t)k * ldn + d0 + 8 * dx;  // inside the padded row
        if constexpr (sizeof(T) == 2) {
          *(uint4*)dst = *(const uint4*)o;
        } else {
          *(float4*)dst = *(const float4*)o;
          *(float4*)(dst + 4) = *(const float4*)(o + 4);
        }
      }
    }
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
  dim3 grid((unsigned)(ldh / CT), (unsigned)(ldn / CT));
  if (dtype == VQMC_BF16)
    cast_kernel<bf16_t><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (bf16_t*)P, (bf16_t*)Pt);
  else
    cast_kernel<float><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (float*)P, (float*)Pt);
  return hipGetLastError();
}

}  // namespace vqmc
