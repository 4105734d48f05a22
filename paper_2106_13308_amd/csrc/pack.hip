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
// With TABLES the same workgroup also writes the pipelined sampler's weight tiles of its
// 64 sites x 64 units (layout: the sampler tables after the band records, see vqmc_band):
// logit tiles of the block's units (and, in the first column of workgroups, the block's b2
// tile) and push tiles, straight from the LDS tile, so the weights are read once.
template <typename T, bool TABLES>
__global__ __launch_bounds__(256) void cast_kernel(int n, int h, int64_t ldh, int64_t ldn,
                                                    const float* __restrict__ P32,
                                                    T* __restrict__ P, T* __restrict__ Pt,
                                                    const float* __restrict__ b2, const int32_t* __restrict__ c,
                                                    uint8_t* __restrict__ ztab, uint8_t* __restrict__ utab,
                                                    bf16_t* __restrict__ Pm, int nzt, int nut,
                                                    const float* __restrict__ b1, int32_t* __restrict__ nonfinite) {
  __shared__ T tile[CT][CT + 2];  // odd row stride in dwords for either T: column reads spread
  const int d0 = blockIdx.y * CT, k0 = blockIdx.x * CT;
  const int t = threadIdx.x;
  bool bad = false;  // a NaN or infinity among the parameters this workgroup reads
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
        bad |= !__builtin_isfinite(v[e]);
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
  if (nonfinite) {  // biases: b2 of the block's sites (first column of workgroups), b1 of its units (first row)
    if (t < CT && k0 == 0 && d0 + t < n) bad |= !__builtin_isfinite(b2[d0 + t]);
    if (t < CT && d0 == 0 && k0 + t < h) bad |= !__builtin_isfinite(b1[k0 + t]);
    if (__ballot(bad) && (t & 63) == 0) atomicOr(nonfinite, 1);
  }
  __syncthreads();
  {
    const int dx = t & 7, kr = t >> 3;  // sites 8 dx .. +7, units kr + 32 s
    int cd[8];  // TABLES, BF16: c of the eight sites, for the masked copy of P^T (0 past n)
    if constexpr (TABLES && sizeof(T) == 2) {
#pragma unroll
      for (int e = 0; e < 8; ++e) cd[e] = (d0 + 8 * dx + e < n) ? c[d0 + 8 * dx + e] : 0;
    }
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
          if constexpr (TABLES) {  // unit k feeds site d iff k < c[d]
            T pm[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) pm[e] = (k < cd[e]) ? o[e] : (T)0;
            *(uint4*)(Pm + (int64_t)k * ldn + d0 + 8 * dx) = *(const uint4*)pm;
          }
        } else {
          *(float4*)dst = *(const float4*)o;
          *(float4*)(dst + 4) = *(const float4*)(o + 4);
        }
      }
    }
  }
  if constexpr (TABLES) {
    const int q = d0 / CT;  // site block
    if constexpr (sizeof(T) == 2) {
      // logit tiles t = 1 + k0/32 + cc: [4 site tiles][64 lanes][8 units], lane = 16 g + i
      uint8_t* zq = ztab + (int64_t)q * nzt * 4096;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int u = t + 256 * r, cc = u >> 8, tt = (u >> 6) & 3, lane = u & 63;
        const int zt = 1 + k0 / 32 + cc;
        if (zt < nzt) {
          const int dl = 16 * tt + (lane & 15), kl = 32 * cc + 8 * (lane >> 4);
          const uint32_t* src = (const uint32_t*)&tile[dl][kl];  // 4-byte aligned: even column
          *(uint4*)(zq + (int64_t)zt * 4096 + tt * 1024 + lane * 16) = make_uint4(src[0], src[1], src[2], src[3]);
        }
      }
      // push tiles i = k0/16 + ii: [2 halves][64 lanes][8 sites], lane = 16 g + unit
      uint8_t* uq = utab + (int64_t)q * nut * 2048;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int u = t + 256 * r, ii = u >> 7, ks = (u >> 6) & 1, lane = u & 63;
        const int ut = k0 / 16 + ii;
        if (ut < nut) {
          const int kl = 16 * ii + (lane & 15), dl = 32 * ks + 8 * (lane >> 4);
          T o[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) o[e] = tile[dl + e][kl];
          *(uint4*)(uq + (int64_t)ut * 2048 + ks * 1024 + lane * 16) = *(const uint4*)o;
        }
      }
      if (k0 == 0) {  // b2 tile: units 0-2 of lane group 0 hold hi, mid, lo of b2
        const int tt = t >> 6, lane = t & 63, i = lane & 15, g = lane >> 4;
        const int d = d0 + 16 * tt + i;
        uint32_t v[3] = {0u, 0u, 0u};
        if (g == 0 && d < n) {
          const float x = b2[d];
          const float hi = __uint_as_float(__float_as_uint(x) & 0xFFFF0000u);
          const float rr = x - hi;
          const float mid = __uint_as_float(__float_as_uint(rr) & 0xFFFF0000u);
          const float lo = rr - mid;
          v[0] = __float_as_uint(hi) >> 16;
          v[1] = __float_as_uint(mid) >> 16;
          v[2] = __float_as_uint(lo) >> 16;
        }
        *(uint4*)(zq + tt * 1024 + lane * 16) = make_uint4(v[0] | (v[1] << 16), v[2], 0u, 0u);
      }
    } else {
      // logit tiles t = 1 + k0/4 + cc: [4 site tiles][64 lanes] floats, unit = lane / 16
      uint8_t* zq = ztab + (int64_t)q * nzt * 1024;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int u = t + 256 * r, cc = u >> 8, tt = (u >> 6) & 3, lane = u & 63;
        const int zt = 1 + k0 / 4 + cc;
        if (zt < nzt) *(float*)(zq + (int64_t)zt * 1024 + tt * 256 + lane * 4) = (float)tile[16 * tt + (lane & 15)][4 * cc + (lane >> 4)];
      }
      // push tiles: [2 halves][64 lanes][8 sites] floats
      uint8_t* uq = utab + (int64_t)q * nut * 4096;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int u = t + 256 * r, ii = u >> 7, ks = (u >> 6) & 1, lane = u & 63;
        const int ut = k0 / 16 + ii;
        if (ut < nut) {
          const int kl = 16 * ii + (lane & 15), dl = 32 * ks + 8 * (lane >> 4);
          float o[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) o[e] = (float)tile[dl + e][kl];
          uint8_t* dst = uq + (int64_t)ut * 4096 + ks * 2048 + lane * 32;
          *(float4*)dst = *(const float4*)o;
          *(float4*)(dst + 16) = *(const float4*)(o + 4);
        }
      }
      if (k0 == 0) {
        const int tt = t >> 6, lane = t & 63, d = d0 + 16 * tt + (lane & 15);
        *(float*)(zq + tt * 256 + lane * 4) = ((lane >> 4) == 0 && d < n) ? b2[d] : 0.f;
      }
    }
  }
}

// c[d] = #{k : m(k) <= d} (0-based site d, 1-based sorted degrees m), from the degrees passed
// by value in chunks: each launch adds its chunk's count (a bisection of the sorted chunk), so
// no host buffer has to outlive an asynchronous copy.
__global__ void degree_count_kernel(int n, DegreeChunk ch, int first, int32_t* __restrict__ c) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  int lo = 0, hi = ch.count;  // first index whose degree exceeds d
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ch.deg[mid] <= d)
      lo = mid + 1;
    else
      hi = mid;
  }
  c[d] = first ? lo : c[d] + lo;
}

hipError_t launch_degree_counts(int n, int h, const int32_t* degrees, int32_t* c, hipStream_t st) {
  for (int k0 = 0; k0 < h; k0 += kDegreeChunk) {
    DegreeChunk ch;
    ch.count = h - k0 < kDegreeChunk ? h - k0 : kDegreeChunk;
    for (int i = 0; i < ch.count; ++i) ch.deg[i] = degrees[k0 + i];
    degree_count_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, ch, k0 == 0, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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

hipError_t launch_cast(int n, int h, const float* P32, int dtype, void* P, void* Pt, hipStream_t st,
                       const float* b2, const int32_t* c, void* tables, const float* b1, int32_t* nonfinite) {
  const int64_t ldh = round_up(h, kPad), ldn = round_up(n, kPad);
  // grid covers the padded extents so that padding is written as zero
  dim3 grid((unsigned)(ldh / CT), (unsigned)(ldn / CT));
  uint8_t *zt = nullptr, *ut = nullptr;
  bf16_t* pm = nullptr;
  int nzt = 0, nut = 0;
  if (tables) {
    int64_t zo, uo, po;
    sample_tables_layout(n, h, dtype, &zo, &uo, &po, &nzt, &nut);
    zt = (uint8_t*)tables + zo;
    ut = (uint8_t*)tables + uo;
    pm = (bf16_t*)((uint8_t*)tables + po);
  }
  if (dtype == VQMC_BF16) {
    if (tables)
      cast_kernel<bf16_t, true><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (bf16_t*)P, (bf16_t*)Pt, b2, c, zt, ut, pm,
                                                       nzt, nut, b1, nonfinite);
    else
      cast_kernel<bf16_t, false><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (bf16_t*)P, (bf16_t*)Pt, b2, c, zt, ut, pm,
                                                        0, 0, b1, nonfinite);
  } else {
    if (tables)
      cast_kernel<float, true><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (float*)P, (float*)Pt, b2, c, zt, ut, pm,
                                                      nzt, nut, b1, nonfinite);
    else
      cast_kernel<float, false><<<grid, 256, 0, st>>>(n, h, ldh, ldn, P32, (float*)P, (float*)Pt, b2, c, zt, ut, pm,
                                                       0, 0, b1, nonfinite);
  }
  return hipGetLastError();
}

}  // namespace vqmc
