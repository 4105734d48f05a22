// Shared device helpers for the VQMC library (gfx950 / CDNA4 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vqmc.h"

namespace vqmc {

typedef uint16_t bf16_t;  // raw bfloat16 bits
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float floatx4_t;
typedef __attribute__((ext_vector_type(4))) double doublex4_t;

constexpr int kPad = VQMC_PAD;  // leading-dimension padding (elements)

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- bfloat16
// float32 -> bfloat16, round to nearest even (NaN stays a quiet NaN).
__device__ inline bf16_t f32_to_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (bf16_t)((b >> 16) | 0x0040u);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (bf16_t)(b >> 16);
}
__device__ inline float bf16_to_f32(bf16_t x) { return __uint_as_float(((uint32_t)x) << 16); }

template <typename T> __device__ inline float to_f32(T x);
template <> __device__ inline float to_f32<float>(float x) { return x; }
template <> __device__ inline float to_f32<bf16_t>(bf16_t x) { return bf16_to_f32(x); }
template <typename T> __device__ inline T from_f32(float x);
template <> __device__ inline float from_f32<float>(float x) { return x; }
template <> __device__ inline bf16_t from_f32<bf16_t>(float x) { return f32_to_bf16(x); }

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al., SC'11: 10 rounds of the 4x32 Philox bijection with Weyl key schedule.
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32 each)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Four consecutive site uniforms u[b, 4*blk .. 4*blk+3] (24-bit dyadic in [0,1)).
// Counter = (site block, global sample index, step, tag), key = seed.
__device__ inline float4 site_uniforms(uint64_t seed, uint64_t step, uint32_t tag, uint64_t sample,
                                       uint32_t blk) {
  const uint4 r = philox4x32_10(make_uint4(blk, (uint32_t)sample, (uint32_t)step, tag),
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const float s = 5.9604644775390625e-8f;  // 2^-24
  return make_float4((float)(r.x >> 8) * s, (float)(r.y >> 8) * s, (float)(r.z >> 8) * s,
                     (float)(r.w >> 8) * s);
}

// ---------------------------------------------------------------- streaming stores
// A non-temporal 16-byte store (global_store_dwordx4 ... nt), for a large output that no later
// kernel of the same call reads while it could still be cached: it does not displace the lines
// the following kernels reuse.
__device__ inline void store_nt(void* p, uint4 v) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, (u32x4*)p);
}

// ---------------------------------------------------------------- numerics
// log(1 + x) for x >= 0 without the cancellation of log(1 + x) near 0: with u = 1 + x
// rounded, log(u) - ((u - 1) - x) / u corrects for the rounding of u (Goldberg, "What
// every computer scientist should know about floating-point arithmetic", Thm. 4); the
// correction is below one ulp of u, so a hardware reciprocal is accurate enough.
__device__ inline float log1p_pos(float x) {
  const float u = 1.f + x;
  return __logf(u) - ((u - 1.f) - x) * __builtin_amdgcn_rcpf(u);
}
// log sigma(t) = min(t, 0) - log1p(exp(-|t|)), stable for large |t|.
__device__ inline float log_sigmoid(float t) { return fminf(t, 0.f) - log1p_pos(__expf(-fabsf(t))); }
// sigma(t) for any t without overflow.
__device__ inline float sigmoid(float t) {
  const float e = __expf(-fabsf(t));
  const float r = 1.f / (1.f + e);
  return t >= 0.f ? r : e * r;
}

// ---------------------------------------------------------------- workgroup barrier
// Barrier whose fences order LDS only: global loads a wave has in flight stay in flight
// across it.  For kernels whose waves exchange data through LDS alone.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// sum_p part[p][i] over nparts rows of stride floats: the loads of eight parts are issued
// together and summed in a fixed order (four running sums, then ((s0 + s1) + (s2 + s3))).
__device__ inline float sum_parts(const float* __restrict__ part, int nparts, int64_t stride, int64_t i) {
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  int p = 0;
  for (; p + 8 <= nparts; p += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(p + u) * stride + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u & 3] += v[u];
  }
  for (; p < nparts; ++p) s[p & 3] += part[(int64_t)p * stride + i];
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// ---------------------------------------------------------------- wave reductions (wave64)
#define VQMC_DPP(v, ctrl) \
  __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false))

// Sum over all 64 lanes; result is wave-uniform.
__device__ inline float wave_sum(float v) {
  v += VQMC_DPP(v, 0xB1);   // quad_perm [1,0,3,2]
  v += VQMC_DPP(v, 0x4E);   // quad_perm [2,3,0,1]
  v += VQMC_DPP(v, 0x141);  // row_half_mirror
  v += VQMC_DPP(v, 0x140);  // row_mirror  -> every lane holds its 16-lane row sum
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

__device__ inline float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

}  // namespace vqmc
