// Device helpers shared by the iteration kernels (kp_kernels.hip) and the
// learned-proposal kernels (kp_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t w[4];
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
  // each round's two 32 x 32 -> 64-bit products as 64-bit multiplies: one
  // v_mad_u64_u32 each instead of a multiply-high and a multiply-low
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  U4 o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

// e-th frontier node: explicit list first, then the implicit tail of ids
__device__ __forceinline__ int32_t frontier_node(const int32_t* F, int32_t e, int32_t f_expl,
                                                 int32_t f_base) {
  return (e < f_expl) ? F[e] : f_base + (e - f_expl);
}

// Box-Muller transform (Box & Muller, 1958) of two Philox words: u1 in
// (0, 1] from the top 24 bits of a plus one ulp, u2 in [0, 1) from b; the
// pair (r cos 2 pi u2, r sin 2 pi u2) with r = sqrt(-2 ln u1) is standard normal.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float* z0, float* z1) {
  const float u1 = (float)((a >> 8) + 1u) * 0x1p-24f;
  const float u2 = (float)(b >> 8) * 0x1p-24f;
  const float r = sqrtf(-2.0f * logf(u1));
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  *z0 = r * cs;
  *z1 = r * sn;
}

}  // namespace kp
