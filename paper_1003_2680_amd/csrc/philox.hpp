// Device-side counter-based Gaussian noise.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): ten rounds, each multiplying words 0 and 2 by the two Philox constants, splitting
// the 64-bit products into halves and forming (hi1^w1^k0, lo1, hi0^w3^k1, lo0); the key
// advances by the two Weyl constants between rounds.  One 32x32->64 multiply per product
// maps to a single v_mad_u64_u32 on CDNA.
//
// Box-Muller turns words (w0,w1) and (w2,w3) into two 53-bit uniforms in (0,1] and then
// into two standard normals: sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).
// The angle uses sincospi(2 u2), which needs no reduction by pi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smg {

// Batched chains: component c belongs to chain c / comps_per_chain, which has its own seed and
// first cycle; its noise is that of component c % comps_per_chain of a one-chain run.
struct ChainKey {
  uint32_t k0, k1;   // seed low / high
  uint32_t c0, c1;   // first cycle low / high
};

struct NoiseArgs {
  uint32_t k0, k1;   // seed low / high (one chain)
  uint32_t sid;      // level | slot<<4 | colour<<12 | kind<<24 (component added per thread)
  uint32_t c2, c3;   // cycle low / high; with `chains`: cycles since each chain's first cycle
  double sqkT;       // sqrt(kT)
  const ChainKey* chains;    // null: one chain keyed by (k0, k1)
  uint32_t comps_per_chain;
};

// Philox key, counter words 1..3 for component `comp`.
__device__ __forceinline__ void noise_key(const NoiseArgs& na, uint32_t comp, uint32_t& k0,
                                          uint32_t& k1, uint32_t& w1, uint32_t& w2,
                                          uint32_t& w3) {
  if (na.chains) {
    const uint32_t ch = comp / na.comps_per_chain;
    const ChainKey key = na.chains[ch];
    const uint64_t cyc = (((uint64_t)key.c1 << 32) | key.c0) + (((uint64_t)na.c3 << 32) | na.c2);
    k0 = key.k0;
    k1 = key.k1;
    w1 = na.sid | ((comp - ch * na.comps_per_chain) << 16);
    w2 = (uint32_t)cyc;
    w3 = (uint32_t)(cyc >> 32);
  } else {
    k0 = na.k0;
    k1 = na.k1;
    w1 = na.sid | (comp << 16);
    w2 = na.c2;
    w3 = na.c3;
  }
}

__device__ __forceinline__ void philox4x32_10(uint32_t& w0, uint32_t& w1, uint32_t& w2,
                                              uint32_t& w3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * w0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * w2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ w1 ^ k0;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ w3 ^ k1;
    w1 = (uint32_t)p1;
    w3 = (uint32_t)p0;
    w0 = n0;
    w2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
  uint64_t v = (((uint64_t)a << 32) | b) >> 11;
  return ((double)v + 0.5) * 0x1p-53;
}

// Two normals of call `call` in stream (sid | comp<<16) at the given cycle.
__device__ __forceinline__ void normal_pair(const NoiseArgs& na, uint32_t comp, uint32_t call,
                                            double& z0, double& z1) {
  uint32_t w0 = call, w1, w2, w3, k0, k1;
  noise_key(na, comp, k0, k1, w1, w2, w3);
  philox4x32_10(w0, w1, w2, w3, k0, k1);
  double u1 = uniform53(w0, w1);
  double u2 = uniform53(w2, w3);
  double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// FP32 variant for the FP32 sweeps of the refined mode: the same Philox words and the same
// 53-bit uniforms, rounded to FP32 (full relative precision down to the smallest uniform, so
// the tail is not clipped), then the hardware log2 / sin / cos (v_sin_f32 and v_cos_f32 take
// revolutions, so the angle 2 pi u2 needs no multiplication by pi).  The normals differ from
// the FP64 ones only by FP32 rounding.
__device__ __forceinline__ void normal_pair_f32(const NoiseArgs& na, uint32_t comp, uint32_t call,
                                                float& z0, float& z1) {
  uint32_t w0 = call, w1, w2, w3, k0, k1;
  noise_key(na, comp, k0, k1, w1, w2, w3);
  philox4x32_10(w0, w1, w2, w3, k0, k1);
  const float u1 = (float)uniform53(w0, w1);
  const float u2 = (float)uniform53(w2, w3);
  const float r = __builtin_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u1));
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

// normals in the storage precision T of the sweep
template <typename T>
__device__ __forceinline__ void normal_pair_t(const NoiseArgs& na, uint32_t comp, uint32_t call,
                                              T& z0, T& z1);
template <>
__device__ __forceinline__ void normal_pair_t<double>(const NoiseArgs& na, uint32_t comp,
                                                      uint32_t call, double& z0, double& z1) {
  normal_pair(na, comp, call, z0, z1);
}
template <>
__device__ __forceinline__ void normal_pair_t<float>(const NoiseArgs& na, uint32_t comp,
                                                     uint32_t call, float& z0, float& z1) {
  normal_pair_f32(na, comp, call, z0, z1);
}

}  // namespace smg
