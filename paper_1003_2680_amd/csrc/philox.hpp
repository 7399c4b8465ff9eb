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
// The FP64 logarithm, square root and sine/cosine of pi t are evaluated here (below) for the
// bounded arguments Box-Muller produces: the general-purpose library routines spend about
// twice the instructions on full-range reduction, scaling and extra-precise arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sincos_table.hpp"

namespace smg {

// Batched chains: component c belongs to chain c / comps_per_chain, which has its own seed and
// first cycle; its noise is that of component c % comps_per_chain of a one-chain run.
struct ChainKey {
  uint32_t k0, k1;   // seed low / high
  uint32_t c0, c1;   // first cycle low / high
};

// Polynomial coefficients of the FP64 Box-Muller (see neg2_log_unit and sincospi_turns).  They
// travel in the kernel arguments so that a wave reads them with scalar loads and the FMAs take
// them as scalar operands, instead of materialising every 64-bit literal in vector registers.
struct BoxMullerCoef {
  double lg[9];   // 1/19, 1/17, ..., 1/3
  double sn[4];   // pi, -pi^3/3!, pi^5/5!, -pi^7/7!   (sin(pi r) = r (sn0 + z (sn1 + ...)), z = r^2)
  double cs[3];   // -pi^2/2!, pi^4/4!, -pi^6/6!        (cos(pi r) = 1 + z (cs0 + z (cs1 + ...)))
  double snq[9];  // (-1)^k pi^(2k+1)/(2k+1)!, k = 8 .. 0   (quarter-turn form, no table)
  double csq[8];  // (-1)^k pi^(2k)/(2k)!, k = 8 .. 1
};

// a z + c and a + c with c wave-uniform (a kernel argument held in scalar registers), written
// in the three-operand encodings, which read the scalar pair directly.  Left to itself the
// compiler picks the two-operand accumulate form, whose addend must sit in vector registers,
// and copies every coefficient there first (two moves per coefficient and lane).
__device__ __forceinline__ double fma_uniform_addend(double a, double z, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(z), "s"(c));
  return r;
}
__device__ __forceinline__ double add_uniform(double a, double c) {
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(c));
  return r;
}

// sum_{i < n} c[n-1-i] z^i by Horner's rule, the coefficients entering as scalar addends:
// n vector instructions for n coefficients.  The series here converge fast (z <= 1/16), so the
// nested order is as accurate as any.
template <int n>
__device__ __forceinline__ double poly_horner(const double (&c)[n], double z) {
  double acc = add_uniform(c[0] * z, c[1]);
#pragma unroll
  for (int i = 2; i < n; ++i) acc = fma_uniform_addend(acc, z, c[i]);
  return acc;
}

struct NoiseArgs {
  uint32_t k0, k1;   // seed low / high (one chain)
  uint32_t sid;      // level | slot<<4 | colour<<12 | kind<<24 (component added per thread)
  uint32_t c2, c3;   // cycle low / high; with `chains`: cycles since each chain's first cycle
  double sqkT;       // sqrt(kT)
  const ChainKey* chains;    // null: one chain keyed by (k0, k1)
  uint32_t comps_per_chain;
  // added to the component index of every draw: a launch over components c0 .. c0+n-1 of a
  // hierarchy numbers them from 0 on shifted pointers and passes c0 here
  uint32_t comp0 = 0;
  // floor(2^32 / comps_per_chain) + 1 (0 when comps_per_chain is 1): comp / comps_per_chain is
  // the high word of comp * cpc_magic for comp and comps_per_chain below 2^16
  uint32_t cpc_magic;
  BoxMullerCoef bm;
};

// The multiplier that turns the division by comps_per_chain into a multiply-high (host).
inline uint32_t chain_divisor_magic(uint32_t comps_per_chain) {
  return comps_per_chain <= 1 ? 0u : (uint32_t)((1ull << 32) / comps_per_chain) + 1u;
}

// The coefficient values (host and device).
inline __host__ __device__ BoxMullerCoef box_muller_coef() {
  return BoxMullerCoef{
      {1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0,
       1.0 / 5.0, 1.0 / 3.0},
      {0x1.921fb54442d18p+1, -0x1.4abbce625be53p+2, 0x1.466bc6775aae2p+1, -0x1.32d2cce62bd86p-1},
      {-0x1.3bd3cc9be45dep+2, 0x1.03c1f081b5ac4p+2, -0x1.55d3c7e3cbffap+0},
      {0x1.aaec32af93359p-21, -0x1.6fadb9f155744p-16, 0x1.e8f434d018d63p-12,
       -0x1.e3074fde8871fp-8, 0x1.50783487ee782p-4, -0x1.32d2cce62bd86p-1, 0x1.466bc6775aae2p+1,
       -0x1.4abbce625be53p+2, 0x1.921fb54442d18p+1},
      {0x1.20c62c2f2d7f5p-18, -0x1.b6e24f44b128fp-14, 0x1.f9d38a3763cc3p-10,
       -0x1.a6d1f2a204a8cp-6, 0x1.e1f506891babbp-3, -0x1.55d3c7e3cbffap+0, 0x1.03c1f081b5ac4p+2,
       -0x1.3bd3cc9be45dep+2}};
}

// Philox key, counter words 1..3 for component `comp` of stream `sid`.  Every caller draws
// for one component per work-group, so `comp` is wave-uniform: taking it from the first lane
// lets the chain lookup, the key and the key schedule of the rounds run on the scalar unit.
__device__ __forceinline__ void noise_key(const NoiseArgs& na, uint32_t sid, uint32_t comp,
                                          uint32_t& k0, uint32_t& k1, uint32_t& w1, uint32_t& w2,
                                          uint32_t& w3) {
  comp = __builtin_amdgcn_readfirstlane(comp) + na.comp0;
  if (na.chains) {
    const uint32_t ch = na.cpc_magic ? __umulhi(comp, na.cpc_magic) : comp;
    // the chain table is read-only while kernels run: scalar loads through the constant space
    typedef const __attribute__((address_space(4))) uint32_t* cword;
    const cword kw = (cword)(const void*)(na.chains + ch);
    ChainKey key;
    key.k0 = kw[0];
    key.k1 = kw[1];
    key.c0 = kw[2];
    key.c1 = kw[3];
    const uint64_t cyc = (((uint64_t)key.c1 << 32) | key.c0) + (((uint64_t)na.c3 << 32) | na.c2);
    k0 = key.k0;
    k1 = key.k1;
    w1 = sid | ((comp - ch * na.comps_per_chain) << 16);
    w2 = (uint32_t)cyc;
    w3 = (uint32_t)(cyc >> 32);
  } else {
    k0 = na.k0;
    k1 = na.k1;
    w1 = sid | (comp << 16);
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
    uint32_t n0, n2;
    if (r < 2) {
      // the counter words w1..w3 are usually uniform across a wave, so the first two rounds
      // keep plain exclusive ors, which the compiler moves to the scalar unit where it can
      n0 = (uint32_t)(p1 >> 32) ^ w1 ^ k0;
      n2 = (uint32_t)(p0 >> 32) ^ w3 ^ k1;
    } else {
      // three-input exclusive or in one instruction (truth table 0x96: odd parity)
      n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), w1, k0, 0x96);
      n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), w3, k1, 0x96);
    }
    w1 = (uint32_t)p1;
    w3 = (uint32_t)p0;
    w0 = n0;
    w2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// ((a 2^32 + b) >> 11) + 1/2, times 2^-53: the two parts a 2^-32 and ((b >> 11) + 1/2) 2^-53 are
// exact doubles, so one rounding of their sum gives the correctly rounded value
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
  const double lo = fma((double)(b >> 11), 0x1p-53, 0x1p-54);
  return fma((double)a, 0x1p-32, lo);
}

// 2 uniform53(a, b), formed with the doubled (exact) scalings: the same rounding, one operation
// fewer
__device__ __forceinline__ double uniform53_x2(uint32_t a, uint32_t b) {
  const double lo = fma((double)(b >> 11), 0x1p-52, 0x1p-53);
  return fma((double)a, 0x1p-31, lo);
}

// -2 ln(u) for u in (0, 1], FP64, within a few ulp (the radius of Box-Muller before its square
// root).  u = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m - 1)/(m + 1),
// |s| <= 0.1716, summed as the odd Taylor series 2 s (1 + s^2/3 + s^4/5 + ... + s^18/19) (the
// first omitted term is below 2^-55 of the sum); the quotient comes from the hardware
// reciprocal refined by one Newton step (relative error below 2^-44) and a residual correction
// of the quotient itself, which squares that error; e ln 2 is added with ln 2 split so that
// e * ln2_hi is exact.  The factor -2 is folded into 2 s and the two parts of
// ln 2 (exact scalings), so the result is -2 times the rounded logarithm, bit for bit.
__device__ __forceinline__ double neg2_log_unit(double u, const BoxMullerCoef& c) {
  int e;
  double m = frexp(u, &e);  // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;  // exact
  const double d = m + 1.0;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  double s = f * r;
  s = fma(fma(-d, s, f), r, s);
  const double z = s * s;
  const double p = poly_horner(c.lg, z);
  const double s2 = -4.0 * s;
  const double lm = fma(s2 * z, p, s2);
  constexpr double LN2_HI = -0x1.62e42fef00000p+0;  // -2 ln 2 with the low 20 bits cleared
  constexpr double LN2_LO = -0x1.473de6af278edp-33; // -2 ln 2 - LN2_HI
  return fma((double)e, LN2_HI, fma((double)e, LN2_LO, lm));
}

// sin(pi t) and cos(pi t) for t in [0, 2], FP64, within a few ulp: k = rint(128 t) and
// r = t - k/128 (exact, |r| <= 1/256); sin(pi r) and cos(pi r) from their Taylor series to
// degree 7 and 6 (|pi r| <= 0.0123: the first omitted terms are below 2^-70 relative); then the
// angle addition with the tabulated sin(pi k/128), cos(pi k/128) (correctly rounded doubles).
__device__ __forceinline__ void sincospi_turns(double t, const BoxMullerCoef& c, double& sn,
                                               double& cs) {
  const double kf = rint(128.0 * t);
  const double r = fma(-0.0078125, kf, t);
  const int k = (int)kf & 255;
  const double z = r * r;
  const double S = r * fma(z, fma(z, fma(z, c.sn[3], c.sn[2]), c.sn[1]), c.sn[0]);
  const double C = fma(z, fma(z, fma(z, c.cs[2], c.cs[1]), c.cs[0]), 1.0);
  const double sk = kSinCosPi128[k][0], ck = kSinCosPi128[k][1];
  sn = fma(sk, C, ck * S);
  cs = fma(ck, C, -(sk * S));
}

// sin(pi t) and cos(pi t) for t in [0, 2] without a table (for kernels whose own loads should
// stay in flight during the noise arithmetic): t = n/2 + r with n the nearest integer to 2t and
// |r| <= 1/4 (exact); sin(pi r) and cos(pi r) from their Taylor series to degree 17 and 16
// (|pi r| <= pi/4: the first omitted terms are below 2^-56); then the quarter-turn rotation by n.
__device__ __forceinline__ void sincospi_quarter(double t, const BoxMullerCoef& c, double& sn,
                                                 double& cs) {
  const double n = rint(2.0 * t);
  const double r = fma(-0.5, n, t);
  const double z = r * r;
  const double S = r * poly_horner(c.snq, z);
  const double C = fma(poly_horner(c.csq, z), z, 1.0);
  const int q = (int)n & 3;
  const double a = (q & 1) ? C : S;  // sin(pi (r + n/2))
  const double b = (q & 1) ? S : C;  // cos(pi (r + n/2))
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

// sqrt(a) for a in [0, 2^10] (Box-Muller's -2 ln u1 <= 75): the hardware reciprocal square
// root refined by a Goldschmidt step and two residual corrections; no scaling is needed in this
// range.  a = +-0 (u1 = 1): the reciprocal root of |a| is +inf, clamped to 2^500 so that every
// step stays finite and gives 0; a positive a is at least 2^-53, far from the clamp.
__device__ __forceinline__ double sqrt_bm(double a) {
  const double y = __builtin_fmin(__builtin_amdgcn_rsq(__builtin_fabs(a)), 0x1p+500);
  double g = a * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, a);
  g = fma(d, h, g);
  d = fma(-g, g, a);
  g = fma(d, h, g);
  return g;
}

// The FP64 normal pair in two stages, so that a kernel can issue its own loads in between:
// normal_start runs Philox, forms both uniforms and issues the load of the angle's table entry;
// normal_finish evaluates the logarithm, the square root and the short sine/cosine series.
struct PendingNormals {
  double u1, r;  // radial uniform; angle remainder r = t - k/128
  double sk, ck; // sin(pi k/128), cos(pi k/128)
};

__device__ __forceinline__ void normal_start(const NoiseArgs& na, uint32_t sid, uint32_t comp,
                                             uint32_t call, PendingNormals& p) {
  uint32_t w0 = call, w1, w2, w3, k0, k1;
  noise_key(na, sid, comp, k0, k1, w1, w2, w3);
  philox4x32_10(w0, w1, w2, w3, k0, k1);
  p.u1 = uniform53(w0, w1);
  const double t = 2.0 * uniform53(w2, w3);
  const double kf = rint(128.0 * t);
  p.r = fma(-0.0078125, kf, t);
  const int k = (int)kf & 255;
  p.sk = kSinCosPi128[k][0];
  p.ck = kSinCosPi128[k][1];
}

__device__ __forceinline__ void normal_finish(const NoiseArgs& na, const PendingNormals& p,
                                              double& z0, double& z1) {
  const BoxMullerCoef& c = na.bm;
  const double rad = sqrt_bm(neg2_log_unit(p.u1, c));
  const double z = p.r * p.r;
  const double S = p.r * fma(z, fma(z, fma(z, c.sn[3], c.sn[2]), c.sn[1]), c.sn[0]);
  const double C = fma(z, fma(z, fma(z, c.cs[2], c.cs[1]), c.cs[0]), 1.0);
  z0 = rad * fma(p.ck, C, -(p.sk * S));
  z1 = rad * fma(p.sk, C, p.ck * S);
}

// Two normals of call `call` in stream (sid | comp<<16) at the given cycle.
__device__ __forceinline__ void normal_pair(const NoiseArgs& na, uint32_t sid, uint32_t comp,
                                            uint32_t call, double& z0, double& z1) {
  PendingNormals p;
  normal_start(na, sid, comp, call, p);
  normal_finish(na, p, z0, z1);
}

// The same normals (to rounding) without the table load: the level-0 colour passes use this form
// so that the angle never waits behind their field loads.
__device__ __forceinline__ void normal_pair_notable(const NoiseArgs& na, uint32_t sid,
                                                    uint32_t comp, uint32_t call, double& z0,
                                                    double& z1) {
  uint32_t w0 = call, w1, w2, w3, k0, k1;
  noise_key(na, sid, comp, k0, k1, w1, w2, w3);
  philox4x32_10(w0, w1, w2, w3, k0, k1);
  const double rad = sqrt_bm(neg2_log_unit(uniform53(w0, w1), na.bm));
  double s, c;
  sincospi_quarter(uniform53_x2(w2, w3), na.bm, s, c);
  z0 = rad * c;
  z1 = rad * s;
}

// FP32 variant for the FP32 sweeps of the refined mode: the same Philox words and the same
// 53-bit uniforms, rounded to FP32 (full relative precision down to the smallest uniform, so
// the tail is not clipped), then the hardware log2 / sin / cos (v_sin_f32 and v_cos_f32 take
// revolutions, so the angle 2 pi u2 needs no multiplication by pi).  The normals differ from
// the FP64 ones only by FP32 rounding.
__device__ __forceinline__ void normal_pair_f32(const NoiseArgs& na, uint32_t sid, uint32_t comp,
                                                uint32_t call, float& z0, float& z1) {
  uint32_t w0 = call, w1, w2, w3, k0, k1;
  noise_key(na, sid, comp, k0, k1, w1, w2, w3);
  philox4x32_10(w0, w1, w2, w3, k0, k1);
  const float u1 = (float)uniform53(w0, w1);
  const float u2 = (float)uniform53(w2, w3);
  const float r = __builtin_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u1));
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

// normals in the storage precision T of the sweep, stream sid (default: na.sid)
template <typename T>
__device__ __forceinline__ void normal_pair_t(const NoiseArgs& na, uint32_t sid, uint32_t comp,
                                              uint32_t call, T& z0, T& z1);
template <>
__device__ __forceinline__ void normal_pair_t<double>(const NoiseArgs& na, uint32_t sid,
                                                      uint32_t comp, uint32_t call, double& z0,
                                                      double& z1) {
  normal_pair(na, sid, comp, call, z0, z1);
}
template <>
__device__ __forceinline__ void normal_pair_t<float>(const NoiseArgs& na, uint32_t sid,
                                                     uint32_t comp, uint32_t call, float& z0,
                                                     float& z1) {
  normal_pair_f32(na, sid, comp, call, z0, z1);
}
template <typename T>
__device__ __forceinline__ void normal_pair_t(const NoiseArgs& na, uint32_t comp, uint32_t call,
                                              T& z0, T& z1) {
  normal_pair_t<T>(na, na.sid, comp, call, z0, z1);
}

}  // namespace smg
