// Normal variates of libxg's kernels (gfx950): the Box-Muller map on a pair
// of generator outputs, with the angle reduced exactly, and the grouped
// compensated sums used by the fused moments.  Shared by every family member's kernels.
//
// u1 = ((e >> 8) + 1) 2^-24 in (0, 1] and u2 = (o >> 8) 2^-24 in [0, 1) are
// exact; z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2), rho = sqrt(-2 ln u1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg_device.h"

namespace xg {
namespace dev {

// sin and cos of the angle 2 pi u2, u2 = (o >> 8) 2^-24, with the angle
// reduced exactly in integer arithmetic on the word o.  With m = o >> 8,
// 4 u2 = m 2^-22 = q + 2f, where q = floor(4 u2 + 1/2) is the quadrant and
// |f| <= 1/4, so 2 pi u2 = q pi/2 + pi f.  Adding 2^29 to o leaves q mod 4 in
// bits 31:30 and (with o's low 8 bits cleared) 2^29 + f 2^31 in bits 29:0,
// so f is exact.  sin(pi f) and cos(pi f) come from polynomials in t = f^2:
// sin(pi f) = f (pi + t (S3 + t (S5 + t S7))) and cos(pi f) = 1 + t (C2 +
// t (C4 + t (C6 + t C8))), with the coefficients of least maximum relative
// error on |f| <= 1/4 (3.8e-9 and 6.4e-11; sincos_fit.py computes them), the
// leading pi f of the sine formed with pi split as pi_hi + pi_lo so that it
// is rounded once.  A quarter-turn rotation by q finishes: odd q swaps sin
// and cos, and the sign bits come straight from the sum (sin is negated in
// quadrants 2 and 3, cos in quadrants 1 and 2).  f = 0 gives exact zeros and
// ones.
constexpr double kPi = 3.14159265358979323846;
constexpr float kPiHi = (float)kPi;
constexpr float kPiLo = (float)(kPi - (double)kPiHi);
constexpr float kS3 = -0x1.4abbbep+2f;
constexpr float kS5 = 0x1.466004p+1f;
constexpr float kS7 = -0x1.2dc85p-1f;
constexpr float kC2 = -0x1.3bd3ccp+2f;
constexpr float kC4 = 0x1.03c1dep+2f;
constexpr float kC6 = -0x1.55c5ep+0f;
constexpr float kC8 = 0x1.d9d57cp-3f;

// sin(pi f) and cos(pi f) of qf = o + 2^29 (f in bits 29:0, as above).
__device__ __forceinline__ void sincos_pi_f(uint32_t qf, float &sp, float &cp) {
  const float f = fmaf((float)(qf & 0x3FFFFF00u), 0x1p-31f, -0.25f);  // exact (22-bit integer, dyadic result)
  const float t = f * f;
  float p = fmaf(kS7, t, kS5);
  p = fmaf(p, t, kS3);
  const float tail = fmaf(p, t, kPiLo);          // pi_lo + t (S3 + t (S5 + t S7))
  sp = fmaf(f, kPiHi, f * tail);                 // sin(pi f)
  float r = fmaf(kC8, t, kC6);
  r = fmaf(r, t, kC4);
  r = fmaf(r, t, kC2);
  cp = fmaf(r, t, 1.0f);                         // cos(pi f)
}

__device__ __forceinline__ void sincos_turn(uint32_t o, float &s, float &c) {
  const uint32_t qf = o + 0x20000000u;
  float sp, cp;
  sincos_pi_f(qf, sp, cp);
  const uint32_t odd = (uint32_t)((int32_t)(qf << 1) >> 31);  // all ones for odd q
  const uint32_t spb = __float_as_uint(sp), cpb = __float_as_uint(cp);
  s = __uint_as_float(xor_and(select_bits(cpb, spb, odd), qf, 0x80000000u));
  c = __uint_as_float(xor_and(select_bits(spb, cpb, odd), qf + 0x40000000u, 0x80000000u));
}

// The same two values without the swap of odd quadrants.  Turning
// (cos pi f, sin pi f) by q quarter turns gives (cos, sin) = (cp, sp),
// (-sp, cp), (-cp, -sp), (sp, -cp) for q = 0, 1, 2, 3: cp is negated exactly
// in quadrants 2 and 3 (the sine's rule) and sp exactly in quadrants 1 and 2
// (the cosine's rule), wherever each one lands.  So a = cos and b = sin for
// even q, a = sin and b = cos for odd q: the same two floats as sincos_turn,
// in an order that depends on q.
__device__ __forceinline__ void sincos_turn_unordered(uint32_t o, float &a, float &b) {
  const uint32_t qf = o + 0x20000000u;
  float sp, cp;
  sincos_pi_f(qf, sp, cp);
  a = __uint_as_float(xor_and(__float_as_uint(cp), qf, 0x80000000u));
  b = __uint_as_float(xor_and(__float_as_uint(sp), qf + 0x40000000u, 0x80000000u));
}

// rho = sqrt(-2 ln u1), u1 = ((e >> 8) + 1) 2^-24 in [2^-24, 1].  u1 is never
// denormal, infinite or NaN, so no special-case guards: the hardware base-2
// logarithm (within 1 ulp, relative, for every such u1), times -2 ln 2 held
// as two floats (one rounding), gives x = -2 ln u1, and the hardware square
// root (v_sqrt_f32) gives rho.  Over all 2^24 values of u1, rho is within
// 1.55 ulp of sqrt(-2 ln u1) (a reciprocal square root refined by a Newton
// step, four instructions more, was within 1.59).  u1 = 1 gives x = -0 and
// rho = -0.
constexpr double kLn2 = 0.69314718055994530942;
constexpr float kM2Ln2Hi = (float)(-2.0 * kLn2);
constexpr float kM2Ln2Lo = (float)(-2.0 * kLn2 - (double)kM2Ln2Hi);

__device__ __forceinline__ float rho_of(uint32_t e) {
  const float u1 = fmaf((float)(e >> 8), 0x1p-24f, 0x1p-24f);  // exact
  const float l2 = __builtin_amdgcn_logf(u1);
  const float x = fmaf(l2, kM2Ln2Hi, l2 * kM2Ln2Lo);
  return __builtin_amdgcn_sqrtf(x);
}

__device__ __forceinline__ void box_muller(uint32_t e, uint32_t o, float &z0, float &z1) {
  const float rho = rho_of(e);
  float s, c;
  sincos_turn(o, s, c);
  z0 = rho * c;
  z1 = rho * s;
}

// box_muller's two variates as {za, zb} = {z0, z1} (za = z1 in odd
// quadrants), for sums over whole pairs, where the order within a pair does
// not matter: three integer operations fewer than box_muller.
__device__ __forceinline__ void box_muller_unordered(uint32_t e, uint32_t o, float &za, float &zb) {
  const float rho = rho_of(e);
  float a, b;
  sincos_turn_unordered(o, a, b);
  za = rho * a;
  zb = rho * b;
}

// Sums of z and z^2 kept by one lane: each pair is added first (z0 + z1, and
// z0^2 + z1^2 as one FMA over the rounded z0^2), pairs accumulate plainly in
// a group of at most four, and each group enters a compensated (Kahan) sum.
struct Moments {
  float s1, c1, s2, c2;  // compensated sums of z and z^2
  float g1, g2;          // plain sums of the open group (-0 when empty)
};

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

__device__ __forceinline__ void group_add(Moments &m, float z0, float z1) {
  m.g1 = m.g1 + (z0 + z1);
  m.g2 = m.g2 + __builtin_fmaf(z1, z1, z0 * z0);
}

__device__ __forceinline__ void group_close(Moments &m) {
  kahan_add(m.s1, m.c1, m.g1);
  kahan_add(m.s2, m.c2, m.g2);
  m.g1 = -0.0f;  // x + -0 == x, so the next group's first add is free
  m.g2 = -0.0f;
}

}  // namespace dev
}  // namespace xg
