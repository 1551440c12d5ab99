// Normal variates of libxg's kernels (gfx950): the Box-Muller map on a pair
// of generator outputs, with the angle reduced exactly, and the compensated
// sum used by the fused moments.  Shared by every family member's kernels.
//
// u1 = ((e >> 8) + 1) 2^-24 in (0, 1] and u2 = (o >> 8) 2^-24 in [0, 1) are
// exact; z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2), rho = sqrt(-2 ln u1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xg {
namespace dev {

// sin(pi x) and cos(pi x) for x = 2 u2 in [0, 2), a multiple of 2^-23.  The
// argument is reduced exactly: 2x = q + 2f with q = rint(2x), |f| <= 1/4, so
// pi x = q pi / 2 + pi f.  sin(pi f) and cos(pi f) come from their Taylor
// series in t = f^2 (the first omitted terms are below 2e-9 and 1.2e-10
// relative at |f| = 1/4), the leading pi f of the sine formed with pi split
// as pi_hi + pi_lo so that it is rounded once.  A quarter-turn rotation by q
// finishes.  f = 0 gives exact zeros and ones.
constexpr double kPi = 3.14159265358979323846;
constexpr float kPiHi = (float)kPi;
constexpr float kPiLo = (float)(kPi - (double)kPiHi);
constexpr float kS3 = (float)(-kPi * kPi * kPi / 6.0);
constexpr float kS5 = (float)(kPi * kPi * kPi * kPi * kPi / 120.0);
constexpr float kS7 = (float)(-kPi * kPi * kPi * kPi * kPi * kPi * kPi / 5040.0);
constexpr float kS9 = (float)(kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi / 362880.0);
constexpr float kC2 = (float)(-kPi * kPi / 2.0);
constexpr float kC4 = (float)(kPi * kPi * kPi * kPi / 24.0);
constexpr float kC6 = (float)(-kPi * kPi * kPi * kPi * kPi * kPi / 720.0);
constexpr float kC8 = (float)(kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi / 40320.0);
constexpr float kC10 = (float)(-kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi * kPi / 3628800.0);

__device__ __forceinline__ void sincospi_unit(float x, float &s, float &c) {
  const float y = 2.0f * x;            // exact
  const float q = rintf(y);            // exact integer 0 .. 4
  const float f = (y - q) * 0.5f;      // exact, |f| <= 1/4
  const float t = f * f;
  float p = fmaf(kS9, t, kS7);
  p = fmaf(p, t, kS5);
  p = fmaf(p, t, kS3);
  const float tail = fmaf(p, t, kPiLo);          // pi_lo + t (S3 + t (S5 + t (S7 + t S9)))
  const float sp = fmaf(f, kPiHi, f * tail);     // sin(pi f)
  float r = fmaf(kC10, t, kC8);
  r = fmaf(r, t, kC6);
  r = fmaf(r, t, kC4);
  r = fmaf(r, t, kC2);
  const float cp = fmaf(r, t, 1.0f);             // cos(pi f)
  const uint32_t qi = (uint32_t)(int)q;
  const bool odd = (qi & 1u) != 0;
  const float s0 = odd ? cp : sp, c0 = odd ? sp : cp;
  // sin is negated in quadrants 2, 3; cos in quadrants 1, 2
  s = __uint_as_float(__float_as_uint(s0) ^ ((qi & 2u) << 30));
  c = __uint_as_float(__float_as_uint(c0) ^ (((qi + 1u) & 2u) << 30));
}

__device__ __forceinline__ void box_muller(uint32_t e, uint32_t o, float &z0, float &z1) {
  const float u1 = (float)((e >> 8) + 1u) * 0x1p-24f;  // (0, 1], exact
  const float u2 = (float)(o >> 8) * 0x1p-24f;         // [0, 1), exact
  const float rho = sqrtf(-2.0f * logf(u1));
  float s, c;
  sincospi_unit(2.0f * u2, s, c);                      // angle 2 pi u2 reduced exactly
  z0 = rho * c;
  z1 = rho * s;
}

struct Moments {
  float s1, c1, s2, c2;  // compensated sums of z and z^2
};

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

}  // namespace dev
}  // namespace xg
