// fastmath.hpp -- compact float32 sin/cos/exp for the per-voxel transmission.
//
// Written from the Taylor series of sin, cos and exp with Cody-Waite
// argument reduction (the reduction constant split into a high part with
// trailing zero bits and a low correction, so k * C_hi is exact in fp32 for
// the supported range of k).  After reduction |r| <= pi/4 (sin/cos) or
// |r| <= ln2/2 (exp); the truncated series errors are below 1e-10 there,
// far under the fp32 rounding of the arithmetic itself.
//
// Range: |x| < 2^15 rad for sincos (k * pi/2 hi part stays exact), and the
// normal float range for exp.  The multislice phases k*dz*delta are far
// inside that range; larger arguments lose accuracy gradually.
#pragma once
#include <hip/hip_runtime.h>

namespace adorym {

// sin r, cos r for |r| <= pi/4 (no argument reduction).
__device__ __forceinline__ void sincos_small_f32(float r, float& s, float& c) {
  const float r2 = r * r;
  float ps = fmaf(r2, -2.5052108385441718775e-8f, 2.7557319223985890653e-6f);
  ps = fmaf(r2, ps, -1.9841269841269841270e-4f);
  ps = fmaf(r2, ps, 8.3333333333333333333e-3f);
  ps = fmaf(r2, ps, -1.6666666666666666667e-1f);
  s = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, 2.0876756987868098979e-9f, -2.7557319223985890653e-7f);
  pc = fmaf(r2, pc, 2.4801587301587301587e-5f);
  pc = fmaf(r2, pc, -1.3888888888888888889e-3f);
  pc = fmaf(r2, pc, 4.1666666666666666667e-2f);
  pc = fmaf(r2, pc, -0.5f);
  c = fmaf(r2, pc, 1.0f);
}

// sin(x), cos(x) for |x| < 2^15.
__device__ __forceinline__ void sincos_f32(float x, float& s, float& c) {
  // pi/2 split: hi has 8 trailing zero bits so k*hi is exact for |k| < 2^16.
  constexpr float kTwoOverPi = 0.636619772367581343f;
  constexpr float kPio2Hi = 1.5707963705062866211f;     // float nearest pi/2
  constexpr float kPio2Lo = -4.3711388286737928865e-8f; // pi/2 - hi
  const float kf = rintf(x * kTwoOverPi);
  // hi part as an exact product split
  float r = fmaf(-kf, kPio2Hi, x);
  r = fmaf(-kf, kPio2Lo, r);
  const int k = (int)kf;
  const float r2 = r * r;
  // sin r = r - r^3/3! + r^5/5! - r^7/7! + r^9/9! - r^11/11!
  float ps = fmaf(r2, -2.5052108385441718775e-8f, 2.7557319223985890653e-6f);
  ps = fmaf(r2, ps, -1.9841269841269841270e-4f);
  ps = fmaf(r2, ps, 8.3333333333333333333e-3f);
  ps = fmaf(r2, ps, -1.6666666666666666667e-1f);
  const float sr = fmaf(r * r2, ps, r);
  // cos r = 1 - r^2/2! + r^4/4! - ... + r^12/12!
  float pc = fmaf(r2, 2.0876756987868098979e-9f, -2.7557319223985890653e-7f);
  pc = fmaf(r2, pc, 2.4801587301587301587e-5f);
  pc = fmaf(r2, pc, -1.3888888888888888889e-3f);
  pc = fmaf(r2, pc, 4.1666666666666666667e-2f);
  pc = fmaf(r2, pc, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  // rotate by k quarter turns (branch-free selects)
  const bool swap = (k & 1) != 0;
  const float s0 = swap ? cr : sr;
  const float c0 = swap ? sr : cr;
  s = (k & 2) ? -s0 : s0;
  c = ((k + 1) & 2) ? -c0 : c0;
}

// exp(x) for float x (flushes to 0 / inf outside the float range).
__device__ __forceinline__ float exp_f32(float x) {
  constexpr float kLog2e = 1.44269504088896340736f;
  constexpr float kLn2Hi = 0.693145751953125f;          // 12 significant bits
  constexpr float kLn2Lo = 1.42860682030941723212e-6f;  // ln2 - hi
  x = fminf(fmaxf(x, -103.0f), 88.7f);
  const float kf = rintf(x * kLog2e);
  float r = fmaf(-kf, kLn2Hi, x);
  r = fmaf(-kf, kLn2Lo, r);
  // exp r, |r| <= 0.347: Taylor to r^8
  float p = fmaf(r, 2.4801587301587301587e-5f, 1.9841269841269841270e-4f);
  p = fmaf(r, p, 1.3888888888888888889e-3f);
  p = fmaf(r, p, 8.3333333333333333333e-3f);
  p = fmaf(r, p, 4.1666666666666666667e-2f);
  p = fmaf(r, p, 1.6666666666666666667e-1f);
  p = fmaf(r, p, 0.5f);
  p = fmaf(r, p, 1.0f);
  p = fmaf(r, p, 1.0f);
  return ldexpf(p, (int)kf);
}

// exp(x) through the hardware base-2 exponential (1 ulp) of x log2(e); the
// rounding of the product adds |x| * 2^-24 relative error, negligible for
// the attenuations here (|x| << 1).  Flushes to 0 / inf outside the range.
__device__ __forceinline__ float exp_hw(float x) {
  return __builtin_amdgcn_exp2f(1.44269504088896340736f * x);
}

}  // namespace adorym
