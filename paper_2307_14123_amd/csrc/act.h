// Activation helpers of the float32 kernels.
#pragma once

namespace qmc {

// float32 tanh from two branch-free pieces, both evaluated, one selected:
//  |x| < 0.625: tanh x = x + x^3 p(x^2), p a quartic fitted to (tanh x - x) / x^3 by weighted
//               least squares with Lawson reweighting toward minimax relative error (max relative
//               error 8e-8 evaluated in float32);
//  otherwise:   tanh |x| = 1 - 2 / (exp(2|x|) + 1) with the hardware exponential and reciprocal
//               (no cancellation since tanh |x| > 0.55; +-inf give +-1, NaN propagates).
__device__ inline float tanh_f32(float x) {
  const float ax = fabsf(x), y = x * x;
  float p = -0.005789994727820158f;
  p = fmaf(p, y, 0.020713651552796364f);
  p = fmaf(p, y, -0.05376197770237923f);
  p = fmaf(p, y, 0.1333169937133789f);
  p = fmaf(p, y, -0.333332896232605f);
  const float small = fmaf(x * y, p, x);
  const float e = __expf(2.f * ax);
  const float big = copysignf(1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f), x);
  return ax < 0.625f ? small : big;
}

}  // namespace qmc
