// Device helpers shared by the pair kernels: the Gaussian radial basis with its
// first two derivatives in the distance, and the indexing of unordered pairs
// (same-spin pairs of each spin block, then up-down pairs, then
// electron-nucleus pairs).
#pragma once

#include <type_traits>

#include "kernels.h"

namespace qmc {

// s = dmax / (K - 1) is the spacing (and width) of the Gaussians, inv_s its reciprocal
__device__ inline double rbf_spacing(double dmax, int K) { return dmax / (K - 1); }

__device__ inline void rbf3(double d, int k, double s, double inv_s, double& r0, double& r1, double& r2) {
  const double x = (d - k * s) * inv_s;
  r0 = exp(-x * x);
  r1 = -2.0 * x * inv_s * r0;
  r2 = (4.0 * x * x - 2.0) * (inv_s * inv_s) * r0;
}

// The same basis for kernels whose outputs are rounded to S.  For float, the exponent
// y = -x^2 log2(e) is formed in float64 and split into an integer n and a fraction f in [0, 1),
// and only 2^f is taken in float32 (the hardware exp2), scaled by 2^n: about one float32 rounding
// at any argument, against a float64 exponential's several dozen float64 instructions.  A NaN
// distance gives NaN; exponents below -200 give 0.
template <typename S>
__device__ inline void rbf3_as(double d, int k, double s, double inv_s, double& r0, double& r1, double& r2) {
  if constexpr (std::is_same<S, float>::value) {
    const double x = (d - k * s) * inv_s;
    double y = -(x * x) * 1.4426950408889634;  // log2(e)
    if (y < -200.0) y = -200.0;
    const double fl = floor(y);
    r0 = (double)ldexpf(__builtin_amdgcn_exp2f((float)(y - fl)), (int)fl);
    r1 = -2.0 * x * inv_s * r0;
    r2 = (4.0 * x * x - 2.0) * (inv_s * inv_s) * r0;
  } else {
    rbf3(d, k, s, inv_s, r0, r1, r2);
  }
}

// unordered pair index of electrons i != j inside their edge type (0 same-spin, 1 up-down)
__device__ inline int ee_pair(const SysDev& s, int i, int j, int& type) {
  const bool ui = i < s.nup, uj = j < s.nup;
  if (ui != uj) {
    type = 1;
    const int a = ui ? i : j, b = ui ? j : i;
    return a * s.ndn + (b - s.nup);
  }
  type = 0;
  int a = i < j ? i : j, b = i < j ? j : i;
  int n = s.nup, off = 0;
  if (!ui) {
    n = s.ndn;
    a -= s.nup;
    b -= s.nup;
    off = s.nup * (s.nup - 1) / 2;
  }
  return off + a * (2 * n - a - 1) / 2 + (b - a - 1);
}

__device__ inline void decode_pair(const SysDev& s, int type, int p, int& i, int& j) {
  if (type == 2) {
    i = p / s.M;
    j = p % s.M;
    return;
  }
  if (type == 1) {
    i = p / s.ndn;
    j = s.nup + p % s.ndn;
    return;
  }
  int n = s.nup, base = 0;
  const int cu = s.nup * (s.nup - 1) / 2;
  if (p >= cu) {
    p -= cu;
    n = s.ndn;
    base = s.nup;
  }
  int a = 0;
  while (p >= n - 1 - a) {
    p -= n - 1 - a;
    ++a;
  }
  i = base + a;
  j = base + a + 1 + p;
}

}  // namespace qmc
