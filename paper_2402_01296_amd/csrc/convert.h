// Device helpers for exact mixed-radix (Garner) conversion between RNS bases.
#pragma once

#include "internal.h"

namespace bcn {

// Workgroups of a launch go to the eight XCDs in turn (workgroup i to XCD i mod 8) and every
// XCD has an L2 of its own.  xcd_order renumbers the workgroups so that each XCD walks one
// contiguous stretch of a work list: in the transforms a limb-major list, so all workgroups of
// one limb run on one or two XCDs, whose L2 keeps that limb's twiddle (and key) tables resident.
__device__ __forceinline__ int xcd_order(int bid, int total) {
  constexpr int X = 8;
  const int per = total / X, rem = total % X, x = bid % X;
  return x * per + min(x, rem) + bid / X;
}

// Mixed-radix digits of x over the first NS limbs of cv.src.
template <int NS>
__device__ __forceinline__ void garner(const double (&x)[NS], double (&v)[NS], const Conv& cv, const Mod* mods) {
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const Mod mi = mods[cv.src[i]];
    double u = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) u = mul_lazy(u - v[k], cv.ginv[i][k], mi);
    v[i] = norm(u, mi);
  }
}

// true when sum_{k<n} v_k M_k > (M-1)/2, i.e. the centred value is negative
template <int NS>
__device__ __forceinline__ bool above_half(const double (&v)[NS], int n, const Conv& cv, const Mod* mods) {
  bool decided = false, neg = false;
#pragma unroll
  for (int k = NS - 1; k >= 0; --k) {
    if (k < n) {
      const double h = (mods[cv.src[k]].q - 1.0) * 0.5;
      if (!decided && v[k] != h) {
        neg = v[k] > h;
        decided = true;
      }
    }
  }
  return neg;
}

}  // namespace bcn
