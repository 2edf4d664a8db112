// Exact modular arithmetic on residues held as binary64 integers.
//
// Every residue of a prime q < 2^41 is stored as a double holding an integer
// in [0, q).  Products are reduced Barrett-style: the quotient is estimated
// in FP64 from a precomputed 1/q, and the remainder is formed exactly with
// fused multiply-adds:
//
//   h  = fl(a*b)                 rounded product
//   l  = fma(a, b, -h)           exact rounding error: a*b = h + l
//   k  = rint(h * (1/q))         quotient estimate, |k - h/q| <= 1/2 + d
//   r  = fma(-k, q, h)           exact: an integer of magnitude <= (1/2 + d) q
//   r  = r + l                   exact, congruent to a*b mod q
//
// With |a| <= q and |b| < 2^46 the estimate error d is below 2^-6 and
// |l| <= q 2^-7, so r lies in (-q, q) ("lazy" form).  All intermediate
// integers stay below 2^53 in magnitude except h, whose rounding is captured
// by l.  On gfx950 each step is one full-rate FP64 VALU instruction, which is
// why residues are FP64 rather than u64 (64-bit integer products are built
// from quarter-rate 32-bit multiplies).
//
// All code using these helpers must be compiled with -ffp-contract=off so
// that the compiler cannot fuse or reassociate the steps above.
#pragma once

#include <hip/hip_runtime.h>

#define BCN_HD __host__ __device__ __forceinline__

namespace bcn {

struct Mod {
  double q;     // the prime, an integer below 2^41
  double qinv;  // 1/q rounded to nearest
};

// a*b mod q in (-q, q).  Requires |a| <= q and |b| < 2^46 (or vice versa).
BCN_HD double mul_lazy(double a, double b, Mod m) {
  double h = a * b;
  double l = fma(a, b, -h);
  double k = rint(h * m.qinv);
  double r = fma(-k, m.q, h);
  return r + l;
}

// (-q, q) -> [0, q)
BCN_HD double norm(double r, Mod m) { return r < 0.0 ? r + m.q : r; }

// any integer |x| < 2^52 -> [0, q)
BCN_HD double reduce(double x, Mod m) {
  double k = rint(x * m.qinv);
  double r = fma(-k, m.q, x);
  return r < 0.0 ? r + m.q : r;
}

// any integer |x| < 2^52 -> (-q/2 - 1, q/2 + 1), congruent mod q
BCN_HD double reduce_lazy(double x, Mod m) {
  double k = rint(x * m.qinv);
  return fma(-k, m.q, x);
}

BCN_HD double mul_mod(double a, double b, Mod m) { return norm(mul_lazy(a, b, m), m); }

BCN_HD double add_mod(double a, double b, Mod m) {
  double s = a + b;
  return s >= m.q ? s - m.q : s;
}

BCN_HD double sub_mod(double a, double b, Mod m) {
  double s = a - b;
  return s < 0.0 ? s + m.q : s;
}

// a*b + c = quo*q + rem exactly, rem in [0, q).  Requires 0 <= a*b < 2^62,
// 0 <= c < 2^22 and q >= 2^24 (the rounding error of a*b plus c then stays
// below q/2, so one correction step on each side suffices).  Used by the
// carry chain of the exact scale-and-round, where a*b can exceed 2^53.
BCN_HD double mul_add_divmod(double a, double b, double c, Mod m, double* quo) {
  double h = a * b;
  double l = fma(a, b, -h) + c;
  double k = rint(h * m.qinv);
  double r = fma(-k, m.q, h) + l;
  if (r < 0.0) { r += m.q; k -= 1.0; }
  if (r >= m.q) { r -= m.q; k += 1.0; }
  *quo = k;
  return r;
}

}  // namespace bcn
