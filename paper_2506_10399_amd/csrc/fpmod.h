// Exact residue arithmetic in fp64 for primes 2^49 < q < 2^50 (device code).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ficgcn {

// Residue arithmetic in fp64 for 2^49 < q < 2^50 (every Q prime of the chain).
// a, b < q are exact doubles; a*b = hi + lo exactly (fma error term); the
// quotient estimate rint(hi * fl(1/q)) is within 1 of a*b/q (its error is
// below hi/q * 2^-52 + 1/2 + |lo|/q < 1/4 + 1/2 + 1/4), so
// r = (hi - qt*q) + lo, computed exactly by one fma and one add of integers
// below 2^52, lies in (-q, q) and one correction (r < 0: add q) makes it the
// residue.  The
// fp64 FMA runs at full rate, where a 64-bit integer Shoup multiply takes
// about ten quarter-rate 32-bit multiplies; the results are the same words.
// Values travel as the bit patterns of the doubles in the uint64 registers
// and LDS words of the pass.
//
// Inside a transform the values are signed representatives in (-q, q):
//   * the product of a in (-q, q) and a twiddle in [0, q) by the same steps
//     without the correction stays in (-q, q) (|a*b| < q^2, so the estimate
//     error is at most 1/4 + 1/2 + 1/8 of q);
//   * a sum or difference t in (-2q, 2q) is brought back by t - q*rint(t/q),
//     which lands in [-q/2 - 1, q/2 + 1] (t/q is known to 2^-51);
// three fp64 operations each, in place of a compare, an add and two selects.
// Sums are brought back on every other stage only (and on a pass's last stage):
// a product with a in (-2q, 2q) still lands in (-3q/2, 3q/2) (the estimate
// error grows to below 1/2 + 1/2, |lo| < q/2), so the next stage's sums stay
// within (-4q, 4q), exact integers below 2^52, and t - q*rint(t/q) brings them
// back as before.  The last pass maps the values to [0, q) once.
__device__ __forceinline__ uint64_t f2b(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double b2f(uint64_t b) { return __longlong_as_double((long long)b); }
// Exact conversions for integers below 2^52: the double 2^52 + v has v as its
// mantissa field, so the two directions are an OR / AND of the exponent bits
// and one fp64 add (instead of the generic 64-bit conversion sequences).
constexpr uint64_t TWO52_BITS = 0x4330000000000000ull;
constexpr double TWO52 = 4503599627370496.0;
__device__ __forceinline__ uint64_t to_fbits(uint64_t v) { return f2b(b2f(v | TWO52_BITS) - TWO52); }
__device__ __forceinline__ uint64_t from_fbits(uint64_t b) { return f2b(b2f(b) + TWO52) & 0x000FFFFFFFFFFFFFull; }

__device__ __forceinline__ double fmulmod(double a, double b, double q, double qinv) {
  const double hi = a * b;
  const double lo = fma(a, b, -hi);
  const double qt = rint(hi * qinv);
  const double r = fma(-qt, q, hi) + lo;
  return r < 0.0 ? r + q : r;
}

// signed product: a in (-q, q), b in [0, q) -> (-q, q)
__device__ __forceinline__ double fmulmod_s(double a, double b, double q, double qinv) {
  const double hi = a * b;
  const double lo = fma(a, b, -hi);
  const double qt = rint(hi * qinv);
  return fma(-qt, q, hi) + lo;
}
// t in (-2q, 2q) -> (-q, q), congruent
__device__ __forceinline__ double sred(double t, double q, double qinv) { return fma(-rint(t * qinv), q, t); }
// (-q, q) -> [0, q)
__device__ __forceinline__ double canon(double r, double q) { return r < 0.0 ? r + q : r; }

}  // namespace ficgcn
