// Word-level modular arithmetic for RNS-CKKS on gfx950 (host-callable too,
// so the same routines can be unit-checked on the CPU).
//
// Moduli are primes q < 2^62.  Residues live in [0, q).
//  * mul_shoup: a * w mod q for a constant w with ws = floor(w * 2^64 / q)
//    (Shoup's precomputed quotient); one high product, two low products.
//  * reduce128: Barrett reduction of a 128-bit value with
//    ratio = floor(2^128 / q); used for variable x variable products and for
//    lazily accumulated sums of such products (up to 2^(128 - 2*bits(q)) terms).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FICGCN_FD __host__ __device__ __forceinline__

namespace ficgcn {

typedef unsigned __int128 u128;

FICGCN_FD uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) >> 64); }

FICGCN_FD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}

FICGCN_FD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

FICGCN_FD uint64_t neg_mod(uint64_t a, uint64_t q) { return a == 0 ? 0 : q - a; }

FICGCN_FD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  uint64_t h = mulhi64(a, ws);
  uint64_t r = a * w - h * q;
  return r >= q ? r - q : r;
}

// Shoup without the final correction: result in [0, 2q) (butterfly-internal use)
FICGCN_FD uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  uint64_t h = mulhi64(a, ws);
  return a * w - h * q;
}

struct Mod {
  uint64_t q;
  uint64_t r_hi, r_lo;   // floor(2^128 / q)
};

// (hi * 2^64 + lo) mod q
FICGCN_FD uint64_t reduce128(uint64_t hi, uint64_t lo, const Mod& m) {
  u128 c = ((u128)lo * m.r_lo) >> 64;
  u128 m1 = (u128)lo * m.r_hi + c;
  u128 m2 = (u128)hi * m.r_lo;
  u128 mid = (u128)(uint64_t)m1 + (uint64_t)m2;
  uint64_t qest = hi * m.r_hi + (uint64_t)(m1 >> 64) + (uint64_t)(m2 >> 64) + (uint64_t)(mid >> 64);
  uint64_t r = lo - qest * m.q;
  if (r >= m.q) r -= m.q;
  if (r >= m.q) r -= m.q;
  return r;
}

FICGCN_FD uint64_t reduce128(u128 x, const Mod& m) { return reduce128((uint64_t)(x >> 64), (uint64_t)x, m); }

FICGCN_FD uint64_t mul_mod(uint64_t a, uint64_t b, const Mod& m) { return reduce128((u128)a * b, m); }

// bit reversal of the low `bits` bits
FICGCN_FD uint32_t bitrev(uint32_t x, int bits) {
#ifdef __HIP_DEVICE_COMPILE__
  return __brev(x) >> (32 - bits);
#else
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
#endif
}

}  // namespace ficgcn
