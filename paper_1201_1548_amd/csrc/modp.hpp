// Arithmetic modulo the table primes 2^30 < p < 2^32 / 3, for host and gfx950
// device code.
//
// Montgomery representation with R = 2^32 (Montgomery, "Modular multiplication
// without trial division", Math. Comp. 44, 1985): x is held as xR mod p.
// redc(t) = t R^{-1} mod p for any t < p 2^32: t + m p < p 2^33 < 2^64 and the
// result is below 2p, which one conditional subtraction fixes; min(r, r - p)
// is that subtraction in unsigned arithmetic (r - p wraps above r exactly when
// r < p).  Since 3p < 2^32, one reduction serves a single product or a sum of
// two or three products of residues (t < 3p^2 < p 2^32).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define BIRES_HD __host__ __device__ __forceinline__
#else
#define BIRES_HD inline
#endif

namespace bires {

struct ModP {
  uint32_t p;     // the prime
  uint32_t pinv;  // -p^{-1} mod 2^32
  uint32_t r2;    // R^2 mod p: Montgomery form of R, and to_mont multiplier
  uint32_t one;   // R mod p: Montgomery form of 1
};

BIRES_HD uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

BIRES_HD uint32_t redc(uint64_t t, uint32_t p, uint32_t pinv) {
  uint32_t m = (uint32_t)t * pinv;
  uint64_t u = t + (uint64_t)m * p;
  uint32_t r = (uint32_t)(u >> 32);
  return umin32(r, r - p);
}

BIRES_HD uint32_t mmul(uint32_t a, uint32_t b, const ModP& q) { return redc((uint64_t)a * b, q.p, q.pinv); }

// (a b + c d) R^{-1} mod p with a single reduction.
BIRES_HD uint32_t mdot2(uint32_t a, uint32_t b, uint32_t c, uint32_t d, const ModP& q) {
  return redc((uint64_t)a * b + (uint64_t)c * d, q.p, q.pinv);
}

// (a b + c d + e f) R^{-1} mod p with a single reduction (residues below p).
BIRES_HD uint32_t mdot3(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e, uint32_t f, const ModP& q) {
  return redc((uint64_t)a * b + (uint64_t)c * d + (uint64_t)e * f, q.p, q.pinv);
}

BIRES_HD uint32_t madd(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t s = a + b;
  return umin32(s, s - p);
}

BIRES_HD uint32_t msub(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t d = a - b;
  return umin32(d, d + p);
}

BIRES_HD uint32_t mneg(uint32_t a, uint32_t p) { return a ? p - a : 0u; }

// -a for a residue a < p that only serves as a factor of mmul/mdot2/mdot3:
// p - a, which is p (congruent to 0) for a = 0.  Factors up to p keep every
// bound above (a sum of three products stays below 3p^2 < p 2^32), and the
// results are still below p; one instruction instead of three.
BIRES_HD uint32_t mneg_factor(uint32_t a, uint32_t p) { return p - a; }

BIRES_HD uint32_t to_mont(uint32_t a, const ModP& q) { return mmul(a, q.r2, q); }   // any 32-bit a (a r2 < p 2^32)
BIRES_HD uint32_t from_mont(uint32_t a, const ModP& q) { return redc((uint64_t)a, q.p, q.pinv); }

// x mod p for any 32-bit x (x < 4p because p > 2^30).
BIRES_HD uint32_t reduce32(uint32_t x, uint32_t p) {
  x = umin32(x, x - 2u * p);
  return umin32(x, x - p);
}

// Montgomery power: a in Montgomery form, result (a^e) in Montgomery form.
BIRES_HD uint32_t mpow(uint32_t a, uint32_t e, const ModP& q) {
  uint32_t r = q.one;
  while (e) {
    if (e & 1u) r = mmul(r, a, q);
    a = mmul(a, a, q);
    e >>= 1;
  }
  return r;
}

// Inverse by Fermat's little theorem; a in Montgomery form, a != 0.
BIRES_HD uint32_t minv(uint32_t a, const ModP& q) { return mpow(a, q.p - 2u, q); }

}  // namespace bires
