// Minimal host big integers for the gcd's normalisation (contents, exact
// quotients, the gcd of leading coefficients).  Sign-magnitude, 32-bit limbs,
// little endian; the magnitude has no leading zero limbs (zero = empty).
#pragma once
#include <stdint.h>

#include <vector>

namespace bires {

struct BigInt {
  bool neg = false;
  std::vector<uint32_t> mag;

  bool is_zero() const { return mag.empty(); }
  int bits() const;                                   // bit length of |x| (0 for zero)
  static BigInt from_twos(const uint32_t* limbs, int L);  // two's complement input
  void to_twos(uint32_t* limbs, int L) const;         // sign-extended; caller checks the size
  static BigInt from_u64(uint64_t v);
};

void trim(std::vector<uint32_t>& m);
int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b);
BigInt big_abs(const BigInt& a);
BigInt big_add(const BigInt& a, const BigInt& b);
BigInt big_mul(const BigInt& a, const BigInt& b);
// Quotient and remainder of |a| by |b| (b != 0), Knuth's algorithm D.
void divmod_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b, std::vector<uint32_t>& q,
                std::vector<uint32_t>& r);
// a / b for b dividing a exactly (signs handled); returns false if not exact.
bool big_divexact(const BigInt& a, const BigInt& b, BigInt& q);
// gcd(|a|, |b|) by Euclid with Knuth-D remainders (gcd(0, 0) = 0).
BigInt big_gcd(const BigInt& a, const BigInt& b);
uint32_t big_mod_small(const BigInt& a, uint32_t p);  // a mod p in [0, p)

}  // namespace bires
