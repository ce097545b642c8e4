// Host big-integer helpers (see bigint.hpp).  Division is Knuth's algorithm D
// (TAOCP vol. 2, 4.3.1) on 32-bit digits with 64-bit intermediates.
#include "bigint.hpp"

#include <algorithm>

namespace bires {

void trim(std::vector<uint32_t>& m) {
  while (!m.empty() && m.back() == 0u) m.pop_back();
}

int BigInt::bits() const {
  if (mag.empty()) return 0;
  return 32 * ((int)mag.size() - 1) + (32 - __builtin_clz(mag.back()));
}

BigInt BigInt::from_twos(const uint32_t* limbs, int L) {
  BigInt r;
  const bool neg = (limbs[L - 1] >> 31) != 0u;
  r.mag.assign(limbs, limbs + L);
  if (neg) {  // magnitude = ~x + 1
    uint64_t carry = 1;
    for (auto& w : r.mag) {
      const uint64_t v = (uint64_t)(uint32_t)~w + carry;
      w = (uint32_t)v;
      carry = v >> 32;
    }
  }
  trim(r.mag);
  r.neg = neg && !r.mag.empty();
  return r;
}

void BigInt::to_twos(uint32_t* limbs, int L) const {
  for (int l = 0; l < L; ++l) limbs[l] = l < (int)mag.size() ? mag[l] : 0u;
  if (neg) {
    uint64_t carry = 1;
    for (int l = 0; l < L; ++l) {
      const uint64_t v = (uint64_t)(uint32_t)~limbs[l] + carry;
      limbs[l] = (uint32_t)v;
      carry = v >> 32;
    }
  }
}

BigInt BigInt::from_u64(uint64_t v) {
  BigInt r;
  while (v) {
    r.mag.push_back((uint32_t)v);
    v >>= 32;
  }
  return r;
}

int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

BigInt big_abs(const BigInt& a) {
  BigInt r = a;
  r.neg = false;
  return r;
}

// |a| + |b| and |a| - |b| (|a| >= |b|) on magnitudes.
static std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0u);
  uint64_t carry = 0;
  for (size_t i = 0; i + 1 < r.size(); ++i) {
    const uint64_t s = carry + (i < a.size() ? a[i] : 0u) + (i < b.size() ? b[i] : 0u);
    r[i] = (uint32_t)s;
    carry = s >> 32;
  }
  r.back() = (uint32_t)carry;
  trim(r);
  return r;
}

static std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> r(a.size(), 0u);
  int64_t borrow = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    int64_t s = (int64_t)a[i] - (i < b.size() ? (int64_t)b[i] : 0) - borrow;
    borrow = s < 0 ? 1 : 0;
    r[i] = (uint32_t)(s + (borrow << 32));
  }
  trim(r);
  return r;
}

BigInt big_add(const BigInt& a, const BigInt& b) {
  BigInt r;
  if (a.neg == b.neg) {
    r.mag = add_mag(a.mag, b.mag);
    r.neg = a.neg;
  } else if (cmp_mag(a.mag, b.mag) >= 0) {
    r.mag = sub_mag(a.mag, b.mag);
    r.neg = a.neg;
  } else {
    r.mag = sub_mag(b.mag, a.mag);
    r.neg = b.neg;
  }
  if (r.mag.empty()) r.neg = false;
  return r;
}

BigInt big_mul(const BigInt& a, const BigInt& b) {
  BigInt r;
  if (a.is_zero() || b.is_zero()) return r;
  r.mag.assign(a.mag.size() + b.mag.size(), 0u);
  for (size_t i = 0; i < a.mag.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.mag.size(); ++j) {
      const uint64_t t = (uint64_t)a.mag[i] * b.mag[j] + r.mag[i + j] + carry;
      r.mag[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    size_t k = i + b.mag.size();
    while (carry) {
      const uint64_t t = (uint64_t)r.mag[k] + carry;
      r.mag[k++] = (uint32_t)t;
      carry = t >> 32;
    }
  }
  trim(r.mag);
  r.neg = a.neg != b.neg;
  return r;
}

void divmod_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b, std::vector<uint32_t>& q,
                std::vector<uint32_t>& r) {
  q.clear();
  r.clear();
  if (cmp_mag(a, b) < 0) {
    r = a;
    return;
  }
  const size_t n = b.size(), m = a.size() - b.size();
  if (n == 1) {  // single-digit divisor
    q.assign(a.size(), 0u);
    uint64_t rem = 0;
    for (size_t i = a.size(); i-- > 0;) {
      const uint64_t cur = (rem << 32) | a[i];
      q[i] = (uint32_t)(cur / b[0]);
      rem = cur % b[0];
    }
    trim(q);
    if (rem) r.push_back((uint32_t)rem);
    return;
  }
  // D1: normalise so the divisor's top digit has its high bit set
  const int s = __builtin_clz(b.back());
  std::vector<uint32_t> v(n), u(a.size() + 1);
  for (size_t i = n; i-- > 0;) v[i] = (b[i] << s) | (s && i ? (uint32_t)(b[i - 1] >> (32 - s)) : 0u);
  u[a.size()] = s ? (uint32_t)(a.back() >> (32 - s)) : 0u;
  for (size_t i = a.size(); i-- > 0;) u[i] = (a[i] << s) | (s && i ? (uint32_t)(a[i - 1] >> (32 - s)) : 0u);
  q.assign(m + 1, 0u);
  const uint64_t B = 1ull << 32;
  for (size_t j = m + 1; j-- > 0;) {
    // D3: estimate qhat from the top two digits
    const uint64_t num = ((uint64_t)u[j + n] << 32) | u[j + n - 1];
    uint64_t qhat = num / v[n - 1];
    uint64_t rhat = num % v[n - 1];
    while (qhat >= B || qhat * v[n - 2] > ((rhat << 32) | u[j + n - 2])) {
      --qhat;
      rhat += v[n - 1];
      if (rhat >= B) break;
    }
    // D4: multiply and subtract
    int64_t borrow = 0;
    uint64_t carry = 0;
    for (size_t i = 0; i < n; ++i) {
      const uint64_t p = qhat * v[i] + carry;
      carry = p >> 32;
      const int64_t t = (int64_t)u[i + j] - (int64_t)(uint32_t)p + borrow;
      u[i + j] = (uint32_t)t;
      borrow = t >> 32;
    }
    const int64_t t = (int64_t)u[j + n] - (int64_t)carry + borrow;
    u[j + n] = (uint32_t)t;
    if (t < 0) {  // D6: add back
      --qhat;
      uint64_t c = 0;
      for (size_t i = 0; i < n; ++i) {
        const uint64_t s2 = (uint64_t)u[i + j] + v[i] + c;
        u[i + j] = (uint32_t)s2;
        c = s2 >> 32;
      }
      u[j + n] += (uint32_t)c;
    }
    q[j] = (uint32_t)qhat;
  }
  trim(q);
  // D8: unnormalise the remainder
  r.assign(n, 0u);
  for (size_t i = 0; i < n; ++i) r[i] = (u[i] >> s) | (s ? (uint32_t)((uint64_t)u[i + 1] << (32 - s)) : 0u);
  trim(r);
}

bool big_divexact(const BigInt& a, const BigInt& b, BigInt& q) {
  std::vector<uint32_t> r;
  divmod_mag(a.mag, b.mag, q.mag, r);
  if (!r.empty()) return false;
  q.neg = (a.neg != b.neg) && !q.mag.empty();
  return true;
}

BigInt big_gcd(const BigInt& a, const BigInt& b) {
  std::vector<uint32_t> x = a.mag, y = b.mag, q, r;
  while (!y.empty()) {
    divmod_mag(x, y, q, r);
    x.swap(y);
    y.swap(r);
  }
  BigInt g;
  g.mag = x;
  return g;
}

uint32_t big_mod_small(const BigInt& a, uint32_t p) {
  uint64_t rem = 0;
  for (size_t i = a.mag.size(); i-- > 0;) rem = ((rem << 32) | a.mag[i]) % p;
  if (a.neg && rem) rem = p - rem;
  return (uint32_t)rem;
}

}  // namespace bires
