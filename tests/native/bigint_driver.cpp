// Test driver for the host big-integer helpers: reads "op x y" lines with
// signed hexadecimal operands from stdin and prints results in hexadecimal.
#include <cstdio>
#include <iostream>
#include <string>

#include "../../paper_1201_1548_amd/csrc/bigint.hpp"

using namespace bires;

static BigInt parse(const std::string& s) {
  BigInt r;
  size_t i = 0;
  if (s[0] == '-') {
    r.neg = true;
    i = 1;
  }
  std::string h = s.substr(i);
  for (size_t end = h.size(); end > 0;) {
    size_t beg = end >= 8 ? end - 8 : 0;
    r.mag.push_back((uint32_t)std::stoul(h.substr(beg, end - beg), nullptr, 16));
    end = beg;
  }
  trim(r.mag);
  if (r.mag.empty()) r.neg = false;
  return r;
}

static std::string show(const BigInt& x) {
  if (x.mag.empty()) return "0";
  std::string s = x.neg ? "-" : "";
  char buf[16];
  snprintf(buf, sizeof buf, "%x", x.mag.back());
  s += buf;
  for (size_t i = x.mag.size() - 1; i-- > 0;) {
    snprintf(buf, sizeof buf, "%08x", x.mag[i]);
    s += buf;
  }
  return s;
}

int main() {
  std::string op, a, b;
  while (std::cin >> op >> a >> b) {
    BigInt x = parse(a), y = parse(b);
    if (op == "mul") {
      std::cout << show(big_mul(x, y)) << "\n";
    } else if (op == "divmod") {
      BigInt q, r;
      divmod_mag(x.mag, y.mag, q.mag, r.mag);
      std::cout << show(q) << " " << show(r) << "\n";
    } else if (op == "gcd") {
      std::cout << show(big_gcd(x, y)) << "\n";
    } else if (op == "modsmall") {
      std::cout << std::hex << big_mod_small(x, (uint32_t)y.mag[0]) << std::dec << "\n";
    } else if (op == "twos") {  // round trip through L = y limbs
      std::vector<uint32_t> l(y.mag[0]);
      x.to_twos(l.data(), (int)l.size());
      std::cout << show(BigInt::from_twos(l.data(), (int)l.size())) << " " << x.bits() << "\n";
    } else if (op == "divexact") {
      BigInt q;
      bool ok = big_divexact(x, y, q);
      std::cout << (ok ? show(q) : std::string("inexact")) << "\n";
    }
  }
  return 0;
}
