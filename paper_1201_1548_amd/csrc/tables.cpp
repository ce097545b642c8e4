// Host construction of the prime table and of the mixed-radix constants.
//
// Primes: the K largest primes below 2^32 / 3, descending (deterministic
// Miller-Rabin with bases 2, 7, 61, exact for n < 4,759,123,141).  3p < 2^32
// lets one Montgomery reduction absorb a sum of three products, and p > 2^30
// keeps every 32-bit word below 4p.  Every job uses a prefix of this table, so
// the Garner constants and the radix products prod_{i<k} p_i are computed
// once for all jobs.
#include "tables.hpp"

#include <cmath>
#include <mutex>

namespace bires {

static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

static uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}

static bool is_prime32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t sp : {2u, 3u, 5u, 7u, 11u, 13u, 61u})
    if (n % sp == 0) return n == sp;
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod64(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

ModP make_modp(uint32_t p) {
  ModP q;
  q.p = p;
  uint32_t inv = p;  // Newton iteration for p^{-1} mod 2^32 (p odd)
  for (int i = 0; i < 5; ++i) inv *= 2u - p * inv;
  q.pinv = 0u - inv;
  q.one = (uint32_t)((((uint64_t)1) << 32) % p);
  q.r2 = (uint32_t)(((unsigned __int128)1 << 64) % p);
  return q;
}

static void build(HostTables& t, int K) {
  t.K = K;
  t.primes.clear();
  for (uint32_t c = PRIME_CEIL; (int)t.primes.size() < K; c -= 2)
    if (is_prime32(c)) t.primes.push_back(make_modp(c));
  t.log2p.resize(K);
  t.cumlog.assign(K + 1, 0.0);
  for (int k = 0; k < K; ++k) {
    // a lower bound of log2 p_k (the relative error of log2 is far below 1e-12)
    t.log2p[k] = std::log2((double)t.primes[k].p) - 1e-12;
    t.cumlog[k + 1] = t.cumlog[k] + t.log2p[k];
  }
  mrc_tables(t.primes, t.gm, t.cm, t.pm, t.pi);
}

void mrc_tables(const std::vector<ModP>& primes, std::vector<uint32_t>& gm, std::vector<uint32_t>& cm,
                std::vector<uint32_t>& pm, std::vector<uint32_t>& pi) {
  const int K = (int)primes.size();
  gm.assign((size_t)K * K, 0u);
  cm.assign(K, 0u);
  pm.assign((size_t)K * K, 0u);
  for (int k = 0; k < K; ++k) {
    const uint64_t pk = primes[k].p;
    for (int j = 0; j < k; ++j) pm[(size_t)k * K + j] = (uint32_t)(((uint64_t)(primes[j].p % pk) << 32) % pk);
    uint64_t prod = 1 % pk;  // prod_{i<j} p_i mod p_k
    for (int j = 0; j < k; ++j) {
      gm[(size_t)j * K + k] = (uint32_t)((prod << 32) % pk);
      prod = mulmod64(prod, primes[j].p % pk, pk);
    }
    const uint64_t inv = powmod64(prod, pk - 2, pk);
    cm[k] = (uint32_t)((inv << 32) % pk);
  }
  // prod_{i<k} p_i as k+1 little-endian limbs at offset k(k+1)/2
  pi.assign((size_t)K * (K + 1) / 2 + K + 1, 0u);
  std::vector<uint32_t> cur(1, 1u);
  for (int k = 0; k < K; ++k) {
    uint32_t* dst = &pi[(size_t)k * (k + 1) / 2];
    for (int l = 0; l <= k && l < (int)cur.size(); ++l) dst[l] = cur[l];
    uint64_t carry = 0;
    for (auto& w : cur) {
      const uint64_t v = (uint64_t)w * primes[k].p + carry;
      w = (uint32_t)v;
      carry = v >> 32;
    }
    if (carry) cur.push_back((uint32_t)carry);
  }
}

size_t crt_operand_offset(int P, int LM) { return ((size_t)P + (size_t)P * LM + LM + 3) & ~(size_t)3; }

void crt_operand_tiles(int P, int LM, int* nct, int* nks) {
  *nct = (4 * LM + 4 + 31) / 32;  // byte columns 0..4 LM + 3
  *nks = (P + 7) / 8;             // 4 P contraction indices, 32 per step
}

CrtHost crt_tables(int P) {
  const HostTables& t = host_tables();
  CrtHost c;
  c.P = P;
  std::vector<uint32_t> M(&t.pi[(size_t)P * (P + 1) / 2], &t.pi[(size_t)P * (P + 1) / 2] + P + 1);
  while (M.size() > 1 && M.back() == 0u) M.pop_back();
  const int LM = (int)M.size();
  c.LM = LM;
  int nct = 0, nks = 0;
  crt_operand_tiles(P, LM, &nct, &nks);
  const size_t ob = crt_operand_offset(P, LM);
  c.buf.assign(ob + (size_t)nct * nks * 256, 0u);
  for (int k = 0; k < P; ++k) {
    const ModP& q = t.primes[k];
    // M / p_k by schoolbook division with a one-limb divisor (exact)
    uint32_t* row = &c.buf[(size_t)P + (size_t)k * LM];
    uint64_t rem = 0;
    for (int l = LM - 1; l >= 0; --l) {
      const uint64_t cur = (rem << 32) | M[l];
      row[l] = (uint32_t)(cur / q.p);
      rem = cur % q.p;
    }
    // (M / p_k) mod p_k by Horner over its limbs
    uint64_t r = 0;
    for (int l = LM - 1; l >= 0; --l) r = ((r << 32) | row[l]) % q.p;
    c.buf[k] = minv(to_mont((uint32_t)r, q), q);
  }
  for (int l = 0; l < LM; ++l) c.buf[(size_t)P + (size_t)P * LM + l] = M[l];
  // balanced base-256 digits of each M / p_k: 4 LM bytes plus one top digit
  const int nd = 4 * LM + 1;
  std::vector<int8_t> dig((size_t)P * nd);
  for (int k = 0; k < P; ++k) {
    const uint32_t* row = &c.buf[(size_t)P + (size_t)k * LM];
    int carry = 0;
    for (int j = 0; j < 4 * LM; ++j) {
      const int v = (int)((row[j >> 2] >> (8 * (j & 3))) & 255u) + carry;
      carry = v >= 128 ? 1 : 0;
      dig[(size_t)k * nd + j] = (int8_t)(v - 256 * carry);
    }
    dig[(size_t)k * nd + 4 * LM] = (int8_t)carry;
  }
  uint8_t* B = (uint8_t*)&c.buf[ob];
  for (int ct = 0; ct < nct; ++ct)
    for (int ks = 0; ks < nks; ++ks)
      for (int L = 0; L < 64; ++L)
        for (int b = 0; b < 16; ++b) {
          const int col = 32 * ct + (L & 31), idx = 32 * ks + 16 * (L >> 5) + b;
          const int k = idx >> 2, s = idx & 3, j = col - s;
          const int8_t e = (k < P && j >= 0 && j < nd) ? dig[(size_t)k * nd + j] : (int8_t)0;
          B[(((size_t)ct * nks + ks) * 64 + L) * 16 + b] = (uint8_t)e;
        }
  return c;
}

static HostTables built() {
  HostTables t;
  build(t, MAX_PRIMES);
  return t;
}

const HostTables& host_tables() {
  static const HostTables t = built();  // thread-safe one-time initialisation
  return t;
}

}  // namespace bires
