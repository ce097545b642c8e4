// Host-side tables: the primes and the mixed-radix constants (see tables.cpp).
#pragma once
#include <stdint.h>

#include <vector>

#include "modp.hpp"

namespace bires {

constexpr int MAX_PRIMES = 2048;
constexpr uint32_t PRIME_CEIL = 1431655765u;  // floor((2^32 - 1) / 3), odd; the table descends from here
constexpr int MAX_POINTS = 8192;  // evaluation points (degree bound + 1) per job
constexpr int MAX_GCD_DEGREE = 8000;

struct HostTables {
  int K = 0;
  std::vector<ModP> primes;     // K primes, descending from below PRIME_CEIL
  std::vector<double> log2p;    // lower bounds of log2 p_k
  std::vector<double> cumlog;   // cumlog[k] = sum_{i<k} log2p[i]
  std::vector<uint32_t> gm;     // [K][K] Montgomery (prod_{i<j} p_i mod p_k), j < k
  std::vector<uint32_t> cm;     // [K] Montgomery (prod_{i<k} p_i)^{-1} mod p_k
  std::vector<uint32_t> pm;     // [K][K] Montgomery (p_j mod p_k) at [k*K + j], j < k
  std::vector<uint32_t> pi;     // prod_{i<k} p_i, k+1 limbs at offset k(k+1)/2
};

ModP make_modp(uint32_t p);
// Mixed-radix tables (layouts as in HostTables) for an arbitrary list of primes.
void mrc_tables(const std::vector<ModP>& primes, std::vector<uint32_t>& gm, std::vector<uint32_t>& cm,
                std::vector<uint32_t>& pm, std::vector<uint32_t>& pi);
const HostTables& host_tables();

// Explicit CRT constants for the first P primes of the table, M = prod_{k<P} p_k:
// one buffer [w (P words) | M_k rows (P x LM words) | M (LM words)] with
// w[k] the Montgomery form of ((M / p_k) mod p_k)^{-1} mod p_k and the rows
// the little-endian limbs of M / p_k, zero-padded to LM = limbs of M.
struct CrtHost {
  int P = 0, LM = 0;
  std::vector<uint32_t> buf;
};
CrtHost crt_tables(int P);

}  // namespace bires
