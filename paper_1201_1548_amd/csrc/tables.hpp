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
// one buffer [w (P words) | M_k rows (P x LM words) | M (LM words) | pad to
// 4 words | B] with w[k] the Montgomery form of ((M / p_k) mod p_k)^{-1} mod
// p_k and the rows the little-endian limbs of M / p_k, zero-padded to LM =
// limbs of M.  B is the int8 operand of the matrix-core CRT: with e_k(j) the
// balanced base-256 digits of M / p_k (j = 0..4 LM), entry (k, s; c) =
// e_k(c - s) (zero outside that range) for contraction index 4 k + s and byte
// column c, stored in operand order: for column tile ct (32 columns) and
// contraction step ks (32 indices, 8 primes) one 1 KiB block whose lane
// L = x + 32 g holds column 32 ct + x, indices 32 ks + 16 g + 0..15.
// crt_operand_offset / crt_operand_tiles give B's word offset and its
// (column tiles, steps).
struct CrtHost {
  int P = 0, LM = 0;
  std::vector<uint32_t> buf;
};
size_t crt_operand_offset(int P, int LM);
void crt_operand_tiles(int P, int LM, int* nct, int* nks);
CrtHost crt_tables(int P);

}  // namespace bires
