// Job planning (host): degrees, the degree bound and the coefficient bound.
//
// Degree bound.  Row t < n of the Sylvester matrix holds f_{m-(c-t)} in column
// c, of x-degree at most min(dx_f, t_f - m + c - t); the g rows likewise.
// Summing over any permutation gives deg R <= n dx_f + m dx_g and
// deg R <= n t_f + m t_g - m n, and the second is at most t_f t_g (the m n of
// Section 2, "Resultants").  D = min of the two + 1 points determine R.
//
// Coefficient bound.  For |x| = 1 every entry f_j(x) has modulus at most the
// 1-norm N_j of f_j, so Hadamard's inequality bounds |R(x)| by
// (sum N_j^2)^{n/2} (sum N'_j^2)^{m/2}, and by Cauchy's estimate on the unit
// circle every coefficient of R is bounded by the same number B.  Reconstruction
// modulo M = prod p_k is exact once M > 2B (symmetric residues).  N_j is
// bounded by cnt_j 2^{bits_j}; all sums are done in log2 with a margin.
#include "plan.hpp"

#include <algorithm>
#include <cmath>

#include "../../include/bires.h"
#include "tables.hpp"

namespace bires {

static int bitlen_abs(const uint32_t* c, int L, bool* nonzero) {
  const uint32_t inv = (c[L - 1] >> 31) ? 0xFFFFFFFFu : 0u;
  bool nz = false;
  int b = 0;
  for (int l = L - 1; l >= 0; --l) {
    nz |= c[l] != 0u;
    const uint32_t x = c[l] ^ inv;
    if (b == 0 && x != 0u) b = 32 * l + (32 - __builtin_clz(x));
  }
  *nonzero = nz;
  return nz ? b + (inv ? 1 : 0) : 0;
}

RowStats scan_host(const uint32_t* limbs, int rows, int ld, int L) {
  RowStats s;
  s.deg.assign(rows, -1);
  s.bits.assign(rows, 0);
  s.cnt.assign(rows, 0);
  for (int j = 0; j < rows; ++j) {
    for (int i = 0; i < ld; ++i) {
      bool nz;
      const int b = bitlen_abs(limbs + ((size_t)j * ld + i) * L, L, &nz);
      if (nz) {
        s.deg[j] = i;
        s.cnt[j]++;
        s.bits[j] = std::max(s.bits[j], b);
      }
    }
  }
  return s;
}

RowStats derive_stats(const RowStats& f) {
  RowStats g;
  const int rows = (int)f.deg.size() - 1;
  if (rows <= 0) return g;
  g.deg.resize(rows);
  g.bits.resize(rows);
  g.cnt.resize(rows);
  for (int j = 0; j < rows; ++j) {
    g.deg[j] = f.deg[j + 1];
    g.cnt[j] = f.cnt[j + 1];
    const int lj = 32 - __builtin_clz((uint32_t)(j + 1));  // (j+1) < 2^lj
    g.bits[j] = f.cnt[j + 1] ? f.bits[j + 1] + lj : 0;
  }
  return g;
}

RowStats worst_stats(int rows, int ld, int L) {
  RowStats s;
  s.deg.assign(rows, ld - 1);
  s.bits.assign(rows, 32 * L);
  s.cnt.assign(rows, ld);
  return s;
}

static int top_row(const RowStats& s) {
  for (int j = (int)s.deg.size() - 1; j >= 0; --j)
    if (s.cnt[j] > 0) return j;
  return -1;
}

// log2 (sum_j N_j^2) with N_j <= cnt_j 2^bits_j, rows 0..top.
static double log2_sum_sq(const RowStats& s, int top) {
  double emax = -1e300;
  for (int j = 0; j <= top; ++j)
    if (s.cnt[j]) emax = std::max(emax, std::log2((double)s.cnt[j]) + s.bits[j]);
  double acc = 0.0;
  for (int j = 0; j <= top; ++j)
    if (s.cnt[j]) acc += std::exp2(2.0 * (std::log2((double)s.cnt[j]) + s.bits[j] - emax));
  return 2.0 * emax + std::log2(acc);
}

double hadamard_log2(const RowStats& f, int m, const RowStats& g, int n) {
  double v = 0.0;
  if (n > 0) v += 0.5 * n * log2_sum_sq(f, m);
  if (m > 0) v += 0.5 * m * log2_sum_sq(g, n);
  // margin against rounding in the log-domain sums (relative error << 1e-9)
  return v + 1e-9 * std::fabs(v) + 1e-6;
}

int make_plan(const RowStats& f, const RowStats& g, Plan& pl) {
  pl = Plan();
  pl.m = top_row(f);
  pl.n = top_row(g);
  if (pl.m < 0 || pl.n < 0) {
    pl.kind_special = 1;
    pl.D = 1;
    return BIRES_OK;
  }
  if (pl.m == 0 && pl.n == 0) {
    pl.kind_special = 2;
    pl.D = 1;
    return BIRES_OK;
  }
  if (pl.m > BIRES_MAX_YDEG || pl.n > BIRES_MAX_YDEG) return BIRES_ETOOBIG;
  for (int j = 0; j <= pl.m; ++j) {
    pl.dxf = std::max(pl.dxf, f.deg[j]);
    if (f.deg[j] >= 0) pl.tf = std::max(pl.tf, f.deg[j] + j);
  }
  for (int j = 0; j <= pl.n; ++j) {
    pl.dxg = std::max(pl.dxg, g.deg[j]);
    if (g.deg[j] >= 0) pl.tg = std::max(pl.tg, g.deg[j] + j);
  }
  const long long b1 = (long long)pl.n * pl.dxf + (long long)pl.m * pl.dxg;
  const long long b2 = (long long)pl.n * pl.tf + (long long)pl.m * pl.tg - (long long)pl.m * pl.n;
  const long long bound = std::min(b1, b2);
  if (bound + 1 > (1 << 20)) return BIRES_ETOOBIG;
  pl.D = (int)bound + 1;
  pl.log2B = hadamard_log2(f, pl.m, g, pl.n);
  const HostTables& t = host_tables();
  const double need = pl.log2B + 1.0;  // M > 2B
  int P = 1;
  while (P <= t.K && t.cumlog[P] <= need) ++P;
  if (P > t.K) return BIRES_ETOOBIG;
  pl.P = P;
  return BIRES_OK;
}

int limbs_for_log2(double log2B) {
  // |v| <= 2^log2B needs floor(log2B) + 1 magnitude bits and one sign bit
  const double bits = std::floor(std::max(log2B, 0.0)) + 2.0;
  return (int)std::ceil(bits / 32.0);
}

}  // namespace bires
