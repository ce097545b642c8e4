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
// modulo M = prod p_k is exact once M > 2B (symmetric residues).  N_j comes
// from the row scan as an upper bound of log2 N_j in 1/1024 bits; all sums are
// done in log2 with a margin.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

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

int32_t log2_fx_up(double x) { return (int32_t)std::ceil((std::log2(x) + 1e-6) * 1024.0); }

// Upper bound of |c| as a double: the top 64 magnitude bits plus one unit of
// the next limb, raised by 2^-52 against the rounding of the conversion.
static double mag_upper(const uint32_t* c, int L) {
  const uint32_t inv = (c[L - 1] >> 31) ? 0xFFFFFFFFu : 0u;
  int t = L - 1;
  while (t > 0 && (c[t] ^ inv) == 0u) --t;
  const uint64_t top = t ? (((uint64_t)(c[t] ^ inv) << 32) | (c[t - 1] ^ inv)) : (uint64_t)(c[0] ^ inv);
  const double v = ((double)top + 1.0) * (1.0 + 0x1p-52);
  return t ? std::ldexp(v, 32 * (t - 1)) : v;
}

RowStats scan_host(const uint32_t* limbs, int rows, int ld, int L) {
  RowStats s;
  s.resize(rows);
  for (int j = 0; j < rows; ++j) {
    int deg = -1, bits = 0, cnt = 0;
    double norm = 0.0;
    for (int i = 0; i < ld; ++i) {
      bool nz;
      const uint32_t* c = limbs + ((size_t)j * ld + i) * L;
      const int b = bitlen_abs(c, L, &nz);
      if (nz) {
        deg = i;
        cnt++;
        bits = std::max(bits, b);
        norm += mag_upper(c, L);
      }
    }
    // the sum's rounding (at most ld 2^-53 relative) is covered by 2^-40
    s.set(j, deg, bits, cnt, cnt ? log2_fx_up(norm * (1.0 + 0x1p-40)) : 0);
  }
  return s;
}

RowStats derive_stats(const RowStats& f) {
  RowStats g;
  const int rows = f.rows() - 1;
  if (rows <= 0) return g;
  g.resize(rows);
  for (int j = 0; j < rows; ++j) {
    const int lj = 32 - __builtin_clz((uint32_t)(j + 1));  // (j+1) < 2^lj
    // row j of the derivative is (j+1) times row j+1: its 1-norm scales by j+1
    g.set(j, f.deg(j + 1), f.cnt(j + 1) ? f.bits(j + 1) + lj : 0, f.cnt(j + 1),
          f.cnt(j + 1) ? f.norm(j + 1) + log2_fx_up((double)(j + 1)) : 0);
  }
  return g;
}

RowStats derive_stats_x(const RowStats& f) {
  RowStats g;
  g.resize(f.rows());
  for (int j = 0; j < f.rows(); ++j) {
    const int d = f.deg(j);
    if (d < 1) continue;  // constant or zero row: its derivative is zero
    // i c_i with i <= d: |i c_i| < 2^(bits + ld) and the 1-norm grows by at most d
    const int ld = 32 - __builtin_clz((uint32_t)d);
    g.set(j, d - 1, f.bits(j) + ld, f.cnt(j), f.norm(j) + log2_fx_up((double)d));
  }
  return g;
}

RowStats worst_stats(int rows, int ld, int L) {
  RowStats s;
  s.resize(rows);
  for (int j = 0; j < rows; ++j) s.set(j, ld - 1, 32 * L, ld, log2_fx_up((double)ld) + 1024 * 32 * L);
  return s;
}

static int top_row(const RowStats& s) {
  for (int j = s.rows() - 1; j >= 0; --j)
    if (s.cnt(j) > 0) return j;
  return -1;
}

// 2^e for e <= 0 as a double (0 below the normal range).
static double pow2_nonpos(int e) {
  if (e < -1022) return 0.0;
  const uint64_t rep = (uint64_t)(e + 1023) << 52;
  double d;
  std::memcpy(&d, &rep, sizeof d);
  return d;
}

// 2^(-r / 1024) for r = 0..1023 (a function-local static: after the first
// call, a guard check instead of std::call_once's per-call cost).
struct FracPow2 {
  double t[1024];
  FracPow2() {
    for (int r = 0; r < 1024; ++r) t[r] = std::exp2(-r / 1024.0);
  }
};
static const double* frac_pow2_neg() {
  static const FracPow2 f;
  return f.t;
}

// log2 (sum_j N_j^2) with log2 N_j <= norm_j / 1024, rows 0..top: with
// d_j = 2 (emax - norm_j) >= 0 (1/1024 bits) each term is 2^(-d_j / 1024) =
// 2^(-(d_j >> 10)) 2^(-(d_j & 1023) / 1024), a power of two times a table
// entry (a term below 2^-1022 of the largest one is dropped, far inside the
// margin of hadamard_log2), so one log2 per call remains.
static double log2_sum_sq(const RowStats& s, int top) {
  const double* fr = frac_pow2_neg();
  int emax = INT32_MIN;
  for (int j = 0; j <= top; ++j)
    if (s.cnt(j)) emax = std::max(emax, (int)s.norm(j));
  if (emax == INT32_MIN) return -INFINITY;
  double acc[2] = {0.0, 0.0};
  for (int j = 0; j <= top; ++j)
    if (s.cnt(j)) {
      const int d = 2 * (emax - s.norm(j));
      acc[j & 1] += pow2_nonpos(-(d >> 10)) * fr[d & 1023];
    }
  return 2.0 * emax / 1024.0 + std::log2(acc[0] + acc[1]);
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
    pl.dxf = std::max(pl.dxf, f.deg(j));
    if (f.deg(j) >= 0) pl.tf = std::max(pl.tf, f.deg(j) + j);
  }
  for (int j = 0; j <= pl.n; ++j) {
    pl.dxg = std::max(pl.dxg, g.deg(j));
    if (g.deg(j) >= 0) pl.tg = std::max(pl.tg, g.deg(j) + j);
  }
  const long long b1 = (long long)pl.n * pl.dxf + (long long)pl.m * pl.dxg;
  const long long b2 = (long long)pl.n * pl.tf + (long long)pl.m * pl.tg - (long long)pl.m * pl.n;
  const long long bound = std::min(b1, b2);
  if (bound + 1 > (1 << 20)) return BIRES_ETOOBIG;
  pl.D = (int)bound + 1;
  pl.log2B = hadamard_log2(f, pl.m, g, pl.n);
  const HostTables& t = host_tables();
  // M > 2^1.001 B: the symmetric residue then sits at least 3e-4 M away from
  // +-M/2, which the explicit CRT's fp64 rounding relies on
  const double need = pl.log2B + 1.001;
  // smallest P with cumlog[P] > need (cumlog increases)
  const auto it = std::upper_bound(t.cumlog.begin() + 1, t.cumlog.end(), need);
  if (it == t.cumlog.end()) return BIRES_ETOOBIG;
  const int P = (int)(it - t.cumlog.begin());
  pl.P = P;
  return BIRES_OK;
}

int limbs_for_log2(double log2B) {
  // |v| <= 2^log2B needs floor(log2B) + 1 magnitude bits and one sign bit
  const double bits = std::floor(std::max(log2B, 0.0)) + 2.0;
  return (int)std::ceil(bits / 32.0);
}

}  // namespace bires
