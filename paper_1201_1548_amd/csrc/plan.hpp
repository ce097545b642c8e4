// Job planning on the host: true degrees, degree bound (number of evaluation
// points) and Hadamard coefficient bound (number of primes).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace bires {

// Per-row statistics of a bivariate input (rows = powers of the eliminated
// variable): x-degree (-1 for a zero row), bit length bound of |c| (|c| < 2^bits),
// non-zero count and an upper bound of log2 of the row's 1-norm in 1/1024
// bits, interleaved per row as the device scan writes them.
constexpr int ROWSTAT_WORDS = 4;
struct RowStats {
  std::vector<int32_t> v;  // [rows][4]: deg, bits, cnt, norm
  int rows() const { return (int)(v.size() / ROWSTAT_WORDS); }
  int32_t deg(int j) const { return v[ROWSTAT_WORDS * j]; }
  int32_t bits(int j) const { return v[ROWSTAT_WORDS * j + 1]; }
  int32_t cnt(int j) const { return v[ROWSTAT_WORDS * j + 2]; }
  int32_t norm(int j) const { return v[ROWSTAT_WORDS * j + 3]; }  // ceil(1024 log2 sum |c|)
  void resize(int rows) { v.assign((size_t)ROWSTAT_WORDS * rows, 0); }
  void set(int j, int32_t d, int32_t b, int32_t c, int32_t n) {
    v[ROWSTAT_WORDS * j] = d;
    v[ROWSTAT_WORDS * j + 1] = b;
    v[ROWSTAT_WORDS * j + 2] = c;
    v[ROWSTAT_WORDS * j + 3] = n;
  }
};
// ceil(1024 log2 x) + margin for x > 0, the fixed-point logarithm of RowStats.
int32_t log2_fx_up(double x);

struct Plan {
  int m = -1, n = -1;       // degrees in y of f and g (-1: zero polynomial)
  int dxf = -1, dxg = -1;   // degrees in x
  int tf = -1, tg = -1;     // total degrees
  int D = 0;                // evaluation points = degree bound + 1
  int P = 0;                // primes
  double log2B = 0.0;       // log2 of the bound on |coefficients of R|
  int kind_special = 0;     // 0: compute; 1: R = 0; 2: R = 1
};

// Statistics of a limb rectangle in host memory.
RowStats scan_host(const uint32_t* limbs, int rows, int ld, int L);
// Statistics of the y-derivative computed from those of f (row j <- (j+1) row j+1).
RowStats derive_stats(const RowStats& f);
// Statistics of the x-derivative (row j <- d/dx row j; rows are powers of y).
RowStats derive_stats_x(const RowStats& f);
// Statistics that every input of the given extents satisfies (for *_bounds).
RowStats worst_stats(int rows, int ld, int L);

// log2 of the Hadamard bound of the Sylvester matrix (entries replaced by
// their 1-norms): (n/2) log2(sum_j N_j^2) + (m/2) log2(sum_j N'_j^2).
double hadamard_log2(const RowStats& f, int m, const RowStats& g, int n);

// Fill a plan; returns 0 or a BIRES_E* code.
int make_plan(const RowStats& f, const RowStats& g, Plan& out);

// Limbs needed for signed values of magnitude at most 2^log2B.
int limbs_for_log2(double log2B);

}  // namespace bires
