// HIP kernels (gfx950) of the multi-modular resultant: the steps (a)-(e) of
// Collins' scheme as summarised in Section 5.1 ("Computing resultants in
// Z[x,y]"), all on the device.
//
//   k_scan        per-row degree / bit-length statistics of an input (planning)
//   k_transpose   exchange x and y in a limb rectangle (res_x, disc_x)
//   k_reduce      (a) coefficients modulo each prime, Montgomery form
//   k_eval_elim   (b)+(c) evaluate at x = a and take the univariate resultant
//                 over F_p, one lane per (prime, point); k_eval_elim_rg24,
//                 _rg32 and _rg64 keep f's coefficient array in registers
//   k_schur       (c) the same elimination by the Schur algorithm on the
//                 displacement generators, one wave per (prime, point)
//   k_psc         principal subresultant coefficients mod p, one lane per point
//   k_interp      (d) interpolation per prime, nodes a = 0..D-1
//   k_interp_mfma (d) interpolation of a batch sharing the nodes, int8 matrix
//                 cores (value digit planes written by the evaluation
//                 kernels, V^{-1} by k_vinv)
//   k_invfact     table of 1/n! mod p (set-up)
//   k_crt_mfma    (e) explicit CRT straight to limbs, int8 matrix cores
//   k_mrc         (e) mixed-radix (Garner) digits per coefficient
//   k_limbs_sum / k_limbs_carry   (e) digits -> two's-complement limbs
//   k_fused       every stage after the reduction in one persistent launch
//   k_gcd_p / k_fiber_chain   gcd mod p, the N^- / N^+ degree chain
//
// Every kernel is batch-native: an array of per-job first-block indices maps
// each block to its job (find_job), so a single job is a batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "job.hpp"
#include "kernels.hpp"

namespace bires {

// Block -> job: starts[0..nj] are the first block of each job (starts[nj] =
// grid size); returns the largest j with starts[j] <= b (uniform, scalar).
// The job j of block b: starts[j] <= b < starts[j + 1] (nj + 1 prefix
// entries; jobs without blocks repeat an entry).  With the launch's block
// count `total`, the guess b nj / total is the answer whenever the jobs have
// equal block counts, and two independent loads confirm it; otherwise (or
// with total = 0) a binary search, whose dependent loads cost a round trip
// to L2 each.
__device__ __forceinline__ int find_job(const int* __restrict__ starts, int nj, int b, int total = 0) {
  if (total > 0) {
    const int g = min((int)(((unsigned long long)b * (unsigned)nj) / (unsigned)total), nj - 1);
    if (starts[g] <= b && b < starts[g + 1]) return g;
  }
  int lo = 0, hi = nj;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (starts[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Global-memory view of a pointer the host guarantees to be device memory:
// loads through it compile to global (not flat) loads, which do not share
// the LDS wait counter.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Lane of the calling thread in its wave.  The device functions that one wave
// runs index with it, so that a block of several waves (the persistent
// launch) can give each wave a task of its own.
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Synchronisation of the threads that run a device function together: the
// whole block, or (WAVE) one wave of it.  A wave's LDS accesses complete in
// order, so the wave needs no barrier; the fences keep the compiler from
// moving memory accesses across the point.
template <bool WAVE>
__device__ __forceinline__ void group_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// planning statistics: for each row j of a rectangle, the x-degree, the
// largest bit length of |c|, the number of non-zero coefficients and an upper
// bound of log2 of the row's 1-norm sum_i |c_ji| in 1/1024 bits (rounded up).
// |c| is bounded by its top 64 magnitude bits plus one unit of the next limb
// (double, raised by 2^-52), the sum by ld 2^-53 relative rounding (raised by
// 2^-40), the logarithm by 10^-6.

__device__ __forceinline__ double mag_upper(const uint32_t* c, int L) {
  const uint32_t inv = (c[L - 1] >> 31) ? 0xFFFFFFFFu : 0u;  // |c| <= (c xor sign) + 1
  int t = L - 1;
  while (t > 0 && (c[t] ^ inv) == 0u) --t;
  const uint64_t top = t ? (((uint64_t)(c[t] ^ inv) << 32) | (c[t - 1] ^ inv)) : (uint64_t)(c[0] ^ inv);
  const double v = ((double)top + 1.0) * (1.0 + 0x1p-52);
  return t ? ldexp(v, 32 * (t - 1)) : v;
}

__global__ void k_scan(const ScanTask* tasks, const int4* bmap) {
  int4 bm = bmap[blockIdx.x];
  const ScanTask& T = tasks[bm.x];
  int j = bm.y + threadIdx.x;
  if (j >= T.rows) return;
  int deg = -1, bits = 0, cnt = 0;
  double norm = 0.0;
  if (T.L == 1) {
    // one-limb coefficients: the row's words eight at a time (loads first),
    // each handled as below, in the same order
    const uint32_t* rowp = T.limbs + (size_t)j * T.ld;
    for (int i0 = 0; i0 < T.ld; i0 += 8) {
      uint32_t w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = rowp[min(i0 + u, T.ld - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 + u >= T.ld || w[u] == 0u) continue;
        const uint32_t inv = (w[u] >> 31) ? 0xFFFFFFFFu : 0u;
        const uint32_t x = w[u] ^ inv;
        const int b = (x ? 32 - __clz(x) : 0) + (inv ? 1 : 0);
        deg = i0 + u;
        ++cnt;
        bits = b > bits ? b : bits;
        norm += ((double)x + 1.0) * (1.0 + 0x1p-52);
      }
    }
    T.out[4 * j + 0] = deg;
    T.out[4 * j + 1] = bits;
    T.out[4 * j + 2] = cnt;
    T.out[4 * j + 3] = cnt ? (int32_t)ceil((log2(norm * (1.0 + 0x1p-40)) + 1e-6) * 1024.0) : 0;
    return;
  }
  for (int i = 0; i < T.ld; ++i) {
    const uint32_t* c = T.limbs + ((size_t)j * T.ld + i) * T.L;
    uint32_t top = c[T.L - 1];
    uint32_t inv = (top >> 31) ? 0xFFFFFFFFu : 0u;   // |c| <= (c xor sign) + 1
    int b = 0;
    bool nz = false;
    for (int l = T.L - 1; l >= 0; --l) {
      uint32_t w = c[l];
      nz |= (w != 0u);
      uint32_t x = w ^ inv;
      if (b == 0 && x != 0u) b = 32 * l + (32 - __clz(x));
    }
    if (nz) {
      deg = i;
      ++cnt;
      b += inv ? 1 : 0;
      bits = b > bits ? b : bits;
      norm += mag_upper(c, T.L);
    }
  }
  T.out[4 * j + 0] = deg;
  T.out[4 * j + 1] = bits;
  T.out[4 * j + 2] = cnt;
  T.out[4 * j + 3] = cnt ? (int32_t)ceil((log2(norm * (1.0 + 0x1p-40)) + 1e-6) * 1024.0) : 0;
}

// ---------------------------------------------------------------------------
// exchange the variables: dst[i][j] = src[j][i] (limb blocks of L words)

__global__ void k_transpose(const uint32_t* src, uint32_t* dst, int rows, int cols, int L) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t total = (size_t)rows * cols * L;
  if (idx >= total) return;
  int l = (int)(idx % L);
  size_t rc = idx / L;
  int i = (int)(rc % cols);
  int j = (int)(rc / cols);
  dst[((size_t)i * rows + j) * L + l] = src[idx];
}

// ---------------------------------------------------------------------------
// (a) reduction modulo the primes.  Each job has ceil(Tf/64) blocks for f
// then ceil(Tg/64) for g, 64 coefficients each; blockIdx.y selects a tile of
// KT primes.  A coefficient
// with limbs w_0..w_{L-1} (two's complement) has value sum w_l 2^{32l} - s 2^{32L};
// its Montgomery residue is built by Horner over the limbs with one two-product
// reduction per limb, then the sign term (R^L)_M is subtracted.

constexpr int KT = 16;

// Local block lb of a job (64 coefficients), primes [k0, k1).
__device__ void dev_reduce(const JobDev& J, int lb, int k0, int k1, TablesDev tab) {
  const int nbf = (J.Tf + 63) / 64;
  const bool isg = lb >= nbf;
  const int T = isg ? J.Tg : J.Tf;
  const int t = (isg ? lb - nbf : lb) * 64 + threadIdx.x;
  if (t >= T || k0 >= J.P) return;
  // residue t is coefficient (j, i) of its rectangle; i >= ld is row padding
  const int lp = isg ? J.lpg : J.lpf;
  const int ld = isg ? J.ldg : J.ldf;
  const int j = t / lp, i = t - j * lp;
  uint32_t* dst = (isg ? J.res_g : J.res_f) + t;
  k1 = min(J.P, k1);
  if (i >= ld) {
    for (int k = k0; k < k1; ++k) dst[(size_t)k * T] = 0u;
    return;
  }
  const uint32_t* src;
  int L;
  uint32_t mult = 0;  // 0: none; else the derivative factor (j+1 or i+1)
  if (!isg && J.kind == 2) {
    // x-derivative: coefficient (j, i) is (i+1) f_{j,i+1}; the last column is zero
    if (i + 1 >= ld) {
      for (int k = k0; k < k1; ++k) dst[(size_t)k * T] = 0u;
      return;
    }
    src = J.limbs_f + ((size_t)j * J.ldf + i + 1) * J.Lf;
    L = J.Lf;
    mult = (uint32_t)(i + 1);
  } else if (!isg) {
    src = J.limbs_f + ((size_t)j * J.ldf + i) * J.Lf;
    L = J.Lf;
  } else if (J.kind != 0) {
    src = J.limbs_f + ((size_t)(j + 1) * J.ldf + i) * J.Lf;  // coefficient (j+1, i) of f
    L = J.Lf;
    mult = (uint32_t)(j + 1);
  } else {
    src = J.limbs_g + ((size_t)j * J.ldg + i) * J.Lg;
    L = J.Lg;
  }
  if (L == 1) {
    // one limb w (the common case): w R mod p, less R mod p when w is
    // negative; w is loaded once, ahead of the stores
    // (the prime constants are loaded eight at a time ahead of their stores)
    const uint32_t w0 = src[0];
    const bool neg = (w0 >> 31) != 0u;
    for (int kb = k0; kb < k1; kb += 8) {
      ModP qs[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) qs[j] = tab.primes[min(kb + j, k1 - 1)];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (kb + j >= k1) break;
        const ModP& q = qs[j];
        uint32_t x = mmul(w0, q.r2, q);
        if (neg) x = msub(x, q.r2, q.p);
        if (mult) x = mmul(x, to_mont(mult, q), q);
        dst[(size_t)(kb + j) * T] = x;
      }
    }
    return;
  }
  const bool negv = (src[L - 1] >> 31) != 0u;
  for (int k = k0; k < k1; ++k) {
    const ModP q = tab.primes[k];
    uint32_t x = 0;
    for (int l = L - 1; l >= 0; --l) x = mdot2(x, q.r2, reduce32(src[l], q.p), q.r2, q);
    if (negv) x = msub(x, mpow(q.r2, (uint32_t)L, q), q.p);
    if (mult) x = mmul(x, to_mont(mult, q), q);
    dst[(size_t)k * T] = x;
  }
}

__global__ void k_reduce(const JobDev* jobs, const int* starts, int nj, TablesDev tab) {
  const int job = find_job(starts, nj, blockIdx.x, gridDim.x);
  dev_reduce(jobs[job], blockIdx.x - starts[job], blockIdx.y * KT, blockIdx.y * KT + KT, tab);
}

// ---------------------------------------------------------------------------
// (c) the univariate resultant over F_p of A = f(a, y) and B = g(a, y) with
// formal degrees m and n, i.e. the determinant of their (m+n) x (m+n)
// Sylvester matrix (Section 2) over F_p.  Coefficients live in LDS, one lane
// per instance: element t of a lane's array is at stride W.
//
// Formal degrees: if the leading coefficient of f(a, y) vanishes (actual
// degree a < m) the determinant equals (-1)^{n(m-a)} g_n^{m-a} res_{a,n}; if
// that of g vanishes, f_m^{n-b} res_{m,b}; if both vanish the first column of
// the Sylvester matrix is zero.
//
// With actual degrees a >= b >= 1 Euclid's rule res(A, B) =
// (-1)^{ab} lc(B)^{a-c} res(B, A mod B) (c = deg(A mod B)) is applied without
// inverses: each elimination A <- lc(B) A - lc(A) y^{a-b} B multiplies the
// remainder by lc(B), so after k eliminations the remainder is lc(B)^k (A mod B)
// and res(A, B) = (-1)^{ab} lc(B)^{a-c-kb} res(B, A_k); positive powers go to
// a numerator, negative ones to a denominator inverted once at the end.

__device__ __forceinline__ int wave_uniform(int x) {
  // 1 when every active lane holds the same value
  return __ballot(x != __builtin_amdgcn_readfirstlane(x)) == 0ull;
}

// The a - b + 1 eliminations of one Euclid step: A <- lc(B) A - A_top y^(a'-b) B
// for a' = a, a-1, ..., b.  Afterwards A holds lc(B)^(a-b+1) (A mod B) in
// its coefficients 0..b-1 (an elimination whose top coefficient is already
// zero only scales A, which keeps that identity).  With wave-uniform a and b
// every loop bound is a scalar.  A and B are disjoint.
//
// The usual step has a = b + 1: its two eliminations run as one pass.  The
// second one's multiplier is the first one's new top coefficient
// lc(B) A_{a-1} - A_a B_{b-1}, computed first; then each coefficient takes
// A_t <- lc(B) (lc(B) A_t - A_a B_{t-1}) - A'_{a-1} B_t
//      = lc(B)^2 A_t - lc(B) A_a B_{t-1} - A'_{a-1} B_t,
// a three-product sum with one reduction (3p < 2^32), and every A_t and B_t
// is read once.  In Montgomery form the two step constants are
// l2 = lc(B)^2 R^{-1} and l1 = -lc(B) A_a R^{-1}, so that
// redc(l2 A_t + l1 B_{t-1} + n2 B_t) equals the two nested reductions.
template <int W>
__device__ __forceinline__ void eliminate(uint32_t* __restrict__ A, const uint32_t* __restrict__ B, int a, int b,
                                          uint32_t lb, const ModP& q) {
  if (a == b + 1) {
    const uint32_t n1 = mneg_factor(A[a * W], q.p);
    const uint32_t n2 = mneg_factor(mdot2(lb, A[(a - 1) * W], n1, B[(b - 1) * W], q), q.p);
    const uint32_t l2 = mmul(lb, lb, q), l1 = mmul(lb, n1, q);
    uint32_t bp = B[0];
    A[0] = mdot2(l2, A[0], n2, bp, q);
    int t = 1;
    for (; t + 4 <= b; t += 4) {
      const uint32_t x0 = A[t * W], x1 = A[(t + 1) * W], x2 = A[(t + 2) * W], x3 = A[(t + 3) * W];
      const uint32_t y0 = B[t * W], y1 = B[(t + 1) * W], y2 = B[(t + 2) * W], y3 = B[(t + 3) * W];
      A[t * W] = mdot3(l2, x0, l1, bp, n2, y0, q);
      A[(t + 1) * W] = mdot3(l2, x1, l1, y0, n2, y1, q);
      A[(t + 2) * W] = mdot3(l2, x2, l1, y1, n2, y2, q);
      A[(t + 3) * W] = mdot3(l2, x3, l1, y2, n2, y3, q);
      bp = y3;
    }
    for (; t < b; ++t) {
      const uint32_t y = B[t * W];
      A[t * W] = mdot3(l2, A[t * W], l1, bp, n2, y, q);
      bp = y;
    }
    return;
  }
  for (; a >= b; --a) {
    const uint32_t nla = mneg_factor(A[a * W], q.p);
    const int s = a - b;
    for (int t = 0; t < s; ++t) A[t * W] = mmul(lb, A[t * W], q);
    int t = s;
    for (; t + 4 <= a; t += 4) {
      const uint32_t x0 = A[t * W], x1 = A[(t + 1) * W], x2 = A[(t + 2) * W], x3 = A[(t + 3) * W];
      const uint32_t y0 = B[(t - s) * W], y1 = B[(t - s + 1) * W], y2 = B[(t - s + 2) * W],
                     y3 = B[(t - s + 3) * W];
      A[t * W] = mdot2(lb, x0, nla, y0, q);
      A[(t + 1) * W] = mdot2(lb, x1, nla, y1, q);
      A[(t + 2) * W] = mdot2(lb, x2, nla, y2, q);
      A[(t + 3) * W] = mdot2(lb, x3, nla, y3, q);
    }
    for (; t < a; ++t) A[t * W] = mdot2(lb, A[t * W], nla, B[(t - s) * W], q);
  }
}

template <int W>
__device__ uint32_t uni_resultant(uint32_t* A, uint32_t* B, int m, int n, const ModP& q) {
  if (m == 0 && n == 0) return q.one;  // empty determinant
  int a = m;
  while (a >= 0 && A[a * W] == 0u) --a;
  int b = n;
  while (b >= 0 && B[b * W] == 0u) --b;
  if (a < 0) return n == 0 ? mpow(B[0], (uint32_t)m, q) : 0u;
  if (b < 0) return m == 0 ? mpow(A[0], (uint32_t)n, q) : 0u;
  if (a < m && b < n) return 0u;
  uint32_t num = q.one, den = q.one;
  bool neg = false;
  if (a < m) {
    num = mpow(B[n * W], (uint32_t)(m - a), q);
    neg = ((n * (m - a)) & 1) != 0;
  } else if (b < n) {
    num = mpow(A[m * W], (uint32_t)(n - b), q);
  }
  if (a < b) {
    uint32_t* T = A; A = B; B = T;
    int t = a; a = b; b = t;
    neg ^= ((a * b) & 1) != 0;
  }
  // Step i (B of degree b_i, lc l_i, remainder degree c_i) contributes
  // l_i^(e_i), e_i = a - c_i - (a - b_i + 1) b_i.  Split e_i = -2(b_i - 1) + d_i:
  // prod_i l_i^(2(b_i - 1)) = prod_t P_t over t = 1..b_0-1 with P the prefix
  // products of l_i^2 and t in [max(c_i, 1), b_i - 1] taking P_i, so a generic
  // step (c_i = b_i - 1, d_i = 0) costs three products and no power.
  uint32_t pfx = q.one;
  // Fast path: while every lane has the same (a, b) and every remainder has
  // degree exactly b - 1, a and b stay scalar and a step's bookkeeping is
  // x = 1 (or 0 at b = 1) and d = (1 - b)(a - b - 1), both uniform.  The
  // first step whose remainder is shorter on some lane finishes in the
  // general loop below without eliminating again.
  bool eliminated = false;
  uint32_t lb_done = 0;
  if (wave_uniform(a) && wave_uniform(b)) {
    int as = __builtin_amdgcn_readfirstlane(a), bs = __builtin_amdgcn_readfirstlane(b);
    while (bs > 0) {
      const uint32_t lb = B[bs * W];
      eliminate<W>(A, B, as, bs, lb, q);
      if (__ballot(A[(bs - 1) * W] == 0u) != 0ull) {
        eliminated = true;
        lb_done = lb;
        break;
      }
      neg ^= ((as * bs) & 1) != 0;
      pfx = mmul(pfx, mmul(lb, lb, q), q);
      if (bs > 1) den = mmul(den, pfx, q);
      const int d = (1 - bs) * (as - bs - 1);
      if (d > 0) num = mmul(num, mpow(lb, (uint32_t)d, q), q);
      else if (d < 0) den = mmul(den, mpow(lb, (uint32_t)(-d), q), q);
      uint32_t* T = A;
      A = B;
      B = T;
      as = bs;
      bs = bs - 1;
    }
    a = as;
    b = bs;
  }
  while (b > 0) {
    const uint32_t lb = eliminated ? lb_done : B[b * W];
    if (eliminated)
      eliminated = false;
    else if (wave_uniform(a) && wave_uniform(b))
      eliminate<W>(A, B, __builtin_amdgcn_readfirstlane(a), __builtin_amdgcn_readfirstlane(b), lb, q);
    else
      eliminate<W>(A, B, a, b, lb, q);
    int c = b - 1;
    while (c >= 0 && A[c * W] == 0u) --c;
    if (c < 0) return 0u;
    neg ^= ((a * b) & 1) != 0;
    pfx = mmul(pfx, mmul(lb, lb, q), q);
    const int x = b - (c > 1 ? c : 1);
    if (x == 1) den = mmul(den, pfx, q);
    else if (x > 1) den = mmul(den, mpow(pfx, (uint32_t)x, q), q);
    const int d = a - c - (a - b + 1) * b + 2 * (b - 1);
    if (d > 0) num = mmul(num, mpow(lb, (uint32_t)d, q), q);
    else if (d < 0) den = mmul(den, mpow(lb, (uint32_t)(-d), q), q);
    uint32_t* T = A; A = B; B = T;
    a = b;
    b = c;
  }
  num = mmul(num, mpow(B[0], (uint32_t)a, q), q);
  uint32_t r = (den == q.one) ? num : mmul(num, minv(den, q), q);
  return neg ? mneg(r, q.p) : r;
}

// a b + c with 32-bit a, b (one v_mad_u64_u32).  Inline assembly keeps a as a
// single 32-bit register where the compiler would keep a zero-extended pair.
// SB: b is wave-uniform and held in a scalar register (the residues read
// through the scalar cache).
template <bool SB = false>
__device__ __forceinline__ uint64_t mad_u64_u32(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t d;
  uint64_t carry;
  if constexpr (SB)
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(a), "s"(b), "v"(c));
  else
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(a), "v"(b), "v"(c));
  return d;
}

// Exact sums of products of residues in 96 bits: 64-bit partial sums (up to
// eight products of residues, below 8 p^2 < 2^64) added with a carry word.
struct Acc96 {
  uint64_t lo = 0;
  uint32_t hi = 0;
  __device__ void add(uint64_t s) {
    lo += s;
    hi += lo < s ? 1u : 0u;
  }
};

// (b) evaluation at x = a.  With Montgomery residues c_M of a row and the
// Montgomery powers (a^i)_M, S = sum_i c_M (a^i)_M is f_j(a) R^2 mod p; S is
// summed exactly and one reduction turns it into f_j(a) R.  The powers live
// in registers, so a coefficient costs one 32x32->64 multiply-add instead of
// the three of a Montgomery Horner step, and the products do not form a
// dependency chain.  Rows longer than EV_PW coefficients are cut into chunks
// of EV_PW, combined by Horner's rule in a^EV_PW.
constexpr int EV_PW = 24;

// S R^{-1} mod p for S = hi 2^64 + lo with hi < 2^32 - 4 (here hi <= 2):
// REDC(lo_lo + hi R^2) = lo_lo R^{-1} + hi R, and lo_hi R R^{-1} = lo_hi.
// The REDC argument is below p 2^32, so its result is below 2p.
__device__ __forceinline__ uint32_t fold96(const Acc96& S, const ModP& q) {
  const uint64_t t = (uint64_t)S.hi * q.r2 + (uint32_t)S.lo;
  return madd(redc(t, q.p, q.pinv), reduce32((uint32_t)(S.lo >> 32), q.p), q.p);
}

// Byte offset of element (row, idx) of a digit plane of the matrix-core
// interpolation with Kp = padded contraction length, in operand order: 1 KiB
// blocks per (32-row tile, 32-wide step), lane l of an operand holding row
// l % 32 and contraction indices 16 (l / 32) + 0..15.
__device__ __forceinline__ size_t im_off(int row, int idx, int Kp) {
  const int rt = row >> 5, r = row & 31, ks = idx >> 5, g = (idx >> 4) & 1, b = idx & 15;
  return ((((size_t)rt * (Kp >> 5) + ks) * 64) + r + 32 * g) * 16 + b;
}

// The four balanced base-256 digits of the symmetric representative v of
// x mod p, packed little-endian into one word.  Adding 128 at each of the
// three low digit positions makes those digits d_s + 128 in [0, 255] (plain
// base 256), with the top digit (|d_3| <= 64) left in the top byte; flipping
// bit 7 of the three low bytes subtracts the 128 again in int8 terms.
__device__ __forceinline__ uint32_t digits4(uint32_t x, uint32_t p) {
  const uint32_t v = x > (p >> 1) ? x - p : x;
  return (v + 0x808080u) ^ 0x808080u;
}

// The value v = R(a) mod p_k (plain residue) of point a of job J: into vals,
// or for a job of the matrix-core interpolation group straight into the
// group's four digit planes of prime k (column ycol), which the
// interpolation reads as its right operand.  Those planes are not cleared:
// columns past the group only reach output columns that are not written,
// and points in [D, Dp) meet zero entries of the inverse Vandermonde planes.
// (A call, not inlined: the register allocation of the evaluation kernels'
// loops stays that of a single store.)
__device__ __noinline__ void put_planes(int8_t* yp, int ycol, int ynp, int ydp, int k, int a, uint32_t v, uint32_t p) {
  const size_t plane = (size_t)ynp * ydp;
  int8_t* base = yp + (size_t)k * 4 * plane + im_off(ycol, a, ydp);
  const uint32_t d = digits4(v, p);
#pragma unroll
  for (int s = 0; s < 4; ++s) base[s * plane] = (int8_t)(d >> (8 * s));
}

__device__ __forceinline__ void put_value(const JobDev& J, int k, int a, uint32_t v, uint32_t p) {
  if (J.yp)
    put_planes(J.yp, J.ycol, J.ynp, J.ydp, k, a, v, p);
  else
    J.vals[(size_t)k * J.D + a] = v;
}

// Read-only data with wave-uniform addresses, read through the scalar cache.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const uint32_t cu32;
typedef __attribute__((address_space(4))) const u32x4 cu4;
typedef __attribute__((address_space(4))) const int32_t ci32;

// Value of the row c[0..d] (zero-padded to a multiple of 4, 16-byte aligned)
// at the point whose powers are pw (NPW of them, a multiple of 8); apw =
// (a^NPW)_M.  d is wave-uniform.  With C = cu32 the coefficients come in by
// scalar loads and feed the products as scalar operands (the data must not
// change during the launch); with C = const uint32_t they are ordinary loads.
// A chunk's NPW words are loaded at once, which can read up to NPW - 4 words
// past the end of a short row: the residue buffers are followed by at least
// that much workspace.  Eight products of residues stay below 8 p^2 < 2^64
// (p < 2^32 / 3), so each 64-bit partial sum takes eight.
template <class C, class C4, int NPW>
__device__ __forceinline__ uint32_t eval_row(C* c, int d, const uint32_t (&pw)[NPW], uint32_t apw, const ModP& q) {
  static_assert(NPW % 8 == 0, "powers come in groups of eight");
  if (d < 0) return 0u;
  const int top = d / NPW;
  uint32_t acc = 0u;
  for (int ch = top; ch >= 0; --ch) {
    C4* cc = (C4*)(c + ch * NPW);
    const int ng = (min(NPW, d + 1 - ch * NPW) + 3) >> 2;
    u32x4 v[NPW / 4];
#pragma unroll
    for (int g = 0; g < NPW / 4; ++g) v[g] = cc[g];
    // The products are v_mad_u64_u32 with the 32-bit power as an operand.
    // Written in C, (uint64_t) pw[i] * c lets the compiler hoist the
    // zero-extended powers out of the row loop as 64-bit register pairs,
    // which doubles their register count.
    Acc96 S;
#pragma unroll
    for (int h = 0; h < NPW / 8; ++h) {
      if (2 * h < ng) {
        constexpr bool SB = std::is_same<C, cu32>::value;
        const u32x4 x = v[2 * h];
        uint64_t t = (uint64_t)x.x * pw[8 * h];
        t = mad_u64_u32<SB>(pw[8 * h + 1], x.y, t);
        t = mad_u64_u32<SB>(pw[8 * h + 2], x.z, t);
        t = mad_u64_u32<SB>(pw[8 * h + 3], x.w, t);
        if (2 * h + 1 < ng) {
          const u32x4 y = v[2 * h + 1];
          t = mad_u64_u32<SB>(pw[8 * h + 4], y.x, t);
          t = mad_u64_u32<SB>(pw[8 * h + 5], y.y, t);
          t = mad_u64_u32<SB>(pw[8 * h + 6], y.z, t);
          t = mad_u64_u32<SB>(pw[8 * h + 7], y.w, t);
        }
        S.add(t);
      }
    }
    const uint32_t r = fold96(S, q);
    acc = ch == top ? r : madd(mmul(acc, apw, q), r, q.p);
  }
  return acc;
}

// (b)+(c): each job has P * ceil(D/W) blocks, prime-major; one lane per
// point a.  The prime's residues (rows at the padded strides lpf, lpg) and
// the row degrees are read with wave-uniform addresses; LDS holds only each
// lane's coefficient arrays, so more blocks fit on a CU.  SC: through the
// scalar cache, which is valid when the residues were written by an earlier
// launch (the staged schedule); the persistent fused launch, which writes
// them itself, uses ordinary loads.
// f(a, y) and g(a, y) modulo p_k (Montgomery form) at the point a = pt into
// the lane arrays A[j W], B[j W] (ascending powers of y).
template <int W, bool SC>
__device__ __forceinline__ void eval_pair(const JobDev& J, int k, int pt, const ModP& q, uint32_t* A, uint32_t* B) {
  typedef typename std::conditional<SC, cu32, const uint32_t>::type RW;
  typedef typename std::conditional<SC, cu4, const u32x4>::type RW4;
  typedef typename std::conditional<SC, ci32, const int32_t>::type RI;
  const int m = J.m, n = J.n;
  const int lpf = J.lpf, lpg = J.lpg;
  RW* Rf = (RW*)(J.res_f + (size_t)k * J.Tf);
  RW* Rg = (RW*)(J.res_g + (size_t)k * J.Tg);
  RI* RDf = (RI*)J.rowdeg_f;
  RI* RDg = (RI*)J.rowdeg_g;
  const uint32_t aM = to_mont((uint32_t)pt, q);
  const int dmax = max(J.ldf, J.kind ? J.ldf : J.ldg) - 1;
  uint32_t pw[EV_PW];
  pw[0] = q.one;
#pragma unroll
  for (int i = 1; i < EV_PW; ++i) pw[i] = i <= dmax ? mmul(pw[i - 1], aM, q) : 0u;
  const uint32_t apw = dmax >= EV_PW ? mmul(pw[EV_PW - 1], aM, q) : 0u;
  for (int j = 0; j <= m; ++j)
    A[j * W] = eval_row<RW, RW4>(Rf + j * lpf, __builtin_amdgcn_readfirstlane(RDf[j]), pw, apw, q);
  for (int j = 0; j <= n; ++j)
    B[j * W] = eval_row<RW, RW4>(Rg + j * lpg, __builtin_amdgcn_readfirstlane(RDg[j]), pw, apw, q);
}

template <int W, bool SC>
__device__ __forceinline__ void dev_eval_elim(const JobDev& J, int lb, TablesDev tab, uint32_t* lds) {
  const int nbpp = (J.D + W - 1) / W;
  const int k = lb / nbpp;
  const int a0 = (lb - k * nbpp) * W;
  const int m = J.m, n = J.n;
  uint32_t* A = lds + lane_id();
  uint32_t* B = A + (m + 1) * W;
  const int pt = a0 + lane_id();
  if (pt >= J.D) return;
  const ModP q = tab.primes[k];
  eval_pair<W, SC>(J, k, pt, q, A, B);
  const uint32_t r = uni_resultant<W>(A, B, m, n, q);
  put_value(J, k, pt, from_mont(r, q), q.p);
}

// Workgroups are dispatched to the 8 XCDs round-robin in blockIdx order, and
// each XCD has its own L2.  This bijection of [0, nb) gives XCD x the
// contiguous logical range [x q + min(x, r), ...) of q + (x < r) blocks
// (q = nb / 8, r = nb % 8), so the blocks of one (job, prime), which share
// that prime's residues, run on one XCD and share its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

template <int W>
__global__ __launch_bounds__(W) void k_eval_elim(const JobDev* jobs, const int* starts, int nj, TablesDev tab) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int job = find_job(starts, nj, b, gridDim.x);
  dev_eval_elim<W, true>(jobs[job], b - starts[job], tab, lds);
}

// ---------------------------------------------------------------------------
// (b)+(c) with one coefficient array in registers.
//
// The Euclid arrays above take (m + n + 2) words of LDS per lane, and that
// LDS, not the register file, limits the blocks resident on a CU.  Here the
// arrays are stored top-aligned: index k holds the coefficient of y^(deg - k),
// so the leading coefficient is always at index 0 and an elimination
//   A <- lc(B) A - lc(A) y^(a'-b) B
// becomes A[j] <- lc(B) A[j+1] - A[0] B[j+1] (j < b), lc(B) A[j+1] (b <= j < a')
// whatever the degree gap, and the fused double step of a normal remainder
// sequence (a = b + 1) becomes
//   A[k] <- l2 A[k+2] + l1 B[k+2] + n2 B[k+1]   (k < b - 1; the last one has
//   no B[k+2] term),
// with the constants of eliminate().  Both read index j+1 or k+2 before
// writing index j or k, so they run in place in ascending order.  Every index
// is a compile-time constant once the loops over the capacity C are unrolled
// (the degrees are wave-uniform, so the guards are scalar branches), which
// lets f's array X live in registers; g's array L stays in LDS at stride 64.
// The two roles alternate every Euclid step.
//
// A wave runs only the uniform normal case: non-zero leading coefficients at
// its points, then remainders of degree exactly b - 1.  At the first
// exception (probability about one in 2^25 per step and point for
// generic inputs) the block gives up, appends its index to a queue, and a
// second launch recomputes the queued blocks with dev_eval_elim.

#define RG_A(k) (AREG ? X[k] : L[(k) * 64])
#define RG_B(k) (AREG ? L[(k) * 64] : X[k])
#define RG_SET_A(k, v)          \
  do {                          \
    const uint32_t v_ = (v);    \
    if (AREG)                   \
      X[k] = v_;                \
    else                        \
      L[(k) * 64] = v_;         \
  } while (0)

// One elimination of A (degree ap) by B (degree bs, leading coefficient lb).
template <int C, bool AREG>
__device__ __forceinline__ void rg_elim(uint32_t (&X)[C], uint32_t* __restrict__ L, int bs, int ap, uint32_t lb,
                                        const ModP& q) {
  const uint32_t nla = mneg_factor(RG_A(0), q.p);
#pragma unroll
  for (int j0 = 0; j0 < C - 1; j0 += 4) {
    if (j0 + 4 < C && j0 + 4 <= bs) {
      uint32_t x[4], y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = RG_A(j0 + 1 + i);
        y[i] = RG_B(j0 + 1 + i);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) RG_SET_A(j0 + i, mdot2(lb, x[i], nla, y[i], q));
    } else if (j0 < ap) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = j0 + i;
        if (j < C - 1) {
          if (j < bs)
            RG_SET_A(j, mdot2(lb, RG_A(j + 1), nla, RG_B(j + 1), q));
          else if (j < ap)
            RG_SET_A(j, mmul(lb, RG_A(j + 1), q));
        }
      }
    }
  }
}

// The two eliminations of a normal step (A of degree bs + 1) as one pass.
template <int C, bool AREG>
__device__ __forceinline__ void rg_fused(uint32_t (&X)[C], uint32_t* __restrict__ L, int bs, uint32_t lb,
                                         const ModP& q) {
  const uint32_t n1 = mneg_factor(RG_A(0), q.p);
  const uint32_t n2 = mneg_factor(mdot2(lb, RG_A(1), n1, RG_B(1), q), q.p);
  const uint32_t l2 = mmul(lb, lb, q), l1 = mmul(lb, n1, q);
#pragma unroll
  for (int k0 = 0; k0 < C - 2; k0 += 4) {
    if (k0 + 5 < C && k0 + 4 < bs) {
      uint32_t x[4], y[5];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = RG_A(k0 + 2 + i);
#pragma unroll
      for (int i = 0; i < 5; ++i) y[i] = RG_B(k0 + 1 + i);
#pragma unroll
      for (int i = 0; i < 4; ++i) RG_SET_A(k0 + i, mdot3(l2, x[i], l1, y[i + 1], n2, y[i], q));
    } else if (k0 < bs) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + i;
        if (k < C - 2) {
          if (k < bs - 1)
            RG_SET_A(k, mdot3(l2, RG_A(k + 2), l1, RG_B(k + 2), n2, RG_B(k + 1), q));
          else if (k == bs - 1)
            RG_SET_A(k, mdot2(l2, RG_A(k + 2), n2, RG_B(k + 1), q));
        }
      }
    }
  }
}

// The eliminations of one Euclid step of the uniform case; returns lc(B) and
// leaves in *short_rem whether some lane's remainder has degree below b - 1.
template <int C, bool AREG>
__device__ __forceinline__ uint32_t rg_step(uint32_t (&X)[C], uint32_t* __restrict__ L, int as, int bs,
                                            bool* short_rem, const ModP& q) {
  const uint32_t lb = RG_B(0);
  if (as == bs + 1)
    rg_fused<C, AREG>(X, L, bs, lb, q);
  else
    for (int ap = as; ap >= bs; --ap) rg_elim<C, AREG>(X, L, bs, ap, lb, q);
  *short_rem = __ballot(RG_A(0) == 0u) != 0ull;
  return lb;
}

// The fused step of a normal sequence with the degree bs = B known at
// compile time: straight-line code, no guards.  Returns l2 = lc(B)^2 R^{-1}
// and whether every lane's remainder keeps degree B - 1.
struct RgStep {
  uint32_t l2;
  bool ok;
};

template <int C, int B, bool AREG>
__device__ __forceinline__ RgStep rg_fstep(uint32_t (&X)[C], uint32_t* __restrict__ L, const ModP& q) {
  static_assert(B >= 1 && B + 1 < C, "A of degree B + 1 must fit");
  // keep the scheduler from hoisting later steps' loads (register pressure)
  __builtin_amdgcn_sched_barrier(0);
  const uint32_t lb = RG_B(0);
  const uint32_t n1 = mneg_factor(RG_A(0), q.p);
  const uint32_t n2 = mneg_factor(mdot2(lb, RG_A(1), n1, RG_B(1), q), q.p);
  const uint32_t l2 = mmul(lb, lb, q), l1 = mmul(lb, n1, q);
#pragma unroll
  for (int k = 0; k < B - 1; ++k) RG_SET_A(k, mdot3(l2, RG_A(k + 2), l1, RG_B(k + 2), n2, RG_B(k + 1), q));
  RG_SET_A(B - 1, mdot2(l2, RG_A(B + 1), n2, RG_B(B), q));
  return RgStep{l2, __ballot(RG_A(0) == 0u) == 0ull};
}

#undef RG_A
#undef RG_B
#undef RG_SET_A

// One step of the unrolled chain of normal steps from the current degree bs
// down to 1: step BV runs when bs >= BV.  (A switch into a fall-through
// sequence would be shorter to issue but makes every case a merge point of
// the register array, which the register allocator answers with copies.)
// In the chain of parity EVEN, A is the register array at even BV.  A step
// of a normal sequence (a = b + 1) has bookkeeping d = 0 and an even a b.
#define RG_CHAIN_STEP(BV, EVEN)                                                  \
  if constexpr (BV + 1 < C) {                                                    \
    if (bs >= BV) {                                                              \
      const RgStep o_ = rg_fstep<C, BV, ((((BV) & 1) == 0) == (EVEN))>(X, L, q); \
      if (!o_.ok) return false;                                                  \
      pfx = mmul(pfx, o_.l2, q);                                                 \
      if (BV > 1) den = mmul(den, pfx, q);                                       \
    }                                                                            \
  }
#define RG_CHAIN(EVEN)                                                                                         \
  RG_CHAIN_STEP(30, EVEN) RG_CHAIN_STEP(29, EVEN) RG_CHAIN_STEP(28, EVEN) RG_CHAIN_STEP(27, EVEN)              \
  RG_CHAIN_STEP(26, EVEN) RG_CHAIN_STEP(25, EVEN) RG_CHAIN_STEP(24, EVEN) RG_CHAIN_STEP(23, EVEN)              \
  RG_CHAIN_STEP(22, EVEN) RG_CHAIN_STEP(21, EVEN) RG_CHAIN_STEP(20, EVEN) RG_CHAIN_STEP(19, EVEN)              \
  RG_CHAIN_STEP(18, EVEN) RG_CHAIN_STEP(17, EVEN) RG_CHAIN_STEP(16, EVEN) RG_CHAIN_STEP(15, EVEN)              \
  RG_CHAIN_STEP(14, EVEN) RG_CHAIN_STEP(13, EVEN) RG_CHAIN_STEP(12, EVEN) RG_CHAIN_STEP(11, EVEN)              \
  RG_CHAIN_STEP(10, EVEN) RG_CHAIN_STEP(9, EVEN) RG_CHAIN_STEP(8, EVEN) RG_CHAIN_STEP(7, EVEN)                 \
  RG_CHAIN_STEP(6, EVEN) RG_CHAIN_STEP(5, EVEN) RG_CHAIN_STEP(4, EVEN) RG_CHAIN_STEP(3, EVEN)                  \
  RG_CHAIN_STEP(2, EVEN) RG_CHAIN_STEP(1, EVEN)

// Powers held in registers by the register-array kernel (fewer than EV_PW, to
// leave room for X; longer rows take one more Horner chunk).
constexpr int RG_PW = 24;

// Returns false (on every active lane) when the block must be recomputed by
// dev_eval_elim.  Needs 1 <= m, n and max(m, n) < C; LDS: (max(m, n) + 1)
// words per lane.
template <int C>
__device__ __forceinline__ bool dev_eval_elim_rg(const JobDev& J, int lb, TablesDev tab, uint32_t* lds) {
  const int nbpp = (J.D + 63) / 64;
  const int k = lb / nbpp;
  const int a0 = (lb - k * nbpp) * 64;
  const int m = J.m, n = J.n;
  const int lpf = J.lpf, lpg = J.lpg;
  cu32* Rf = (cu32*)(J.res_f + (size_t)k * J.Tf);
  cu32* Rg = (cu32*)(J.res_g + (size_t)k * J.Tg);
  ci32* RDf = (ci32*)J.rowdeg_f;
  ci32* RDg = (ci32*)J.rowdeg_g;
  uint32_t* L = lds + lane_id();
  const int pt = a0 + lane_id();
  if (pt >= J.D) return true;
  const ModP q = tab.primes[k];
  const uint32_t aM = to_mont((uint32_t)pt, q);
  const int dmax = max(J.ldf, J.kind ? J.ldf : J.ldg) - 1;
  uint32_t pw[RG_PW];
  pw[0] = q.one;
#pragma unroll
  for (int i = 1; i < RG_PW; ++i) pw[i] = i <= dmax ? mmul(pw[i - 1], aM, q) : 0u;
  const uint32_t apw = dmax >= RG_PW ? mmul(pw[RG_PW - 1], aM, q) : 0u;
  // f's values go through L (a loop with runtime trip counts cannot fill a
  // register array), then g's take their place
  for (int t = 0; t <= m; ++t)
    L[t * 64] = eval_row<cu32, cu4>(Rf + (m - t) * lpf, __builtin_amdgcn_readfirstlane(RDf[m - t]), pw, apw, q);
  uint32_t X[C];
#pragma unroll
  for (int t = 0; t < C; ++t) X[t] = t <= m ? L[t * 64] : 0u;
  for (int t = 0; t <= n; ++t)
    L[t * 64] = eval_row<cu32, cu4>(Rg + (n - t) * lpg, __builtin_amdgcn_readfirstlane(RDg[n - t]), pw, apw, q);
  if (__ballot(X[0] == 0u || L[0] == 0u) != 0ull) return false;
  uint32_t num = q.one, den = q.one, pfx = q.one;
  bool neg = false, areg = true;
  int as = m, bs = n;
  if (m < n) {
    areg = false;
    as = n;
    bs = m;
    neg = ((m * n) & 1) != 0;
  }
  if (as != bs + 1) {
    // the first step of a pair with a != b + 1 (only the first can be)
    bool short_rem;
    const uint32_t lb = areg ? rg_step<C, true>(X, L, as, bs, &short_rem, q)
                             : rg_step<C, false>(X, L, as, bs, &short_rem, q);
    if (short_rem) return false;
    // bookkeeping of uni_resultant's fast path (remainder degree bs - 1)
    neg ^= ((as * bs) & 1) != 0;
    pfx = mmul(pfx, mmul(lb, lb, q), q);
    if (bs > 1) den = mmul(den, pfx, q);
    const int d = (1 - bs) * (as - bs - 1);
    if (d > 0)
      num = mmul(num, mpow(lb, (uint32_t)d, q), q);
    else if (d < 0)
      den = mmul(den, mpow(lb, (uint32_t)(-d), q), q);
    areg = !areg;
    as = bs;
    bs -= 1;
  }
  if constexpr (C > 32) {
    // steps above the unrolled chain's reach (B > 30): the fused step with
    // wave-uniform guards (a normal step: d = 0 and a b even, so only pfx
    // and den change)
    while (bs > 30) {
      bool short_rem;
      const uint32_t lb = areg ? rg_step<C, true>(X, L, as, bs, &short_rem, q)
                               : rg_step<C, false>(X, L, as, bs, &short_rem, q);
      if (short_rem) return false;
      pfx = mmul(pfx, mmul(lb, lb, q), q);
      den = mmul(den, pfx, q);
      areg = !areg;
      as = bs;
      bs -= 1;
    }
  }
  uint32_t last;
  if (bs == 0) {
    // the constant remainder is in the array that does not hold A
    last = mpow(areg ? L[0] : X[0], (uint32_t)as, q);
  } else if (areg == ((bs & 1) == 0)) {
    RG_CHAIN(true)
    last = L[0];  // the last step (B = 1, odd) eliminated into L
  } else {
    RG_CHAIN(false)
    last = X[0];
  }
  num = mmul(num, last, q);
  uint32_t r = den == q.one ? num : mmul(num, minv(den, q), q);
  if (neg) r = mneg(r, q.p);
  put_value(J, k, pt, from_mont(r, q), q.p);
  return true;
}

template <int C>
__device__ __forceinline__ void eval_elim_rg_block(const JobDev* jobs, const int* starts, int nj, TablesDev tab,
                                                   int* fb_count, int* fb_queue, uint32_t* lds) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int job = find_job(starts, nj, b, gridDim.x);
  const bool ok = dev_eval_elim_rg<C>(jobs[job], b - starts[job], tab, lds);
  if (__ballot(!ok) != 0ull && threadIdx.x == 0) fb_queue[atomicAdd(fb_count, 1)] = b;
}

// C = 24 is held to RG24_WAVES waves per SIMD (76 VGPRs, no spills); C = 32
// runs at RG32_WAVES (102 VGPRs; at 5 waves it spills inside the chain).
#ifndef RG24_WAVES
#define RG24_WAVES 6
#endif
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RG24_WAVES, 8))) void k_eval_elim_rg24(
    const JobDev* jobs, const int* starts, int nj, TablesDev tab, int* fb_count, int* fb_queue) {
  extern __shared__ __align__(16) uint32_t lds[];
  eval_elim_rg_block<24>(jobs, starts, nj, tab, fb_count, fb_queue, lds);
}

#ifndef RG32_WAVES
#define RG32_WAVES 4
#endif
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RG32_WAVES, 8))) void k_eval_elim_rg32(
    const JobDev* jobs, const int* starts, int nj, TablesDev tab, int* fb_count, int* fb_queue) {
  extern __shared__ __align__(16) uint32_t lds[];
  eval_elim_rg_block<32>(jobs, starts, nj, tab, fb_count, fb_queue, lds);
}

// C = 64 (jobs with 32 <= max(m, n) < 64): the steps above degree 30 run the
// guarded fused step in a loop, the rest the unrolled chain.  Its LDS (65
// words per lane) allows 9 blocks per CU, against 4 for the LDS kernel at
// m = n = 63.
#ifndef RG64_WAVES
#define RG64_WAVES 2
#endif
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RG64_WAVES, 8))) void k_eval_elim_rg64(
    const JobDev* jobs, const int* starts, int nj, TablesDev tab, int* fb_count, int* fb_queue) {
  extern __shared__ __align__(16) uint32_t lds[];
  eval_elim_rg_block<64>(jobs, starts, nj, tab, fb_count, fb_queue, lds);
}

// The queued blocks of k_eval_elim_rg, recomputed with the general kernel.
__global__ __launch_bounds__(64) void k_eval_elim_fb(const JobDev* jobs, const int* starts, int nj, TablesDev tab,
                                                     const int* fb_count, const int* fb_queue) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int cnt = *fb_count;
  for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int b = fb_queue[i];
    const int job = find_job(starts, nj, b);
    dev_eval_elim<64, true>(jobs[job], b - starts[job], tab, lds);
  }
}

// ---------------------------------------------------------------------------
// (c) by the displacement structure of the Sylvester matrix (Section 5.1,
// "Computing resultants in Z[x,y]", eq. displ-sylvester): one wave per
// (prime, point) instance, lanes over the generator rows.
//
// S is the transposed Sylvester matrix of the section's example: n columns
// holding f_m .. f_0 shifted down by one per column, then m columns holding
// g_n .. g_0; det S = res(f, g).  With F the down-shift of size r = m + n and
// A = Z_n (+) Z_m the block down-shift with blocks matching S's two column
// blocks, S - F S A^T = G B^T with G = [column 0, column n] of S and B =
// [e_0, e_n] (only the block-leading columns survive the subtraction).
// For any R with R - F R A^T = G B^T, F and A strictly lower triangular, the
// first row of R is g_0 B^T and its first column G b_0^T (g_0, b_0 the first
// rows of G, B), so the pivot is d = g_0 b_0^T; writing g_0 = (c0, c1) and
// b_0 = (e0, e1), the Schur complement scaled by d has the generators
//   G' = [c1 G_0 - c0 G_1, F l],   B' = [e1 B_0 - e0 B_1, A u],
// l = G b_0^T (the first column), u = B g_0^T (the first row), restricted to
// rows 1..: the projector I - b_0^T g_0 / d is (c1, -c0)^T (e1, -e0) / d and
// F l u A^T / d is the other rank-one term.  Row i of F l is l_{i-1}; row i of
// A u is u_{i-1} except at the block start i = n, where it is 0.  Without
// divisions the generators after step k describe c_k times the k-th Schur
// complement, c_0 = 1, c_{k+1} = c_k d_k, so det S = prod_k d_k / prod_k c_k.
// A pivot that vanishes (a leading principal minor of S is 0 mod p, or a
// formal leading coefficient vanishes at the point) sends the wave to
// Euclid's algorithm on lane 0 for that instance.
// NR rows per lane: r <= 64 NR.
template <int NR>
__global__ __launch_bounds__(64) void k_schur(const JobDev* jobs, const int* starts, int nj, TablesDev tab,
                                              int* fallbacks) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int job = find_job(starts, nj, b, gridDim.x);
  const JobDev& J = jobs[job];
  const int lb = b - starts[job];
  const int k = lb / J.D, pt = lb - k * J.D;
  const int m = J.m, n = J.n, r = m + n;
  const int lane = threadIdx.x;
  const ModP q = tab.primes[k];
  const uint32_t* Rf = J.res_f + (size_t)k * J.Tf;
  const uint32_t* Rg = J.res_g + (size_t)k * J.Tg;
  const uint32_t aM = to_mont((uint32_t)pt, q);
  const int dmax = max(J.ldf, J.kind ? J.ldf : J.ldg) - 1;
  uint32_t pw[EV_PW];
  pw[0] = q.one;
#pragma unroll
  for (int i = 1; i < EV_PW; ++i) pw[i] = i <= dmax ? mmul(pw[i - 1], aM, q) : 0u;
  const uint32_t apw = dmax >= EV_PW ? mmul(pw[EV_PW - 1], aM, q) : 0u;
  // generator rows i = lane + 64 h: G = (f_{m-i}(a), g_{n-i}(a)), B = ([i = 0], [i = n]);
  // f(a, y) and g(a, y) also go to LDS (ascending) for the Euclid fallback
  uint32_t* Af = lds;
  uint32_t* Bg = lds + m + 1;
  uint32_t g0[NR], g1[NR], b0[NR], b1[NR];
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int i = lane + 64 * h;
    uint32_t fv = 0u, gv = 0u;
    if (i <= m) {
      fv = eval_row<const uint32_t, const u32x4>(Rf + (m - i) * J.lpf, J.rowdeg_f[m - i], pw, apw, q);
      Af[m - i] = fv;
    }
    if (i <= n) {
      gv = eval_row<const uint32_t, const u32x4>(Rg + (n - i) * J.lpg, J.rowdeg_g[n - i], pw, apw, q);
      Bg[n - i] = gv;
    }
    g0[h] = fv;
    g1[h] = gv;
    b0[h] = i == 0 ? q.one : 0u;
    b1[h] = i == n ? q.one : 0u;
  }
  __syncthreads();  // the LDS copies are complete before a fallback reads them
  uint32_t num = q.one, den = q.one, c = q.one;
  bool ok = true;
  for (int s = 0; s < r; ++s) {
    const int hs = s >> 6, ls = s & 63;
    uint32_t x0 = g0[0], x1 = g1[0], y0 = b0[0], y1 = b1[0];
#pragma unroll
    for (int h = 1; h < NR; ++h)
      if (hs == h) x0 = g0[h], x1 = g1[h], y0 = b0[h], y1 = b1[h];
    const uint32_t c0 = __builtin_amdgcn_readlane(x0, ls), c1 = __builtin_amdgcn_readlane(x1, ls);
    const uint32_t e0 = __builtin_amdgcn_readlane(y0, ls), e1 = __builtin_amdgcn_readlane(y1, ls);
    const uint32_t d = mdot2(c0, e0, c1, e1, q);
    if (d == 0u) {
      ok = false;
      break;
    }
    num = mmul(num, d, q);
    den = mmul(den, c, q);
    c = mmul(c, d, q);
    if (s == r - 1) break;
    const uint32_t nc0 = mneg_factor(c0, q.p), ne0 = mneg_factor(e0, q.p);
    uint32_t l[NR], u[NR];
#pragma unroll
    for (int h = 0; h < NR; ++h) {
      l[h] = mdot2(e0, g0[h], e1, g1[h], q);
      u[h] = mdot2(c0, b0[h], c1, b1[h], q);
      g0[h] = mdot2(c1, g0[h], nc0, g1[h], q);
      b0[h] = mdot2(e1, b0[h], ne0, b1[h], q);
    }
#pragma unroll
    for (int h = 0; h < NR; ++h) {
      uint32_t lp = __shfl_up(l[h], 1), up = __shfl_up(u[h], 1);
      if (lane == 0) {
        lp = h ? __builtin_amdgcn_readlane(l[h > 0 ? h - 1 : 0], 63) : 0u;
        up = h ? __builtin_amdgcn_readlane(u[h > 0 ? h - 1 : 0], 63) : 0u;
      }
      g1[h] = lp;
      b1[h] = lane + 64 * h == n ? 0u : up;
    }
  }
  if (ok) {
    if (lane == 0) put_value(J, k, pt, from_mont(mmul(num, minv(den, q), q), q), q.p);
  } else if (lane == 0) {
    put_value(J, k, pt, from_mont(uni_resultant<1>(Af, Bg, m, n, q), q), q.p);
    atomicAdd(fallbacks, 1);
  }
}

// ---------------------------------------------------------------------------
// Principal subresultant coefficients modulo one prime (Section 3.2.2,
// "(Exact) Computation of N" and "Computation of N^-"): sr_i(a) for every
// index i of the formal degrees (m, n) and every point a, one lane per point.
// sr_i is the determinant of the Sylvester-like matrix with n - i rows of f
// and m - i rows of g restricted to the columns of y^(m+n-i-1) .. y^i.  Row
// operations on that matrix give the recurrence the lanes run (A, B of formal
// degrees a, b):
//   sres_i(A, B) = (-1)^((a-i)(b-i)) sres_i(B, A)            (row blocks exchanged);
//   a > b:  sres_b(A, B) = lc(B)^(a-b)                        (triangular matrix);
//   formal lc(A) = 0, i < b: sres_i(A, B) = (-1)^(b-i) lc(B) sres_i(A of degree a-1, B);
//   formal lc(B) = 0, i < b: sres_i(A, B) = lc(A) sres_i(A, B of degree b-1)
//                             (expansion along the first column);
//   a >= b, R = A mod B of degree c: sres_i(A, B) = 0 for c < i < b and
//   sres_i(A, B) = (-1)^((a-i)(b-i)) lc(B)^(a-c) sres_i(B, R) for i <= c
//   (A's rows minus multiples of B's rows are R's rows; the first a - c
//   B-rows then form a triangular block with lc(B) on its diagonal).
// The eliminations of eliminate() leave scaled remainders s R, whose scalar
// s (a product of powers of leading coefficients) is tracked, so every sr_i(a)
// is num / den with den a product of such scalars; each lane writes its
// (num, den) pairs and inverts its denominators together (one inverse and
// three products per index, Montgomery's simultaneous inversion).  The sign
// of index i is (-1)^(E0 + i E1): (a-i)(b-i) = ab + i (a+b+1) mod 2.

struct PscOut {
  uint32_t* num;  // [K][D] numerators (Montgomery), then the values sr_i(a) (plain)
  uint32_t* den;  // [K][D] denominators (Montgomery)
  int32_t K;      // indices 0..K-1
};

template <int W>
__device__ void psc_lane(uint32_t* A, uint32_t* B, int m, int n, int pt, int D, const ModP& q, PscOut o) {
  uint32_t Nn = q.one, Nd = q.one;
  int E0 = 0, E1 = 0;
  auto emit = [&](int i, uint32_t vn, uint32_t vd) {
    if (i >= o.K) return;  // indices above K are not asked for
    uint32_t x = mmul(Nn, vn, q);
    if ((E0 ^ (i & E1)) & 1) x = mneg(x, q.p);
    o.num[(size_t)i * D + pt] = x;
    o.den[(size_t)i * D + pt] = mmul(Nd, vd, q);
  };
  int a = m, b = n;
  if (a > b)
    emit(b, mpow(B[b * W], (uint32_t)(a - b), q), q.one);
  else if (a < b)
    emit(a, mpow(A[a * W], (uint32_t)(b - a), q), q.one);
  if (a < b) {
    uint32_t* T = A; A = B; B = T;
    const int t = a; a = b; b = t;
    E0 ^= (a * b) & 1;
    E1 ^= (a + b + 1) & 1;
  }
  // formal degrees (only the first pair can have vanishing leading coefficients)
  while (b >= 1) {
    const bool za = A[a * W] == 0u, zb = B[b * W] == 0u;
    if (!za && !zb) break;
    if (za && zb) {  // the first column is zero
      for (int i = 0; i < b; ++i) emit(i, 0u, q.one);
      b = 0;
      break;
    }
    if (zb) {
      Nn = mmul(Nn, A[a * W], q);
      --b;
      emit(b, mpow(B[b * W], (uint32_t)(a - b), q), q.one);
      continue;
    }
    E0 ^= b & 1;
    E1 ^= 1;
    Nn = mmul(Nn, B[b * W], q);
    --a;
    if (a < b) {
      uint32_t* T = A; A = B; B = T;
      const int t = a; a = b; b = t;
      E0 ^= (a * b) & 1;
      E1 ^= (a + b + 1) & 1;
      emit(b, mpow(B[b * W], (uint32_t)(a - b), q), q.one);
    }
  }
  // actual degrees from here: A = sA A*, B = sB B* with A*, B* the exact pair
  uint32_t sA = q.one, sB = q.one;
  while (b >= 1) {
    const uint32_t lb = B[b * W];
    eliminate<W>(A, B, a, b, lb, q);
    int c = b - 1;
    while (c >= 0 && A[c * W] == 0u) --c;
    for (int i = c + 1; i < b; ++i) emit(i, 0u, q.one);
    if (c < 0) break;
    // A now holds lb^(a-b+1) sA (A* mod B*): the remainder's scalar
    const uint32_t sR = mmul(mpow(lb, (uint32_t)(a - b + 1), q), sA, q);
    E0 ^= (a * b) & 1;
    E1 ^= (a + b + 1) & 1;
    Nn = mmul(Nn, mpow(lb, (uint32_t)(a - c), q), q);
    Nd = mmul(Nd, mpow(sB, (uint32_t)(a - c), q), q);
    emit(c, mpow(A[c * W], (uint32_t)(b - c), q), mpow(sR, (uint32_t)(b - c), q));
    uint32_t* T = A; A = B; B = T;
    a = b;
    b = c;
    sA = sB;
    sB = sR;
  }
  // simultaneous inversion of the K denominators: num_i <- num_i d_0 .. d_{i-1},
  // then with inv = 1 / (d_0 .. d_i) from the top, num_i inv = num_i / d_i
  uint32_t pre = q.one;
  for (int i = 0; i < o.K; ++i) {
    const size_t x = (size_t)i * D + pt;
    o.num[x] = mmul(o.num[x], pre, q);
    pre = mmul(pre, o.den[x], q);
  }
  uint32_t inv = minv(pre, q);
  for (int i = o.K - 1; i >= 0; --i) {
    const size_t x = (size_t)i * D + pt;
    const uint32_t v = mmul(o.num[x], inv, q);
    inv = mmul(inv, o.den[x], q);
    o.num[x] = from_mont(v, q);
  }
}

// One block of W lanes = W consecutive points; prime index 0 of tab (the
// caller passes the table shifted to its prime).  LDS: (m + n + 2) W words.
template <int W>
__global__ __launch_bounds__(W) void k_psc(JobDev J, TablesDev tab, PscOut o) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int pt = blockIdx.x * W + (int)threadIdx.x;
  if (pt >= J.D) return;
  uint32_t* A = lds + threadIdx.x;
  uint32_t* B = A + (J.m + 1) * W;
  const ModP q = tab.primes[0];
  eval_pair<W, true>(J, 0, pt, q, A, B);
  psc_lane<W>(A, B, J.m, J.n, pt, J.D, q, o);
}

void launch_psc(const JobDev& J, TablesDev tab, uint32_t* num, uint32_t* den, int K, hipStream_t s) {
  const PscOut o{num, den, K};
  const size_t lds = (size_t)(J.m + J.n + 2) * 64 * sizeof(uint32_t);
  hipLaunchKernelGGL(k_psc<64>, dim3((J.D + 63) / 64), dim3(64), lds, s, J, tab, o);
}

size_t psc_lds_bytes(int m, int n) { return (size_t)(m + n + 2) * 64 * sizeof(uint32_t); }


// ---------------------------------------------------------------------------
// (d) interpolation per prime on the nodes a = 0, 1, ..., D-1.
//
// Sums of products are accumulated exactly in 96 bits (four products of
// values below 2^31 fit in 64 bits) and reduced once per output.


// The 96-bit sum reduced modulo p (plain result).
__device__ __forceinline__ uint32_t reduce96(const Acc96& A, const ModP& q, uint32_t r3) {
  // x = lo_lo + 2^32 lo_hi + 2^64 hi = lo_lo + lo_hi (R)_plain + hi (R^2)_plain;
  // with Montgomery constants R^2 = (R)_M and R^3 = (R^2)_M one two-product
  // reduction gives lo_hi R + hi R^2 mod p.
  const uint32_t l0 = reduce32((uint32_t)A.lo, q.p);
  const uint32_t l1 = reduce32((uint32_t)(A.lo >> 32), q.p);
  const uint32_t h = reduce32(A.hi, q.p);
  return madd(mdot2(l1, q.r2, h, r3, q), l0, q.p);
}

// Divided differences on equally spaced nodes are scaled forward
// differences: c_k = sum_{i<=k} v_i (-1)^{k-i} / (i! (k-i)!), a triangular
// convolution of a_i = v_i / i! with b_j = (-1)^j / j!.  The Newton form
// P(x) = sum_k c_k prod_{t<k} (x - t) is then expanded by Horner's rule over
// blocks of KB nodes: P = sum_b N_{b KB}(x) T_b(x) with
// T_b = sum_{r<KB} c_{b KB + r} prod_{t=b KB}^{b KB + r - 1} (x - t) and
// N_{(b+1) KB} = N_{b KB} Q_b, Q_b = prod_{t=b KB}^{(b+1) KB - 1} (x - t), so
// P <- P Q_b + T_b from the top block down; T_b and Q_b are built with KB
// lane-parallel steps in one wave each.  One block per (job, prime).
constexpr int KB = 32;

// Per-prime block tables of the Newton-to-monomial step (k_interp_tables):
// W[k][b][j][r] = [x^j] prod_{t<r} (x - 32 b - t) and Q[k][b][j] = [x^j]
// prod_{t<32} (x - 32 b - t), plain residues, for blocks b < nb and primes
// k < P.  With them T_b[j] = sum_{r>=j} W[k][b][j][r] c_{32 b + r} is a set of
// independent dot products instead of a 32-step recurrence per block.
struct InterpTab {
  const uint32_t* W = nullptr;
  const uint32_t* Q = nullptr;
  int nb = 0;
};

// LDS layout (words): region R (2 D + 144) holding first a (D + 8, zeros past
// D) and b (4 zeros, then D values, then 8 zeros), later the two padded
// Horner buffers (D + 72 each, coefficient idx at 36 + idx, zeros outside the
// current degree); then the Newton coefficients (D); then T_b, Q_b per block.
// Each thread produces four consecutive outputs of a contraction and keeps a
// sliding window of four operands in registers, so a multiply-add costs a
// quarter of an LDS read instead of two.
__device__ void dev_interp(const JobDev& J, int k, TablesDev tab, uint32_t* lds, InterpTab it = InterpTab{}) {
  const int D = J.D;
  const ModP q = tab.primes[k];
  const uint32_t r3 = mmul(q.r2, q.r2, q);  // (R^2)_M = R^3 mod p
  const int nb = (D + KB - 1) / KB;
  uint32_t* A = lds;                 // a_i = v_i / i!, i < D + 8 (zero past D)
  uint32_t* Bz = lds + D + 8;        // b_j = (-1)^j / j! at Bz[4 + j], zero outside [0, D)
  uint32_t* C = lds + 2 * D + 144;   // Newton coefficients
  uint32_t* TQ = C + D;              // per block: T_b (KB words) then Q_b (KB+1 words)
  const uint32_t* invf = tab.invfact + (size_t)k * tab.dmax;
  const uint32_t* v = J.vals + (size_t)k * D;
  for (int i = threadIdx.x; i < D + 8; i += blockDim.x) {
    uint32_t av = 0u, bv = 0u;
    if (i < D) {
      const uint32_t f = invf[i];  // Montgomery form of 1/i!
      av = mmul(v[i], f, q);
      const uint32_t bj = from_mont(f, q);
      bv = (i & 1) ? mneg(bj, q.p) : bj;
    }
    A[i] = av;
    Bz[4 + i] = bv;
    if (i < 4) Bz[i] = 0u;
  }
  __syncthreads();
  // c_kk = sum_{i <= kk} a_i b_{kk-i} for kk = kk0 .. kk0 + 3: the window
  // holds b_{kk0+u-i}; terms with kk0 + u < i read the zeros below b_0
  for (int kk0 = 4 * threadIdx.x; kk0 < D; kk0 += 4 * blockDim.x) {
    const uint32_t* bb = Bz + 4 + kk0;
    uint64_t w0 = bb[0], w1 = bb[1], w2 = bb[2], w3 = bb[3];
    Acc96 c0, c1, c2, c3;
    for (int i = 0; i < kk0 + 4; i += 4) {
      // four products per partial sum: 4 p^2 < 2^64
      uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint64_t a = A[i + g];
        s0 += a * w0;
        s1 += a * w1;
        s2 += a * w2;
        s3 += a * w3;
        w3 = w2;
        w2 = w1;
        w1 = w0;
        w0 = bb[-(i + g) - 1];
      }
      c0.add(s0);
      c1.add(s1);
      c2.add(s2);
      c3.add(s3);
    }
    C[kk0] = reduce96(c0, q, r3);
    if (kk0 + 1 < D) C[kk0 + 1] = reduce96(c1, q, r3);
    if (kk0 + 2 < D) C[kk0 + 2] = reduce96(c2, q, r3);
    if (kk0 + 3 < D) C[kk0 + 3] = reduce96(c3, q, r3);
  }
  __syncthreads();
  // T_b and Q_b: from the tables when the caller has them, else one wave per
  // block (lanes hold coefficients 0..KB); meanwhile the Horner buffers are cleared
  for (int i = threadIdx.x; i < 2 * D + 144; i += blockDim.x) lds[i] = 0u;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  if (it.W && nb <= it.nb) {
    const uint32_t* W = it.W + (size_t)k * it.nb * KB * KB;
    const uint32_t* Qt = it.Q + (size_t)k * it.nb * (KB + 1);
    for (int o = threadIdx.x; o < nb * KB; o += blockDim.x) {
      const int b = o / KB, j = o - b * KB, base = b * KB, len = min(KB, D - base);
      uint32_t T = 0u;
      if (j < len) {
        const uint32_t* w = W + ((size_t)b * KB + j) * KB;
        Acc96 acc;
        int r = j;
        for (; r + 4 <= len; r += 4) {
          uint64_t sm = (uint64_t)w[r] * C[base + r];
          sm += (uint64_t)w[r + 1] * C[base + r + 1];
          sm += (uint64_t)w[r + 2] * C[base + r + 2];
          sm += (uint64_t)w[r + 3] * C[base + r + 3];
          acc.add(sm);
        }
        uint64_t sm = 0;
        for (; r < len; ++r) sm += (uint64_t)w[r] * C[base + r];
        acc.add(sm);
        T = reduce96(acc, q, r3);
      }
      TQ[b * (2 * KB + 1) + j] = T;
    }
    for (int o = threadIdx.x; o < nb * (KB + 1); o += blockDim.x) {
      const int b = o / (KB + 1), j = o - b * (KB + 1);
      TQ[b * (2 * KB + 1) + KB + j] = Qt[(size_t)b * (KB + 1) + j];
    }
  }
  for (int b = wave; b < nb && !(it.W && nb <= it.nb); b += nwaves) {
    const int base = b * KB;
    const int len = min(KB, D - base);
    uint32_t T = lane == 0 ? C[base + len - 1] : 0u;
    for (int r = len - 2; r >= 0; --r) {  // T <- T (x - (base + r)) + c_{base + r}
      const uint32_t tM = to_mont((uint32_t)(base + r), q);
      const uint32_t up = __shfl_up(T, 1);
      uint32_t nt = msub(lane ? up : 0u, mmul(T, tM, q), q.p);
      if (lane == 0) nt = madd(nt, C[base + r], q.p);
      T = lane <= KB ? nt : 0u;
    }
    uint32_t Q = lane == 0 ? 1u : 0u;
    for (int r = 0; r < KB; ++r) {        // Q <- Q (x - (base + r))
      const uint32_t tM = to_mont((uint32_t)(base + r), q);
      const uint32_t up = __shfl_up(Q, 1);
      const uint32_t nq = msub(lane ? up : 0u, mmul(Q, tM, q), q.p);
      Q = lane <= KB ? nq : 0u;
    }
    if (lane < KB) TQ[b * (2 * KB + 1) + lane] = T;
    if (lane <= KB) TQ[b * (2 * KB + 1) + KB + lane] = Q;
  }
  __syncthreads();
  // Horner over blocks: P <- P Q_b + T_b.  The buffers are zero outside the
  // coefficients written so far (degrees only grow), so the windows need no
  // bounds: indices run from -36 to the degree + 35.
  uint32_t* P0 = lds + 36;
  uint32_t* P1 = lds + (D + 72) + 36;
  int degP = min(KB, D - (nb - 1) * KB) - 1;
  for (int j = threadIdx.x; j <= degP; j += blockDim.x) P0[j] = TQ[(nb - 1) * (2 * KB + 1) + j];
  __syncthreads();
  for (int b = nb - 2; b >= 0; --b) {
    const uint32_t* T = TQ + b * (2 * KB + 1);
    const uint32_t* Qb = T + KB;
    const int degN = degP + KB;
    uint32_t qv[KB + 1];
#pragma unroll
    for (int t = 0; t <= KB; ++t) qv[t] = Qb[t];
    for (int j0 = 4 * threadIdx.x; j0 <= degN; j0 += 4 * blockDim.x) {
      // outputs j0 + u = sum_t q_t P[j0 + u - t] (+ T[j0 + u] below KB);
      // the window holds P[j0 + u - t]
      const uint32_t* pp = P0 + j0;
      uint64_t w0 = pp[0], w1 = pp[1], w2 = pp[2], w3 = pp[3];
      Acc96 c0, c1, c2, c3;
      // eight products per partial sum: 8 p^2 < 2^64 (p < 2^32 / 3)
#pragma unroll
      for (int t0 = 0; t0 <= KB; t0 += 8) {
        uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          const int t = t0 + g;
          if (t <= KB) {
            const uint64_t qt = qv[t];
            s0 += qt * w0;
            s1 += qt * w1;
            s2 += qt * w2;
            s3 += qt * w3;
            w3 = w2;
            w2 = w1;
            w1 = w0;
            w0 = pp[-t - 1];
          }
        }
        c0.add(s0);
        c1.add(s1);
        c2.add(s2);
        c3.add(s3);
      }
      if (j0 < KB) {
        c0.add(T[j0]);
        c1.add(T[j0 + 1]);
        c2.add(T[j0 + 2]);
        c3.add(T[j0 + 3]);
      }
      P1[j0] = reduce96(c0, q, r3);
      if (j0 + 1 <= degN) P1[j0 + 1] = reduce96(c1, q, r3);
      if (j0 + 2 <= degN) P1[j0 + 2] = reduce96(c2, q, r3);
      if (j0 + 3 <= degN) P1[j0 + 3] = reduce96(c3, q, r3);
    }
    __syncthreads();
    uint32_t* tmp = P0; P0 = P1; P1 = tmp;
    degP = degN;
  }
  uint32_t* out = J.coefs + (size_t)k * D;
  for (int j = threadIdx.x; j < D; j += blockDim.x) out[j] = P0[j];
}

__global__ __launch_bounds__(256) void k_interp(const JobDev* jobs, const int* starts, int nj, TablesDev tab,
                                                InterpTab it) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int job = find_job(starts, nj, blockIdx.x, gridDim.x);
  dev_interp(jobs[job], blockIdx.x - starts[job], tab, lds, it);
}

// The tables of InterpTab for blocks b < nb (grid x) and primes k < P (grid
// y): one wave holds N_{b,r} (coefficients 0..32 on lanes 0..32) and steps
// r = 0..31, N <- N (x - (32 b + r)).
__global__ __launch_bounds__(64) void k_interp_tables(int nb, TablesDev tab, uint32_t* W, uint32_t* Q) {
  const int b = blockIdx.x, k = blockIdx.y, lane = threadIdx.x;
  const ModP q = tab.primes[k];
  uint32_t* w = W + ((size_t)k * nb + b) * KB * KB;
  uint32_t N = lane == 0 ? q.one : 0u;
  for (int r = 0; r < KB; ++r) {
    if (lane < KB) w[lane * KB + r] = from_mont(N, q);
    const uint32_t tM = to_mont((uint32_t)(b * KB + r), q);
    const uint32_t up = __shfl_up(N, 1);
    const uint32_t nn = msub(lane ? up : 0u, mmul(N, tM, q), q.p);
    N = lane <= KB ? nn : 0u;
  }
  if (lane <= KB) Q[((size_t)k * nb + b) * (KB + 1) + lane] = from_mont(N, q);
}

size_t interp_lds_words(int D) { return (size_t)3 * D + 144 + (size_t)((D + KB - 1) / KB) * (2 * KB + 1); }

// (d) interpolation of a batch whose jobs share D and P, on the int8 matrix
// cores.  With nodes 0..D-1 the coefficients are C = V^{-1} Y (one column of
// Y per job, V the Vandermonde matrix), a dense product per prime.
//
// V^{-1} mod p is built once per (D, P) by synthetic division: column a holds
// the coefficients of N(x) / (x - a) times 1 / N'(a), N = prod_b (x - b),
// N'(a) = (-1)^(D-1-a) a! (D-1-a)!.  Every residue is stored as four balanced
// base-256 digits of its symmetric representative (int8; |x| < 2^30, so the
// top digit lies in [-64, 64]); then C = sum_{s,t} 256^(s+t) A_s Y_t, and the
// 16 int8 products v_mfma_i32_32x32x32_i8 are summed into 7 int32
// accumulators by weight u = s + t (|G_u| <= 4 Dp 2^14 < 2^31 for Dp < 2^15).
// The epilogue reduces sum_u G_u 256^u mod p.  Matrices are stored per prime
// and digit plane in operand order, padded with zeros to multiples of 32: for
// row tile rt (32 rows) and contraction step ks (32 indices) one 1 KiB block
// holds lane L = r + 32 g's 16 bytes (row 32 rt + r, indices 32 ks + 16 g +
// 0..15), so each operand load of a wave reads 1 KiB contiguously.

typedef int im_v4i __attribute__((ext_vector_type(4)));
typedef int im_v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void put_digits(int8_t* base, size_t plane, size_t off, uint32_t d) {
#pragma unroll
  for (int s = 0; s < 4; ++s) base[s * plane + off] = (int8_t)(d >> (8 * s));
}

// V^{-1} mod p_k for k = blockIdx.x: Ap[k][s][i][a] (s: digit, i: coefficient,
// a: node), Dp x Dp per plane, zero outside [0, D)^2.  LDS: 2 (D + 1) words.
__global__ __launch_bounds__(256) void k_vinv(int D, int Dp, TablesDev tab, int8_t* Ap) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int k = blockIdx.x;
  const ModP q = tab.primes[k];
  uint32_t* cur = lds;
  uint32_t* nxt = lds + D + 1;
  for (int j = threadIdx.x; j <= D; j += blockDim.x) cur[j] = j == 0 ? q.one : 0u;
  __syncthreads();
  for (int b = 0; b < D; ++b) {  // cur has degree b: cur <- cur (x - b)
    const uint32_t bM = to_mont((uint32_t)b, q);
    for (int j = threadIdx.x; j <= b + 1; j += blockDim.x) {
      const uint32_t lo = j ? cur[j - 1] : 0u;
      const uint32_t hi = j <= b ? mmul(bM, cur[j], q) : 0u;
      nxt[j] = msub(lo, hi, q.p);
    }
    __syncthreads();
    uint32_t* t = cur;
    cur = nxt;
    nxt = t;
  }
  const size_t plane = (size_t)Dp * Dp;
  int8_t* base = Ap + (size_t)k * 4 * plane;
  const uint32_t* invf = tab.invfact + (size_t)k * tab.dmax;
  for (int a = threadIdx.x; a < Dp; a += blockDim.x) {
    if (a >= D) {
      for (int i = 0; i < Dp; ++i) put_digits(base, plane, im_off(i, a, Dp), 0u);
      continue;
    }
    uint32_t w = mmul(invf[a], invf[D - 1 - a], q);
    if ((D - 1 - a) & 1) w = mneg(w, q.p);
    const uint32_t aM = to_mont((uint32_t)a, q);
    uint32_t qj = cur[D];  // q_{D-1} = leading coefficient of N
    for (int j = D - 1; j >= 0; --j) {
      put_digits(base, plane, im_off(j, a, Dp), digits4(from_mont(mmul(w, qj, q), q), q.p));
      if (j) qj = madd(cur[j], mmul(aM, qj, q), q.p);  // q_{j-1} = n_j + a q_j
    }
    for (int i = D; i < Dp; ++i) put_digits(base, plane, im_off(i, a, Dp), 0u);
  }
}

// A block of four waves computes a 64 x 64 block of C for one prime, wave w
// the 32 x 32 tile (row tile 2 br + w%2, column tile 2 bc + w/2); grid
// ceil(nit/2) ceil(nnt/2) P blocks in XCD order, so that the blocks of one
// prime, which share its operand planes, run on one XCD and share its L2.
// Accumulator register r of lane l holds row 8 (r/4) + 4 (l/32) + r%4 and
// column l%32 of the tile; operand lanes hold row (A) or column (Y) l%32 and
// contraction indices 16 (l/32) + 0..15 of the 32-wide step.
//
// The operand blocks of a step (1 KiB per tile and digit plane, 16 in all:
// the two row tiles' A planes and the two column tiles' Y planes) go from
// global memory straight into LDS (global_load_lds_dwordx4, no registers),
// each wave fetching four, into a ring of IM_STAGES stages.  A step waits for
// its own stage only (vmcnt leaves the younger stage in flight), then a
// barrier makes every wave's part visible and frees the oldest stage for the
// loads of step s + IM_STAGES - 1.  Each wave reads its tile's eight operand
// blocks from LDS: the block's two row tiles share the A planes and its two
// column tiles the Y planes, so a step fetches half the bytes of four
// independent tiles.  Tiles past the matrix (odd nit or nnt) clamp their
// loads to the last tile and write nothing.
constexpr int IM_STAGES = 3;
constexpr int IM_STAGE_BYTES = 16 * 1024;

__device__ __forceinline__ void im_fetch(const int8_t* src, int8_t* dst) {
  __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                   (void __attribute__((address_space(3)))*)dst, 16, 0, 0);
}

// vmcnt(n) with the other counters left alone (gfx9 s_waitcnt encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8), then the block
// barrier.  The compiler inserts no wait of its own for LDS written by
// global_load_lds, and s_barrier alone does not order memory accesses for
// it: the empty asm statements with a memory clobber keep the LDS reads of
// the step below the wait and the barrier.
#define IM_WAIT_VM_BARRIER(n)                                                        \
  do {                                                                               \
    asm volatile("" ::: "memory");                                                   \
    __builtin_amdgcn_s_waitcnt((((n) & 15) | (((n) >> 4) << 14)) | 0x0F70);          \
    __builtin_amdgcn_s_barrier();                                                    \
    asm volatile("" ::: "memory");                                                   \
  } while (0)

// The same product in the persistent launch, whose register budget (four
// waves per SIMD for the evaluation) cannot hold seven 32 x 32 accumulators
// per wave: a block of four waves computes a 64 x 32 block of C (coefficient
// rows 64 br .., jobs 32 bc .., prime k), wave w the 32 x 16 tile of row tile
// 2 br + w % 2 and column half w / 2 on v_mfma_i32_16x16x32_i8, with all seven
// weight classes of both 16-row halves in 56 accumulator registers.  The
// operand blocks of a step (A planes of the two row tiles, Y planes of the
// column tile: 12 KiB) go through a ring of three stages in LDS (36 KiB), each
// wave fetching three; a wave reads the 8 bytes per lane of its
// 16 x 32 operands (row or column l % 16, indices 8 (l / 16) + 0..7 of the
// step, contiguous in the 1 KiB operand-order blocks).  Accumulator register
// j of lane l: row 4 (l / 16) + j, column l % 16.  Logical block lb: prime
// lb / (nbr nbc), then row pair fastest.
constexpr int IMB_STAGE_BYTES = 12 * 1024;
constexpr int IMB_STAGES = 3;

__device__ __forceinline__ void dev_interp_blk(uint32_t* const* gco, int N, int Np, int D, int Dp, const int8_t* Ap,
                                               const int8_t* Yp, TablesDev tab, int lb, int8_t* im_lds) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63, c16 = l & 15, qd = l >> 4;
  const int nit = Dp >> 5, nct = Np >> 5, nbr = (nit + 1) >> 1;
  const int k = lb / (nbr * nct), rem = lb - k * (nbr * nct);
  const int br = rem % nbr, bc = rem / nbr;
  const int it = 2 * br + (w & 1), hc = w >> 1;
  const size_t pa = (size_t)Dp * Dp, py = (size_t)Np * Dp;
  // this wave's three fetches per step: blocks 3 w .. 3 w + 2 of the twelve
  // (0-7: the A planes of row tiles 2 br, 2 br + 1; 8-11: the Y planes)
  const int8_t* src[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int f = 3 * w + i;
    if (f < 8)
      src[i] = Ap + (size_t)k * 4 * pa + (size_t)(f & 3) * pa + (size_t)min(2 * br + (f >> 2), nit - 1) * Dp * 32 + 16 * l;
    else
      src[i] = Yp + (size_t)k * 4 * py + (size_t)(f - 8) * py + (size_t)bc * Dp * 32 + 16 * l;
  }
  const int nsteps = Dp >> 5;
  // this lane's operand bytes within a block; the wave's A blocks start at
  // (w % 2) 4 KiB, its Y half 256 bytes into the Y blocks
  const int off = (c16 + 32 * (qd >> 1)) * 16 + 8 * (qd & 1);
  const int ra = (w & 1) * 4096 + off, ry = 8192 + hc * 256 + off;
  const int n0 = bc * 32 + hc * 16, i0 = it * 32;
  uint32_t* const cp = it < nit && n0 + c16 < N ? gco[n0 + c16] : nullptr;
  const ModP q = tab.primes[k];
  typedef long long i8x8;
  im_v4i G[2][7];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < 7; ++u) G[h][u] = (im_v4i){0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < IMB_STAGES - 1; ++st) {
    if (st < nsteps) {
#pragma unroll
      for (int i = 0; i < 3; ++i) im_fetch(src[i] + st * 1024, im_lds + st * IMB_STAGE_BYTES + (3 * w + i) * 1024);
    }
  }
  for (int s = 0; s < nsteps; ++s) {
    // this wave's fetches of step s (and the loads before them) are done
    // once at most those of step s + 1 remain
    if (s + 1 < nsteps)
      IM_WAIT_VM_BARRIER(3);
    else
      IM_WAIT_VM_BARRIER(0);
    const int8_t* sb = im_lds + (s % IMB_STAGES) * IMB_STAGE_BYTES;
    i8x8 a[2][4], y[4];
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      a[0][pl] = *(const i8x8*)(sb + ra + pl * 1024);
      a[1][pl] = *(const i8x8*)(sb + ra + pl * 1024 + 256);
      y[pl] = *(const i8x8*)(sb + ry + pl * 1024);
    }
    // the stage read at step s - 1 is free: every wave passed this barrier
    // after its reads of it completed
    const int sn = s + IMB_STAGES - 1;
    if (sn < nsteps) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        im_fetch(src[i] + (size_t)sn * 1024, im_lds + (sn % IMB_STAGES) * IMB_STAGE_BYTES + (3 * w + i) * 1024);
    }
    // digit sd of A against digit td of Y into class sd + td
#pragma unroll
    for (int sd = 0; sd < 4; ++sd)
#pragma unroll
      for (int td = 0; td < 4; ++td)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          G[h][sd + td] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a[h][sd], y[td], G[h][sd + td], 0, 0, 0);
  }
  uint32_t wu[7];  // Montgomery forms of 256^u
  wu[0] = q.one;
  const uint32_t m256 = to_mont(256u, q);
#pragma unroll
  for (int u = 1; u < 7; ++u) wu[u] = mmul(wu[u - 1], m256, q);
  if (cp) {
    uint32_t* dst = cp + (size_t)k * D;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = i0 + 16 * h + 4 * qd + j;
        // |G_u| <= 4 Dp 2^14 <= 2^28 and w_u < p < 2^31: the class sums lie
        // within 7 * 2^58.5 < 2^62 < p 2^32, and adding p 2^32 leaves a value
        // in [0, 2 p 2^32), where redc gives one below 2p
        int64_t acc = (int64_t)q.p << 32;
#pragma unroll
        for (int u = 0; u < 7; ++u) acc += (int64_t)G[h][u][j] * (int64_t)(int32_t)wu[u];
        const uint32_t v = redc((uint64_t)acc, q.p, q.pinv);
        if (i < D) dst[i] = umin32(v, v - q.p);
      }
  }
}

size_t fused_interp_lds_bytes() { return (size_t)IMB_STAGES * IMB_STAGE_BYTES; }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_interp_mfma(
    uint32_t* const* gco, int N, int Np, int D, int Dp, const int8_t* Ap, const int8_t* Yp, TablesDev tab) {
  extern __shared__ __align__(16) int8_t im_lds[];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, r32 = l & 31, g = l >> 5;
  const int nit = Dp >> 5, nnt = Np >> 5, nbr = (nit + 1) >> 1, nbc = (nnt + 1) >> 1;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int k = lb / (nbr * nbc), rem = lb - k * nbr * nbc;
  const int br = rem % nbr, bc = rem / nbr;
  const int it = 2 * br + (w & 1), nt = 2 * bc + (w >> 1);
  const bool live = it < nit && nt < nnt;
  const size_t pa = (size_t)Dp * Dp, py = (size_t)Np * Dp;
  // this wave's four fetches per step: waves 0, 1 the A planes of row tiles
  // 2 br, 2 br + 1, waves 2, 3 the Y planes of column tiles 2 bc, 2 bc + 1
  // (operand-order blocks: 1 KiB per (tile, step), lane l holds bytes 16 l..)
  const int8_t* src;
  size_t pstride;
  if (w < 2) {
    src = Ap + (size_t)k * 4 * pa + (size_t)min(2 * br + w, nit - 1) * Dp * 32 + 16 * l;
    pstride = pa;
  } else {
    src = Yp + (size_t)k * 4 * py + (size_t)min(2 * bc + w - 2, nnt - 1) * Dp * 32 + 16 * l;
    pstride = py;
  }
  // stage layout: [row tile 0: 4 planes][row tile 1][column tile 0][column tile 1], 1 KiB each
  int8_t* const dst0 = im_lds + w * 4096;
  const int ra = (w & 1) * 4096 + 16 * l, ry = 8192 + (w >> 1) * 4096 + 16 * l;
  const int nsteps = Dp >> 5;
  const int n0 = nt * 32, i0 = it * 32;
  // each column's output row (null past the group or the matrix), loaded
  // before the products so that its latency is hidden; every job of the
  // group has P primes
  uint32_t* const cpp = l < 32 && live && n0 + l < N ? gco[n0 + l] : nullptr;
  const ModP q = tab.primes[k];  // likewise
#pragma unroll
  for (int st = 0; st < IM_STAGES - 1; ++st) {
    if (st < nsteps) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) im_fetch(src + pl * pstride + st * 1024, dst0 + st * IM_STAGE_BYTES + pl * 1024);
    }
  }
  im_v16i G0 = {0}, G1 = {0}, G2 = {0}, G3 = {0}, G4 = {0}, G5 = {0}, G6 = {0};
  for (int s = 0; s < nsteps; ++s) {
    // this wave's fetches of step s (and the loads before them) are done
    // once at most those of step s + 1 remain
    if (s + 1 < nsteps)
      IM_WAIT_VM_BARRIER(4);
    else
      IM_WAIT_VM_BARRIER(0);
    const int8_t* sb = im_lds + (s % IM_STAGES) * IM_STAGE_BYTES;
    const im_v4i a0 = *(const im_v4i*)(sb + ra), a1 = *(const im_v4i*)(sb + ra + 1024),
                 a2 = *(const im_v4i*)(sb + ra + 2048), a3 = *(const im_v4i*)(sb + ra + 3072);
    const im_v4i y0 = *(const im_v4i*)(sb + ry), y1 = *(const im_v4i*)(sb + ry + 1024),
                 y2 = *(const im_v4i*)(sb + ry + 2048), y3 = *(const im_v4i*)(sb + ry + 3072);
    // the stage read at step s - 1 is free: every wave passed this barrier
    // after its reads of it completed
    const int sn = s + IM_STAGES - 1;
    if (sn < nsteps) {
      int8_t* d = dst0 + (sn % IM_STAGES) * IM_STAGE_BYTES;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) im_fetch(src + pl * pstride + (size_t)sn * 1024, d + pl * 1024);
    }
    G0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, y0, G0, 0, 0, 0);
    G1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, y1, G1, 0, 0, 0);
    G1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, y0, G1, 0, 0, 0);
    G2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, y2, G2, 0, 0, 0);
    G2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, y1, G2, 0, 0, 0);
    G2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, y0, G2, 0, 0, 0);
    G3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, y3, G3, 0, 0, 0);
    G3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, y2, G3, 0, 0, 0);
    G3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, y1, G3, 0, 0, 0);
    G3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a3, y0, G3, 0, 0, 0);
    G4 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, y3, G4, 0, 0, 0);
    G4 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, y2, G4, 0, 0, 0);
    G4 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a3, y1, G4, 0, 0, 0);
    G5 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, y3, G5, 0, 0, 0);
    G5 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a3, y2, G5, 0, 0, 0);
    G6 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a3, y3, G6, 0, 0, 0);
  }
  // every wave's last reads are done before the ring is reused for the transposes
  __syncthreads();
  uint32_t(*tile)[33] = (uint32_t(*)[33])(im_lds + w * (32 * 33 * 4));
  uint32_t** colp = (uint32_t**)(im_lds + 4 * (32 * 33 * 4)) + 32 * w;
  if (l < 32) colp[l] = cpp ? cpp + (size_t)k * D : nullptr;
  uint32_t wu[7];  // Montgomery forms of 256^u
  wu[0] = q.one;
  const uint32_t m256 = to_mont(256u, q);
#pragma unroll
  for (int u = 1; u < 7; ++u) wu[u] = mmul(wu[u - 1], m256, q);
  // |G_u| <= 4 Dp 2^14 <= 2^28 and w_u < p < 2^31, so sum_u G_u w_u lies
  // within 7 * 2^58.5 < 2^62 < p 2^32; adding p 2^32 (a multiple of p) makes
  // it non-negative and below 2 p 2^32, where one Montgomery reduction
  // leaves a value below 3p, hence one more conditional subtraction
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int32_t gv[7] = {G0[r], G1[r], G2[r], G3[r], G4[r], G5[r], G6[r]};
    int64_t acc = (int64_t)q.p << 32;
#pragma unroll
    for (int u = 0; u < 7; ++u) acc += (int64_t)gv[u] * (int64_t)(int32_t)wu[u];
    const uint32_t v = redc((uint64_t)acc, q.p, q.pinv);
    tile[r32][8 * (r >> 2) + 4 * g + (r & 3)] = umin32(v, v - q.p);  // [column][row]
  }
  __syncthreads();
  // lanes 0-31 write column n0 + 2c, lanes 32-63 column n0 + 2c + 1: 32 rows each
  const int i = i0 + r32;
  for (int c = 0; c < 16; ++c) {
    const int col = 2 * c + g;
    uint32_t* dst = colp[col];
    if (dst && i < D) dst[i] = tile[col][r32];
  }
}

static size_t interp_mfma_lds_bytes() {
  // the stage ring, reused after the products for four transposes and column pointers
  const size_t ring = (size_t)IM_STAGES * IM_STAGE_BYTES;
  const size_t epi = 4 * (32 * 33 * 4) + 4 * 32 * sizeof(uint32_t*);
  return ring > epi ? ring : epi;
}

// Inverse factorials per prime: invfact[k][n] = Montgomery form of 1/n!.
// One thread per prime: prefix products, one Fermat inverse, backward products.
__global__ void k_invfact(const ModP* primes, int K, uint32_t* invfact, int dmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const ModP q = primes[k];
  uint32_t* t = invfact + (size_t)k * dmax;
  uint32_t f = q.one;  // 0! in Montgomery form
  t[0] = f;
  for (int n = 1; n < dmax; ++n) {
    f = mmul(f, to_mont((uint32_t)n, q), q);
    t[n] = f;  // n! for now
  }
  uint32_t inv = minv(f, q);  // 1/(dmax-1)!
  for (int n = dmax - 1; n >= 1; --n) {
    t[n] = inv;
    inv = mmul(inv, to_mont((uint32_t)n, q), q);  // 1/(n-1)! = n / n!
  }
  t[0] = q.one;
}

void launch_invfact(const ModP* primes, int K, uint32_t* invfact, int dmax, hipStream_t s) {
  hipLaunchKernelGGL(k_invfact, dim3((K + 63) / 64), dim3(64), 0, s, primes, K, invfact, dmax);
}

// ---------------------------------------------------------------------------
// (e) mixed-radix conversion (Garner).  With primes p_0 > p_1 > ... the value
// is sum_j v_j prod_{i<j} p_i, v_j in [0, p_j), and
// v_k = (x_k - sum_{j<k} v_j prod_{i<j} p_i) (prod_{i<k} p_i)^{-1} mod p_k.
// The symmetric lift is negative exactly when the digit vector exceeds
// ((p_k - 1)/2)_k lexicographically from the top, because
// sum_k (p_k - 1)/2 prod_{i<k} p_i = (M - 1)/2.  Digits are stored [P][D].

__device__ __forceinline__ int lift_negative(const uint32_t* v, int stride, int P, const ModP* primes) {
  for (int kk = P - 1; kk >= 0; --kk) {
    const uint32_t h = (primes[kk].p - 1u) >> 1;
    const uint32_t x = v[kk * stride];
    if (x != h) return x > h ? 1 : 0;
  }
  return 0;
}

// One wave per coefficient, lanes over primes k = lane + 64 t: lane k keeps
// acc_k = sum_{j<k} v_j prod_{i<j} p_i mod p_k; at step j the owner lane of j
// finishes v_j and broadcasts it.
template <bool WAVE>
__device__ void dev_mrc_wave(const JobDev& J, int c, TablesDev tab, uint32_t* lds) {
  const int P = J.P, D = J.D;
  const int lane = lane_id();
  uint32_t* x = lds;        // residues, then digits
  uint32_t* acc = lds + P;  // running prefix values
  for (int kk = lane; kk < P; kk += 64) {
    x[kk] = J.coefs[(size_t)kk * D + c];
    acc[kk] = 0u;
  }
  for (int j = 0; j < P; ++j) {
    const int owner = j & 63;
    uint32_t v = 0;
    if (lane == owner) {
      const ModP qj = tab.primes[j];
      v = mmul(msub(x[j], acc[j], qj.p), tab.cm[j], qj);
      x[j] = v;
      J.digits[(size_t)j * D + c] = v;
    }
    v = __builtin_amdgcn_readlane(v, owner);
    const uint32_t* g = tab.gm + (size_t)j * tab.K;
    for (int kk = lane; kk < P; kk += 64) {
      if (kk > j) {
        const ModP qk = tab.primes[kk];
        acc[kk] = madd(acc[kk], mmul(reduce32(v, qk.p), g[kk], qk), qk.p);
      }
    }
  }
  group_sync<WAVE>();
  if (lane == 0) J.negflag[c] = lift_negative(x, 1, P, tab.primes);
}

__global__ __launch_bounds__(64) void k_mrc(const JobDev* jobs, const int* starts, int nj, TablesDev tab) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int job = find_job(starts, nj, blockIdx.x, gridDim.x);
  dev_mrc_wave<false>(jobs[job], blockIdx.x - starts[job], tab, lds);
}

// (e) limb assembly, pass 1: one thread per (limb l, coefficient c) forms the
// 96-bit column sum S_l = sum_k d_k limb_l(prod_{i<k} p_i), with d_k the digit
// (non-negative lift) or p_k - 1 - digit (negative lift: then
// M - v - 1 = sum (p_k - 1 - v_k) prod_{i<k} p_i).  Flat index l * D + c,
// 256 per block; sums stored [Lacc][D].
__device__ void dev_limbs_sum(const JobDev& J, int lb, TablesDev tab) {
  const int idx = lb * (int)blockDim.x + threadIdx.x;
  const int D = J.D;
  if (idx >= D * J.Lacc) return;
  const int l = idx / D;
  const int c = idx - l * D;
  const int neg = J.negflag[c];
  uint64_t lo = 0;
  uint32_t hi = 0;
  for (int k = l; k < J.P; ++k) {
    uint32_t d = J.digits[(size_t)k * D + c];
    if (neg) d = tab.primes[k].p - 1u - d;
    const uint64_t prod = (uint64_t)d * tab.pi[(size_t)k * (k + 1) / 2 + l];
    lo += prod;
    hi += (lo < prod) ? 1u : 0u;
  }
  J.acc_lo[idx] = lo;
  J.acc_hi[idx] = hi;
}

__global__ void k_limbs_sum(const JobDev* jobs, const int* starts, int nj, TablesDev tab) {
  const int job = find_job(starts, nj, blockIdx.x, gridDim.x);
  dev_limbs_sum(jobs[job], blockIdx.x - starts[job], tab);
}

// (e) limb assembly, pass 2: one lane per output coefficient propagates the
// carries; a negative lift writes the bitwise complement (two's complement of
// -(C + 1) is ~C).  The 64 coefficients of a block are staged in LDS and
// written out contiguously when they fit.  Overflow of the caller's limb count
// sets err.
constexpr int CARRY_STAGE_MAXL = 128;

// stage_ld > 0: LDS rows of stage_ld words (>= Lcap + 1 of every job); 0: direct writes.
template <bool WAVE>
__device__ void dev_limbs_carry(const JobDev& J, int lb, int stage_ld, uint32_t* lds) {
  const int c0 = lb * 64;
  const int lane = lane_id();
  const int c = c0 + lane;
  const int Lc = J.Lcap, D = J.D;
  const bool staged = stage_ld > 0;
  const int ld = stage_ld;
  bool nz = false;
  if (c <= J.degcap) {
    uint32_t* o = staged ? lds + lane * ld : J.out + (size_t)c * Lc;
    if (c >= D) {
      for (int l = 0; l < Lc; ++l) o[l] = 0u;
    } else {
      const int neg = J.negflag[c];
      const uint32_t flip = neg ? 0xFFFFFFFFu : 0u;
      uint64_t carry = 0;  // < 2^50
      nz = neg != 0;
      uint32_t last = 0;
      for (int l = 0; l < Lc; ++l) {
        uint64_t lo = 0;
        uint32_t hi = 0;
        if (l < J.Lacc) {
          lo = J.acc_lo[(size_t)l * D + c];
          hi = J.acc_hi[(size_t)l * D + c];
        }
        const uint64_t s = lo + carry;
        const uint32_t ovf = s < lo ? 1u : 0u;
        const uint32_t w = (uint32_t)s;
        carry = (s >> 32) + ((uint64_t)(hi + ovf) << 32);
        nz |= w != 0u;
        last = w ^ flip;
        o[l] = last;
      }
      if (carry != 0u || ((last >> 31) != (flip >> 31))) atomicOr(J.err, 1);
    }
  }
  {
    // one atomic per wave: the highest non-zero coefficient of the 64
    const uint64_t any = __ballot(nz);
    if (any && lane == 0) atomicMax(J.deg_out, c0 + 63 - __clzll((long long)any));
  }
  if (staged) {
    group_sync<WAVE>();
    const int nc = min(64, J.degcap + 1 - c0);
    uint32_t* dst = J.out + (size_t)c0 * Lc;
    for (int i = lane; i < nc * Lc; i += 64) {
      const int r = i / Lc;
      dst[i] = lds[r * ld + (i - r * Lc)];
    }
  }
}

__global__ __launch_bounds__(64) void k_limbs_carry(const JobDev* jobs, const int* starts, int nj, int stage_ld) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int job = find_job(starts, nj, blockIdx.x, gridDim.x);
  dev_limbs_carry<false>(jobs[job], blockIdx.x - starts[job], stage_ld, lds);
}

// (e) explicit CRT on the int8 matrix cores.  With M = prod_{k<P} p_k,
// M_k = M / p_k and w_k = M_k^{-1} mod p_k, let y_k be the symmetric
// representative of x_k w_k mod p_k (|y_k| < p_k / 2).  Then X = sum_k y_k M_k
// is congruent to the coefficient modulo every p_k and X / M = sum_k y_k / p_k,
// so the coefficient is X - t M with t the integer nearest to that sum (the
// planner takes M > 2^1.001 B, B the coefficient bound, and fp64 gives the sum
// within P 2^-52 of its value, far inside the margin of more than 3e-4 to a
// half-integer).
//
// X is a contraction: with y_k = sum_s d_ks 256^s and M_k = sum_j e_kj 256^j in
// balanced base-256 digits (int8), X = sum_c S_c 256^c where
// S_c = sum_{k,s} d_ks e_k(c - s).  For one coefficient per row that is a
// product [rows x 4P] x [4P x byte columns] whose right operand depends only on
// P (crt_tables builds it in operand order); |S_c| < 2^23 for P <= 128.
// One wave per 32 NT coefficients of one job, in NT row tiles of 32 (NT = 2
// up to 48 primes, 1 above, for registers): the lanes form the digit words
// of their rows' y_k straight into the left operands (lane x + 32 g: row x
// of each tile, primes 8 ks + 4 g + 0..3 of step ks, four digits each), then
// for each tile of 32 byte columns, low to high, v_mfma_i32_32x32x32_i8 over
// the steps for every row tile with one right operand, the tiles through
// LDS, and lane l < 32 NT folds row l's 32 columns into eight 32-bit limbs of
// X - t M with a signed carry kept in a register (at NT = 2 every lane has a
// row of the serial carry chain).  The limbs are staged in LDS rows of sld
// words and written as one contiguous range.
constexpr int CRT_MAXP = 128;

// Every lane runs the same instructions: indices past the job's primes or
// degree bound are clamped for the loads and their values masked to zero, and
// all KSMAX steps run (the left operand is zero past the job's KS steps), so
// the loads of a phase are issued together instead of behind per-lane branches.
//
// A job has ceil(min(D, degcap + 1) / rows) blocks.  The coefficients above
// the last block up to the output capacity (the degree bound of the
// extents, which can be twice D) are zero; each block of the job writes an
// equal share of them while its residue loads are in flight.
//
// Up to 64 primes the right operand blocks of column tile ct + 2 are loaded
// while tile ct is folded (two register sets, the loop unrolled by two),
// which hides the L2 latency behind two tiles of work; above, those of tile
// ct + 1.
template <int KSMAX>
__device__ __forceinline__ void crt_load_b(im_v4i (&B)[KSMAX], const __attribute__((address_space(1))) uint32_t* Bt,
                                           int ct, int NCT, int KS) {
  const __attribute__((address_space(1))) uint32_t* Bn = Bt + (size_t)min(ct, NCT - 1) * KS * 256;
#pragma unroll
  for (int ks = 0; ks < KSMAX; ++ks)
    B[ks] = *(const __attribute__((address_space(1))) im_v4i*)(Bn + (size_t)min(ks, KS - 1) * 256);
}

// The same on one wave of a larger block (the persistent launch), with its
// own LDS slice: block b of the launch's nb, one operand set for registers.
template <int KSMAX, int NT>
__device__ __forceinline__ void dev_crt(const JobDev* jobs, const int* starts, int nj, int sld, int cps, TablesDev tab,
                                        int b, int nb, uint32_t* lds) {
  constexpr int ROWS = 32 * NT;
  const int l = lane_id(), x = l & 31, g = l >> 5;
  const int job = find_job(starts, nj, b, nb);
  const JobDev& J = jobs[job];
  const int P = J.P, D = J.D, Lc = J.Lcap, LM = J.crt_LM;
  const int KS = (P + 7) >> 3, NCT = (4 * LM + 4 + 31) >> 5;
  const int bj = b - starts[job], c0 = bj * ROWS;
  int32_t* T = (int32_t*)lds;     // [ROWS][33]: the accumulator tiles, [row][column]
  uint32_t* O = lds + ROWS * 33;  // [ROWS][sld]: limbs of the rows, then the prime constants
  const uint32_t* wv = J.crt;
  const uint32_t* Mw = J.crt + P + (size_t)P * LM;
  const __attribute__((address_space(1))) uint32_t* Bt =
      gmem(J.crt) + (((size_t)P + (size_t)P * LM + LM + 3) & ~(size_t)3) + 4 * l;
  bool rv[NT];
  // this lane's residues (primes 8 ks + 4 g + j) of its row in each tile, all
  // issued before the barrier
  uint32_t xr[NT][KSMAX * 4];
#pragma unroll
  for (int h = 0; h < NT; ++h) {
    rv[h] = c0 + 32 * h + x < D;
    const __attribute__((address_space(1))) uint32_t* col = gmem(J.coefs) + min(c0 + 32 * h + x, D - 1);
#pragma unroll
    for (int u = 0; u < KSMAX * 4; ++u) xr[h][u] = col[(size_t)min(8 * (u >> 2) + 4 * g + (u & 3), P - 1) * D];
  }
  // the first column tile's operand blocks, also issued before the barrier
  im_v4i Ba[KSMAX];
  crt_load_b<KSMAX>(Ba, Bt, 0, NCT, KS);
  {
    // this block's share of the zero coefficients above the job's last block
    const int nbj = (min(D, J.degcap + 1) + ROWS - 1) / ROWS, cz = nbj * ROWS;
    if (cz <= J.degcap) {
      const long long nw = (long long)(J.degcap + 1 - cz) * Lc, share = (nw + nbj - 1) / nbj;
      const long long w0 = bj * share, w1 = min(nw, w0 + share);
      uint32_t* dst = J.out + (size_t)cz * Lc;
      for (long long i = w0 + l; i < w1; i += 64) dst[i] = 0u;
    }
  }
  // per-prime constants staged in LDS at stride cps (the batch's largest
  // prime count, rounded up to even): p, -p^{-1} mod 2^32, w_k, 1 / p_k; then
  // the words of M, zero from LM up to the last byte column's limb
  uint32_t* Cp = O + ROWS * sld;
  double* Ci = (double*)(Cp + 3 * cps);
  uint32_t* Ms = Cp + 5 * cps;
  for (int k = l; k < P; k += 64) {
    const ModP q = tab.primes[k];
    Cp[k] = q.p;
    Cp[cps + k] = q.pinv;
    Cp[2 * cps + k] = wv[k];
    Ci[k] = tab.inv_p[k];
  }
  for (int w = l; w < 8 * NCT; w += 64) Ms[w] = w < LM ? Mw[w] : 0u;
  group_sync<true>();
  im_v4i A[NT][KSMAX];
  double f[NT];
#pragma unroll
  for (int h = 0; h < NT; ++h) f[h] = 0.0;
#pragma unroll
  for (int ks = 0; ks < KSMAX; ++ks) {
    uint32_t d[NT][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = 4 * ks + j, kl = 8 * ks + 4 * g + j, k = min(kl, P - 1);
      const uint32_t p = Cp[k], pinv = Cp[cps + k], wk = Cp[2 * cps + k];
      const double ip = Ci[k];
#pragma unroll
      for (int h = 0; h < NT; ++h) {
        const bool live = rv[h] && kl < P;
        const uint32_t y = redc((uint64_t)xr[h][u] * wk, p, pinv);
        const int32_t ys = y > (p >> 1) ? (int32_t)(y - p) : (int32_t)y;
        f[h] = fma((double)(live ? ys : 0), ip, f[h]);
        d[h][j] = digits4(y, p) & (0u - (uint32_t)live);
      }
    }
#pragma unroll
    for (int h = 0; h < NT; ++h) A[h][ks] = (im_v4i){(int)d[h][0], (int)d[h][1], (int)d[h][2], (int)d[h][3]};
  }
  // from here on lane l < ROWS owns row c0 + l (row x of tile g)
  int64_t tq = 0;
  bool row = false;
#pragma unroll
  for (int h = 0; h < NT; ++h) {
    const double fs = f[h] + __shfl_xor(f[h], 32);
    if (g == h) {
      tq = (int64_t)floor(fs + 0.5);
      row = rv[h];
    }
  }
  const bool owner = l < ROWS;
  int64_t carry = 0;
  uint32_t last = 0;
  bool bad = false, nz = false;
  // one column tile: products, the tiles through LDS, the carry chain
  auto tile = [&](int ct, const im_v4i(&B)[KSMAX]) {
    im_v16i acc[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) acc[h] = (im_v16i){0};
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks)
#pragma unroll
      for (int h = 0; h < NT; ++h) acc[h] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[h][ks], B[ks], acc[h], 0, 0, 0);
    // accumulator register r of lane l: row 8 (r / 4) + 4 g + r % 4 of its tile, column x
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) T[(32 * h + 8 * (r >> 2) + 4 * g + (r & 3)) * 33 + x] = acc[h][r];
    group_sync<true>();
    if (owner) {
      const int32_t* t = T + l * 33;
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const int L = 8 * ct + w;
        // |S_c| <= P (3 * 128 + 64) 128 < 2^23 (the top digit of y_k is at most
        // 64 in size), so t_0 + 2^8 t_1 and t_2 + 2^8 t_3 fit in 32 bits
        const int32_t lo = t[4 * w] + (t[4 * w + 1] << 8), hi = t[4 * w + 2] + (t[4 * w + 3] << 8);
        const int64_t v = carry + (int64_t)lo + ((int64_t)hi << 16) - tq * (int64_t)Ms[L];
        const uint32_t limb = (uint32_t)v;
        carry = v >> 32;
        if (L < Lc) {
          O[l * sld + L] = limb;
          nz |= limb != 0u;
          last = limb;
        } else if (limb != ((int32_t)last < 0 ? 0xFFFFFFFFu : 0u)) {
          bad = true;
        }
      }
    }
    group_sync<true>();
  };
  for (int ct = 0; ct < NCT; ++ct) {
    tile(ct, Ba);
    crt_load_b<KSMAX>(Ba, Bt, ct + 1, NCT, KS);
  }
  if (owner) {
    // limbs above the last byte column: the carry's extension
    for (int L = 8 * NCT; L < Lc; ++L) {
      const uint32_t limb = (uint32_t)carry;
      carry >>= 32;
      O[l * sld + L] = limb;
      nz |= limb != 0u;
      last = limb;
    }
    if (row && (bad || carry != ((int32_t)last < 0 ? -1 : 0))) atomicOr(J.err, 1);
  }
  // one atomic per wave: the highest non-zero coefficient of the block
  const uint64_t any = __ballot(owner && row && nz);
  if (any && l == 0) atomicMax(J.deg_out, c0 + 63 - __clzll((long long)any));
  group_sync<true>();
  // rows c0 .. c0 + nr - 1 are one contiguous range of nr Lc words
  const int nr = min(ROWS, J.degcap + 1 - c0);
  uint32_t* dst = J.out + (size_t)c0 * Lc;
  const int dq = 64 / Lc, dr = 64 - dq * Lc;
  int r = l / Lc, L = l - r * Lc;
  for (int i = l; i < nr * Lc; i += 64) {
    dst[i] = O[r * sld + L];
    r += dq;
    L += dr;
    if (L >= Lc) {
      L -= Lc;
      ++r;
    }
  }
}

// The staged kernel keeps its own copy of the body above (with two operand
// sets up to 64 primes): called through the device function, the compiler
// schedules the operand loads differently and takes 255 VGPRs for 48 primes
// (one wave per SIMD, 30 -> 44 us for 256 degree-20 pairs) instead of 150.
template <int KSMAX, int NT>
__global__ __launch_bounds__(64) void k_crt_mfma(const JobDev* jobs, const int* starts, int nj, int sld, int cps,
                                                 TablesDev tab) {
  constexpr int ROWS = 32 * NT;
  extern __shared__ __align__(16) uint32_t lds[];
  const int l = threadIdx.x, x = l & 31, g = l >> 5;
  const int job = find_job(starts, nj, blockIdx.x, gridDim.x);
  const JobDev& J = jobs[job];
  const int P = J.P, D = J.D, Lc = J.Lcap, LM = J.crt_LM;
  const int KS = (P + 7) >> 3, NCT = (4 * LM + 4 + 31) >> 5;
  const int bj = blockIdx.x - starts[job], c0 = bj * ROWS;
  int32_t* T = (int32_t*)lds;     // [ROWS][33]: the accumulator tiles, [row][column]
  uint32_t* O = lds + ROWS * 33;  // [ROWS][sld]: limbs of the rows, then the prime constants
  const uint32_t* wv = J.crt;
  const uint32_t* Mw = J.crt + P + (size_t)P * LM;
  const __attribute__((address_space(1))) uint32_t* Bt =
      gmem(J.crt) + (((size_t)P + (size_t)P * LM + LM + 3) & ~(size_t)3) + 4 * l;
  bool rv[NT];
  // this lane's residues (primes 8 ks + 4 g + j) of its row in each tile, all
  // issued before the barrier
  uint32_t xr[NT][KSMAX * 4];
#pragma unroll
  for (int h = 0; h < NT; ++h) {
    rv[h] = c0 + 32 * h + x < D;
    const __attribute__((address_space(1))) uint32_t* col = gmem(J.coefs) + min(c0 + 32 * h + x, D - 1);
#pragma unroll
    for (int u = 0; u < KSMAX * 4; ++u) xr[h][u] = col[(size_t)min(8 * (u >> 2) + 4 * g + (u & 3), P - 1) * D];
  }
  // the first column tiles' operand blocks (two sets up to 64 primes, one
  // above, for registers), also issued before the barrier
  constexpr bool B2 = KSMAX <= 8;
  im_v4i Ba[KSMAX], Bb[B2 ? KSMAX : 1];
  crt_load_b<KSMAX>(Ba, Bt, 0, NCT, KS);
  if constexpr (B2) crt_load_b<KSMAX>(Bb, Bt, 1, NCT, KS);
  {
    // this block's share of the zero coefficients above the job's last block
    const int nbj = (min(D, J.degcap + 1) + ROWS - 1) / ROWS, cz = nbj * ROWS;
    if (cz <= J.degcap) {
      const long long nw = (long long)(J.degcap + 1 - cz) * Lc, share = (nw + nbj - 1) / nbj;
      const long long w0 = bj * share, w1 = min(nw, w0 + share);
      uint32_t* dst = J.out + (size_t)cz * Lc;
      for (long long i = w0 + l; i < w1; i += 64) dst[i] = 0u;
    }
  }
  // per-prime constants staged in LDS at stride cps (the batch's largest
  // prime count, rounded up to even): p, -p^{-1} mod 2^32, w_k, 1 / p_k; then
  // the words of M, zero from LM up to the last byte column's limb
  uint32_t* Cp = O + ROWS * sld;
  double* Ci = (double*)(Cp + 3 * cps);
  uint32_t* Ms = Cp + 5 * cps;
  for (int k = l; k < P; k += 64) {
    const ModP q = tab.primes[k];
    Cp[k] = q.p;
    Cp[cps + k] = q.pinv;
    Cp[2 * cps + k] = wv[k];
    Ci[k] = tab.inv_p[k];
  }
  for (int w = l; w < 8 * NCT; w += 64) Ms[w] = w < LM ? Mw[w] : 0u;
  __syncthreads();
  im_v4i A[NT][KSMAX];
  double f[NT];
#pragma unroll
  for (int h = 0; h < NT; ++h) f[h] = 0.0;
#pragma unroll
  for (int ks = 0; ks < KSMAX; ++ks) {
    uint32_t d[NT][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = 4 * ks + j, kl = 8 * ks + 4 * g + j, k = min(kl, P - 1);
      const uint32_t p = Cp[k], pinv = Cp[cps + k], wk = Cp[2 * cps + k];
      const double ip = Ci[k];
#pragma unroll
      for (int h = 0; h < NT; ++h) {
        const bool live = rv[h] && kl < P;
        const uint32_t y = redc((uint64_t)xr[h][u] * wk, p, pinv);
        const int32_t ys = y > (p >> 1) ? (int32_t)(y - p) : (int32_t)y;
        f[h] = fma((double)(live ? ys : 0), ip, f[h]);
        d[h][j] = digits4(y, p) & (0u - (uint32_t)live);
      }
    }
#pragma unroll
    for (int h = 0; h < NT; ++h) A[h][ks] = (im_v4i){(int)d[h][0], (int)d[h][1], (int)d[h][2], (int)d[h][3]};
  }
  // from here on lane l < ROWS owns row c0 + l (row x of tile g)
  int64_t tq = 0;
  bool row = false;
#pragma unroll
  for (int h = 0; h < NT; ++h) {
    const double fs = f[h] + __shfl_xor(f[h], 32);
    if (g == h) {
      tq = (int64_t)floor(fs + 0.5);
      row = rv[h];
    }
  }
  const bool owner = l < ROWS;
  int64_t carry = 0;
  uint32_t last = 0;
  bool bad = false, nz = false;
  // one column tile: products, the tiles through LDS, the carry chain
  auto tile = [&](int ct, const im_v4i(&B)[KSMAX]) {
    im_v16i acc[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) acc[h] = (im_v16i){0};
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks)
#pragma unroll
      for (int h = 0; h < NT; ++h) acc[h] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[h][ks], B[ks], acc[h], 0, 0, 0);
    // accumulator register r of lane l: row 8 (r / 4) + 4 g + r % 4 of its tile, column x
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) T[(32 * h + 8 * (r >> 2) + 4 * g + (r & 3)) * 33 + x] = acc[h][r];
    __syncthreads();
    if (owner) {
      const int32_t* t = T + l * 33;
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const int L = 8 * ct + w;
        // |S_c| <= P (3 * 128 + 64) 128 < 2^23 (the top digit of y_k is at most
        // 64 in size), so t_0 + 2^8 t_1 and t_2 + 2^8 t_3 fit in 32 bits
        const int32_t lo = t[4 * w] + (t[4 * w + 1] << 8), hi = t[4 * w + 2] + (t[4 * w + 3] << 8);
        const int64_t v = carry + (int64_t)lo + ((int64_t)hi << 16) - tq * (int64_t)Ms[L];
        const uint32_t limb = (uint32_t)v;
        carry = v >> 32;
        if (L < Lc) {
          O[l * sld + L] = limb;
          nz |= limb != 0u;
          last = limb;
        } else if (limb != ((int32_t)last < 0 ? 0xFFFFFFFFu : 0u)) {
          bad = true;
        }
      }
    }
    __syncthreads();
  };
  if constexpr (B2) {
    for (int ct = 0; ct < NCT; ct += 2) {
      tile(ct, Ba);
      crt_load_b<KSMAX>(Ba, Bt, ct + 2, NCT, KS);
      if (ct + 1 < NCT) {
        tile(ct + 1, Bb);
        crt_load_b<KSMAX>(Bb, Bt, ct + 3, NCT, KS);
      }
    }
  } else {
    for (int ct = 0; ct < NCT; ++ct) {
      tile(ct, Ba);
      crt_load_b<KSMAX>(Ba, Bt, ct + 1, NCT, KS);
    }
  }
  if (owner) {
    // limbs above the last byte column: the carry's extension
    for (int L = 8 * NCT; L < Lc; ++L) {
      const uint32_t limb = (uint32_t)carry;
      carry >>= 32;
      O[l * sld + L] = limb;
      nz |= limb != 0u;
      last = limb;
    }
    if (row && (bad || carry != ((int32_t)last < 0 ? -1 : 0))) atomicOr(J.err, 1);
  }
  // one atomic per wave: the highest non-zero coefficient of the block
  const uint64_t any = __ballot(owner && row && nz);
  if (any && l == 0) atomicMax(J.deg_out, c0 + 63 - __clzll((long long)any));
  __syncthreads();
  // rows c0 .. c0 + nr - 1 are one contiguous range of nr Lc words
  const int nr = min(ROWS, J.degcap + 1 - c0);
  uint32_t* dst = J.out + (size_t)c0 * Lc;
  const int dq = 64 / Lc, dr = 64 - dq * Lc;
  int r = l / Lc, L = l - r * Lc;
  for (int i = l; i < nr * Lc; i += 64) {
    dst[i] = O[r * sld + L];
    r += dq;
    L += dr;
    if (L >= Lc) {
      L -= Lc;
      ++r;
    }
  }
}

// ---------------------------------------------------------------------------
// (a9) every stage after the reduction in one persistent launch of blocks of
// four waves, one stage after the other.  The tasks of a stage are claimed in
// chunks from counters: the blocks of XCD x (dispatch is round-robin over the
// eight XCDs in blockIdx order) claim from the x-th eighth of the stage's
// task range first, where the tasks of one (job, prime) share their residues
// and those of one prime its matrix planes in that XCD's L2, then from the
// other eighths.  A stage ends when its count of finished tasks reaches its
// total.  Only running blocks claim tasks and no task waits on anything, so
// the stages drain whichever blocks the device holds at once; a block that
// starts late finds the ranges taken.  Each task runs the staged kernel's
// device function on the same data; the residues come from the reduction's
// earlier launch, which keeps the scalar cache valid for the evaluation.  A
// wait that exceeds its time bound sets err and lets the block go on, so
// every wave exits.

#ifndef FUSED_WAIT_TICKS
#define FUSED_WAIT_TICKS 500000000ull  // 5 s of the 100 MHz wall clock
#endif

// A stage's counters (FUSED_STAGE_INTS ints): eight claim heads, then eight
// per-XCD counts of finished tasks, each in a 128-byte line of its own (the
// atomics on one line are serialised).
constexpr int FUSED_LINE = 32;
static_assert(FUSED_STAGE_INTS == 16 * FUSED_LINE, "counters of a stage");

// Claims the next chunk of at most K of a stage's T tasks for the calling
// wave (lane 0 claims for it): returns the first task and sets end, or -1
// once every range is taken.  Head x counts the tasks taken from range x,
// [T x / 8, T (x + 1) / 8); r walks the ranges starting from the wave's XCD.
// Another XCD's range is first read with a plain load, so that the waves
// that finish their own do not queue atomics on a range already taken.
__device__ __forceinline__ int fused_claim(int* ctr, int T, int K, int xcd, int& r, int& end) {
  while (r < 8) {
    const int x = (xcd + r) & 7;
    const int lo = (int)(((long long)T * x) >> 3), hi = (int)(((long long)T * (x + 1)) >> 3);
    int c = hi - lo;
    if (lane_id() == 0) {
      int* h = ctr + FUSED_LINE * x;
      if (r == 0 || __hip_atomic_load(h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < hi - lo)
        c = __hip_atomic_fetch_add(h, K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    c = __builtin_amdgcn_readfirstlane(c);
    if (c < hi - lo) {
      end = min(hi, lo + c + K);
      return lo + c;
    }
    ++r;
  }
  return -1;
}

// The same for the whole block (thread 0 claims; s_claim passes it on).
__device__ __forceinline__ int fused_claim_block(int* heads, int T, int K, int xcd, int& r, int& end,
                                                 int* s_claim) {
  __syncthreads();  // the previous claim has been read
  if (threadIdx.x == 0) {
    int e = 0;
    s_claim[0] = fused_claim(heads, T, K, xcd, r, e);
    s_claim[1] = e;
  }
  __syncthreads();
  end = s_claim[1];
  return s_claim[0];
}

// The end of a stage.  cnt: the calling wave's finished tasks (uniform in
// the wave, 0 outside the stage).  The block's count goes to its XCD's
// counter in one release by thread 0, after every wave's memory accesses
// have completed (an agent-scope release writes the XCD's L2 back, so one
// per block instead of one per wave); then that thread waits, with plain
// atomic loads (an acquire in the loop would invalidate the caches at every
// poll, under the feet of the blocks still working), until the eight
// counters add up to the stage's T tasks, and acquires once; the block
// barrier passes that on to the other waves.
__device__ __forceinline__ void fused_stage_end(const FusedPlan& F, int* ctr, int cnt, int T, int xcd, int* s_cnt) {
  if (lane_id() == 0 && cnt) atomicAdd(s_cnt, cnt);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int n = *s_cnt;
    *s_cnt = 0;
    if (n) __hip_atomic_fetch_add(ctr + FUSED_LINE * (8 + xcd), n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    for (;;) {
      int done = 0;
#pragma unroll
      for (int x = 0; x < 8; ++x)
        done += __hip_atomic_load(ctr + FUSED_LINE * (8 + x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (done >= T) break;
      __builtin_amdgcn_s_sleep(8);
      if (wall_clock64() - t0 > FUSED_WAIT_TICKS) {
        atomicOr(F.err, 2);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// C: register capacity of the evaluation's register Euclid (0: none);
// KSMAX: contraction steps of the CRT's left operand (P <= 8 KSMAX).  The
// register budget holds four waves per SIMD up to 48 primes.
template <int C, int KSMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KSMAX <= 8 ? 4 : 2, 8))) void k_fused(
    FusedPlan F, TablesDev tab) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int s_claim[2], s_cnt;
  // the wave's index is uniform across it (the compiler does not know that
  // threadIdx.x >> 6 is), so every task index below is a scalar
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = lane_id();
  const int xcd = blockIdx.x & 7;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  // (b)+(c) evaluation and elimination: wave tasks
  {
    int* c = F.ctr;
    const int T = F.n_rg + F.n_ee;
    int cnt = 0;
    if (w < F.wv[0]) {
      uint32_t* sl = lds + w * F.lw[0];
      int r = 0, e = 0;
      for (int t0 = fused_claim(c, T, F.kc[0], xcd, r, e); t0 >= 0; t0 = fused_claim(c, T, F.kc[0], xcd, r, e)) {
        for (int t = t0; t < e; ++t, ++cnt) {
          if (t < F.n_rg) {
            if constexpr (C > 0) {
              const int job = find_job(F.st_rg, F.nj, t, F.n_rg);
              const bool ok = dev_eval_elim_rg<C>(F.jobs[job], t - F.st_rg[job], tab, sl);
              if (__ballot(!ok) != 0ull && lane == 0) F.fb_queue[atomicAdd(F.fb_count, 1)] = t;
            }
          } else {
            const int u = t - F.n_rg;
            const int job = find_job(F.st_ee, F.nj, u, F.n_ee);
            dev_eval_elim<64, true>(F.jobs[job], u - F.st_ee[job], tab, sl);
          }
        }
      }
    }
    fused_stage_end(F, c, cnt, T, xcd, &s_cnt);
  }
  if constexpr (C > 0) {
    // the queued blocks, recomputed by the LDS kernel's function
    int* c = F.ctr + 1 * FUSED_STAGE_INTS;
    const int T = __hip_atomic_load(F.fb_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int cnt = 0;
    if (T > 0 && w < F.wv[1]) {
      uint32_t* sl = lds + w * F.lw[1];
      int r = 0, e = 0;
      for (int t0 = fused_claim(c, T, 1, xcd, r, e); t0 >= 0; t0 = fused_claim(c, T, 1, xcd, r, e)) {
        for (int i = t0; i < e; ++i, ++cnt) {
          const int b = __hip_atomic_load(F.fb_queue + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int job = find_job(F.st_rg, F.nj, b, F.n_rg);
          dev_eval_elim<64, true>(F.jobs[job], b - F.st_rg[job], tab, sl);
        }
      }
    }
    // (no queued block: every block reads the same count, no wait)
    if (T > 0) fused_stage_end(F, c, cnt, T, xcd, &s_cnt);
  }
  // (d) interpolation: block tasks, on the matrix cores for a group, else
  // per (job, prime)
  {
    int* c = F.ctr + 2 * FUSED_STAGE_INTS;
    const int T = F.im ? F.n_im : F.n_ip;
    InterpTab it;
    it.W = F.itW;
    it.Q = F.itQ;
    it.nb = F.itNB;
    int r = 0, e = 0, cnt = 0;
    for (int t0 = fused_claim_block(c, T, F.kc[2], xcd, r, e, s_claim); t0 >= 0;
         t0 = fused_claim_block(c, T, F.kc[2], xcd, r, e, s_claim)) {
      for (int b = t0; b < e; ++b, ++cnt) {
        if (F.im) {
          dev_interp_blk(F.gco, F.gN, F.gNp, F.gD, F.gDp, F.Ap, F.Yp, tab, b, (int8_t*)lds);
        } else {
          const int job = find_job(F.st_ip, F.nj, b, F.n_ip);
          dev_interp(F.jobs[job], b - F.st_ip[job], tab, lds, it);
        }
        __syncthreads();  // the next task refills the LDS read above
      }
    }
    // the block's count once (wave 0 holds it)
    fused_stage_end(F, c, w == 0 ? cnt : 0, T, xcd, &s_cnt);
  }
  // (e) reconstruction
  if (F.crt) {
    int* c = F.ctr + 3 * FUSED_STAGE_INTS;
    if (w < F.wv[2]) {
      uint32_t* sl = lds + w * F.lw[2];
      int r = 0, e = 0;
      for (int t0 = fused_claim(c, F.n_crt, F.kc[3], xcd, r, e); t0 >= 0;
           t0 = fused_claim(c, F.n_crt, F.kc[3], xcd, r, e))
        for (int t = t0; t < e; ++t)
          dev_crt<KSMAX, 1>(F.jobs, F.st_crt, F.nj, F.sld, F.cps, tab, t, F.n_crt, sl);
    }
    // the launch's end orders the results: no count, no wait
  } else {
    {
      int* c = F.ctr + 3 * FUSED_STAGE_INTS;
      int cnt = 0;
      if (w < F.wv[2]) {
        uint32_t* sl = lds + w * F.lw[2];
        int r = 0, e = 0;
        for (int t0 = fused_claim(c, F.n_mrc, F.kc[3], xcd, r, e); t0 >= 0;
             t0 = fused_claim(c, F.n_mrc, F.kc[3], xcd, r, e)) {
          for (int t = t0; t < e; ++t, ++cnt) {
            const int job = find_job(F.st_mrc, F.nj, t, F.n_mrc);
            dev_mrc_wave<true>(F.jobs[job], t - F.st_mrc[job], tab, sl);
          }
        }
      }
      fused_stage_end(F, c, cnt, F.n_mrc, xcd, &s_cnt);
    }
    {
      int* c = F.ctr + 4 * FUSED_STAGE_INTS;
      int r = 0, e = 0, cnt = 0;
      for (int t0 = fused_claim_block(c, F.n_sum, F.kc[4], xcd, r, e, s_claim); t0 >= 0;
           t0 = fused_claim_block(c, F.n_sum, F.kc[4], xcd, r, e, s_claim)) {
        for (int b = t0; b < e; ++b, ++cnt) {
          const int job = find_job(F.st_sum, F.nj, b, F.n_sum);
          dev_limbs_sum(F.jobs[job], b - F.st_sum[job], tab);
        }
      }
      fused_stage_end(F, c, w == 0 ? cnt : 0, F.n_sum, xcd, &s_cnt);
    }
    {
      int* c = F.ctr + 5 * FUSED_STAGE_INTS;
      if (w < F.wv[3]) {
        uint32_t* sl = lds + w * F.lw[3];
        int r = 0, e = 0;
        for (int t0 = fused_claim(c, F.n_car, F.kc[5], xcd, r, e); t0 >= 0;
             t0 = fused_claim(c, F.n_car, F.kc[5], xcd, r, e)) {
          for (int t = t0; t < e; ++t) {
            const int job = find_job(F.st_car, F.nj, t, F.n_car);
            dev_limbs_carry<true>(F.jobs[job], t - F.st_car[job], F.stage_ld, sl);
          }
        }
      }
    }
  }
}

#define BIRES_FUSED_KERNEL(C, KS)                                                             \
  ((C) == 24 ? ((KS) == 6 ? (const void*)k_fused<24, 6> : (const void*)k_fused<24, 16>)     \
   : (C) == 32 ? ((KS) == 6 ? (const void*)k_fused<32, 6> : (const void*)k_fused<32, 16>)   \
               : ((KS) == 6 ? (const void*)k_fused<0, 6> : (const void*)k_fused<0, 16>))

int fused_capacity(int c) { return c == 24 || c == 32 ? c : 0; }
int fused_crt_steps(int max_primes) { return max_primes <= 48 ? 6 : 16; }

int fused_blocks_per_cu(int C, int KS, size_t lds_bytes) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, BIRES_FUSED_KERNEL(C, KS), 256, lds_bytes) != hipSuccess)
    return 0;
  return per_cu;
}

void launch_fused(int C, int KS, const FusedPlan& F, size_t lds_bytes, int blocks, TablesDev tab, hipStream_t s) {
  void* args[] = {(void*)&F, (void*)&tab};
  (void)hipLaunchKernel(BIRES_FUSED_KERNEL(C, KS), dim3(blocks), dim3(256), args, lds_bytes, s);
}

// ---------------------------------------------------------------------------
// (a8) modular gcd per prime (Section 5.1, "Computing gcds in Z[x]", step (b)).
// One block per prime: Euclid's algorithm over F_p on a, b without inverses
// (each elimination A <- lc(B) A - lc(A) y^s B changes A only by a unit
// factor, so the last non-zero remainder is the gcd up to a unit); the result
// is made monic with one inverse.  Then waves 0 and 1 divide a and b exactly
// by the monic gcd (synthetic division, sequential over the quotient).
// Outputs are scaled for the integer reconstruction: beta g, (lc a / beta) a/g,
// (lc b / beta) b/g, whose images multiply to lc(a) a and lc(b) b.

// Euclid's algorithm over F_p on X (degree a) and Y (degree b) in LDS, run by
// the whole block, without inverses: each elimination X <- lc(Y) X - lc(X)
// y^s Y changes X only by a unit factor, so the last non-zero remainder is an
// associate of the gcd.  Leading coefficients must be non-zero.  Returns the
// gcd's degree d, with an associate of the gcd in Y[0..d] (the pointers are
// swapped as the roles alternate; both arrays need max(a, b) + 1 words).
__device__ int block_gcd_fp(uint32_t*& X, uint32_t*& Y, int a, int b, const ModP& q) {
  const int tid = threadIdx.x;
  if (a < b) {
    uint32_t* T = X; X = Y; Y = T;
    int t = a; a = b; b = t;
  }
  int d = 0;
  for (;;) {
    if (b == 0) {  // a non-zero constant divides both
      d = 0;
      break;
    }
    const uint32_t lb = Y[b];
    if (a == b + 1) {
      // the usual step: both eliminations in one pass, as in eliminate()
      // (X_t <- lb^2 X_t - lb X_a Y_{t-1} - X'_{a-1} Y_t with X'_{a-1} the
      // first elimination's new top coefficient)
      const uint32_t nla = mneg(X[a], q.p);
      const uint32_t n2 = mneg(mdot2(lb, X[a - 1], nla, Y[b - 1], q), q.p);
      const uint32_t l2 = mmul(lb, lb, q), l1 = mmul(lb, nla, q);
      __syncthreads();  // every thread has read X[a], X[a-1] before they can be overwritten below
      for (int t = tid; t < b; t += blockDim.x)
        X[t] = t ? mdot3(l2, X[t], l1, Y[t - 1], n2, Y[t], q) : mdot2(l2, X[0], n2, Y[0], q);
      __syncthreads();
    } else {
      for (int aa = a; aa >= b; --aa) {
        const uint32_t nla = mneg(X[aa], q.p);
        const int s = aa - b;
        __syncthreads();  // every thread has read X[aa] before it can be overwritten below
        for (int t = tid; t < aa; t += blockDim.x)
          X[t] = t < s ? mmul(lb, X[t], q) : mdot2(lb, X[t], nla, Y[t - s], q);
        __syncthreads();
      }
    }
    int c = b - 1;
    while (c >= 0 && X[c] == 0u) --c;
    if (c < 0) {
      d = b;
      break;
    }
    uint32_t* T = X; X = Y; Y = T;
    a = b;
    b = c;
  }
  return d;
}

__global__ __launch_bounds__(256) void k_gcd_p(GcdDev G, TablesDev tab) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int k = blockIdx.x;
  const ModP q = tab.primes[k];
  const int da = G.da, db = G.db;
  const int mx = da > db ? da : db;
  const int mn = da < db ? da : db;
  uint32_t* A0 = lds;
  uint32_t* B0 = A0 + da + 1;
  uint32_t* X = B0 + db + 1;
  uint32_t* Y = X + mx + 1;
  uint32_t* Gm = Y + mx + 1;
  const int tid = threadIdx.x;
  const uint32_t* ra = G.res_a + (size_t)k * (da + 1);
  const uint32_t* rb = G.res_b + (size_t)k * (db + 1);
  for (int i = tid; i <= da; i += blockDim.x) A0[i] = X[i] = ra[i];
  for (int i = tid; i <= db; i += blockDim.x) B0[i] = Y[i] = rb[i];
  __syncthreads();
  if (A0[da] == 0u || B0[db] == 0u) {
    if (tid == 0) G.gdeg[k] = -2;
    return;
  }
  const int d = block_gcd_fp(X, Y, da, db, q);
  // monic gcd (Montgomery) in Gm; b == 0 means gcd 1
  const uint32_t inv = d ? minv(Y[d], q) : q.one;
  for (int i = tid; i <= d; i += blockDim.x) Gm[i] = d ? mmul(Y[i], inv, q) : q.one;
  __syncthreads();
  const uint32_t beta = G.sc[3 * k], sa = G.sc[3 * k + 1], sb = G.sc[3 * k + 2];
  uint32_t* F = G.F + (size_t)k * (mn + 1);
  for (int i = tid; i <= mn; i += blockDim.x) F[i] = i <= d ? mmul(Gm[i], beta, q) : 0u;
  // cofactors: wave 0 divides a, wave 1 divides b (in X and Y as work arrays)
  const int wave = tid >> 6, lane = tid & 63;
  __shared__ int bad_any;
  if (tid == 0) bad_any = 0;
  __syncthreads();
  if (wave < 2) {
    const int dn = wave ? db : da;
    const uint32_t* src = wave ? B0 : A0;
    uint32_t* W = wave ? Y : X;
    uint32_t* out = wave ? G.QB + (size_t)k * (db + 1) : G.QA + (size_t)k * (da + 1);
    const uint32_t scl = wave ? sb : sa;
    for (int i = lane; i <= dn; i += 64) W[i] = src[i];
    bool bad = false;
    for (int kq = dn - d; kq >= 0; --kq) {
      const uint32_t qc = W[kq + d];
      for (int i = lane; i < d; i += 64) W[kq + i] = msub(W[kq + i], mmul(qc, Gm[i], q), q.p);
      if (lane == 0) out[kq] = mmul(qc, scl, q);
    }
    for (int i = lane; i < d; i += 64) bad |= W[i] != 0u;
    for (int i = dn - d + 1 + lane; i <= dn; i += 64) out[i] = 0u;
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(&bad_any, 1);
  }
  __syncthreads();
  if (tid == 0) G.gdeg[k] = bad_any ? -3 : d;
}

// ---------------------------------------------------------------------------
// The degree chain of the N^- / N^+ test (Section 3.2.2) over F_p, one block:
//   S_0 = R* mod p, S_i = gcd(S_{i-1}, sr_i) (i >= 1, until S_i is constant),
//   and deg gcd(R^inf, Q) = the degrees of the gcds removed from Q by
//   H <- H / gcd(H, R*) until that gcd is constant.
// Inputs in Montgomery form or plain as stated; every gcd is block_gcd_fp.

// Degree of v[0..n) (-1 for zero), computed by the block.
__device__ int block_degree(const uint32_t* v, int n, int* red) {
  int top = -1;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (v[i] != 0u) top = i;
  __syncthreads();
  if (threadIdx.x == 0) *red = -1;
  __syncthreads();
  if (top >= 0) atomicMax(red, top);
  __syncthreads();
  const int d = *red;
  __syncthreads();
  return d;
}

__global__ __launch_bounds__(256) void k_fiber_chain(ChainDev C, TablesDev tab) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int red;
  const ModP q = tab.primes[0];
  const int tid = threadIdx.x;
  const int mx = max(max(C.dr + 1, C.D), C.Dq);
  uint32_t* S = lds;            // current S_i, then R* for the common part
  uint32_t* X = S + mx;
  uint32_t* Y = X + mx;
  uint32_t* H = Y + mx;         // Q / (removed gcds)
  for (int i = tid; i < mx; i += blockDim.x) S[i] = i <= C.dr ? C.rstar[i] : 0u;
  int ds = block_degree(S, C.dr + 1, &red);
  const int d0 = ds;
  if (tid == 0) C.out[0] = ds;
  int i = 1;
  for (; i < C.K && ds >= 1; ++i) {
    const uint32_t* sr = C.srs + (size_t)i * C.D;
    for (int t = tid; t < C.D; t += blockDim.x) Y[t] = to_mont(sr[t], q);
    const int db = block_degree(Y, C.D, &red);
    if (db >= 0) {  // gcd(S, 0) = S
      for (int t = tid; t <= ds; t += blockDim.x) X[t] = S[t];
      __syncthreads();
      uint32_t* Xp = X;
      uint32_t* Yp = Y;
      const int d = block_gcd_fp(Xp, Yp, ds, db, q);
      __syncthreads();
      for (int t = tid; t <= d; t += blockDim.x) S[t] = Yp[t];
      ds = d;
      __syncthreads();
    }
    if (tid == 0) C.out[i] = ds;
  }
  for (; i < C.K; ++i)
    if (tid == 0) C.out[i] = 0;
  // the common part of R and Q with Q's multiplicities
  for (int t = tid; t < mx; t += blockDim.x) {
    S[t] = t <= C.dr ? C.rstar[t] : 0u;
    H[t] = t < C.Dq ? to_mont(C.qpol[t], q) : 0u;
  }
  int dh = block_degree(H, C.Dq, &red);
  int total = 0;
  while (dh >= 1 && d0 >= 1) {
    for (int t = tid; t <= dh; t += blockDim.x) X[t] = H[t];
    for (int t = tid; t <= d0; t += blockDim.x) Y[t] = S[t];
    __syncthreads();
    uint32_t* Xp = X;
    uint32_t* Yp = Y;
    const int d = block_gcd_fp(Xp, Yp, dh, d0, q);
    __syncthreads();
    if (d == 0) break;
    total += d;
    // H <- H / G (G = Yp[0..d], made monic), wave 0 by synthetic division
    const uint32_t inv = minv(Yp[d], q);
    for (int t = tid; t <= d; t += blockDim.x) Yp[t] = mmul(Yp[t], inv, q);
    __syncthreads();
    if (tid < 64) {
      for (int kq = dh - d; kq >= 0; --kq) {
        const uint32_t qc = H[kq + d];
        for (int t = tid; t < d; t += 64) H[kq + t] = msub(H[kq + t], mmul(qc, Yp[t], q), q.p);
        if (tid == 0) Xp[kq] = qc;  // the quotient (Xp is free again)
      }
    }
    __syncthreads();
    dh -= d;
    for (int t = tid; t < mx; t += blockDim.x) H[t] = t <= dh ? Xp[t] : 0u;
    __syncthreads();
  }
  if (tid == 0) {
    C.out[C.K] = total;
    C.out[C.K + 1] = dh < 0 ? 1 : 0;
  }
}

size_t fiber_chain_lds_bytes(int dr, int D, int Dq) {
  int mx = dr + 1 > D ? dr + 1 : D;
  if (Dq > mx) mx = Dq;
  return (size_t)4 * mx * sizeof(uint32_t);
}

void launch_fiber_chain(const ChainDev& C, TablesDev tab, hipStream_t s) {
  hipLaunchKernelGGL(k_fiber_chain, dim3(1), dim3(256), fiber_chain_lds_bytes(C.dr, C.D, C.Dq), s, C, tab);
}

size_t gcd_lds_bytes(int da, int db) {
  const int mx = da > db ? da : db, mn = da < db ? da : db;
  return (size_t)(da + db + 2 + 2 * (mx + 1) + mn + 1) * sizeof(uint32_t);
}

void launch_gcd_p(const GcdDev& g, TablesDev tab, hipStream_t s) {
  hipLaunchKernelGGL(k_gcd_p, dim3(g.P), dim3(256), gcd_lds_bytes(g.da, g.db), s, g, tab);
}

// dst[r][0..n) = src[idx[r]][0..n) (row stride of src: ld words)
__global__ void k_gather_rows(const uint32_t* src, int ld, const int* idx, int rows, int n, uint32_t* dst) {
  const int r = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows || c >= n) return;
  dst[(size_t)r * n + c] = src[(size_t)idx[r] * ld + c];
}

void launch_gather_rows(const uint32_t* src, int ld, const int* idx, int rows, int n, uint32_t* dst, hipStream_t s) {
  if (rows <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((n + 255) / 256, rows), dim3(256), 0, s, src, ld, idx, rows, n, dst);
}

// ---------------------------------------------------------------------------
// launchers

// Issue-rate probe for the roofline: every lane runs 16 independent chains
// of one VALU instruction (inline assembly, so the compiler can neither fold
// nor reorder them), or for K = 5 sixteen int8 matrix-core products
// v_mfma_i32_32x32x32_i8 per round over four independent accumulators; the
// host divides the SIMD-cycles of the launch by the wave instructions
// issued.  Writes one word per thread.
template <int K>
__global__ __launch_bounds__(256) void k_issue_rate(uint32_t* out, uint32_t s, int iters) {
  if constexpr (K == 5) {
    const im_v4i x = {(int)(threadIdx.x * 0x01010101u), (int)s, 3, -5}, y = {7, (int)threadIdx.x, -1, 9};
    im_v16i c0 = {0}, c1 = {0}, c2 = {0}, c3 = {0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, y, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(y, x, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, x, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(y, y, c3, 0, 0, 0);
      }
    }
    uint32_t r = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) r += (uint32_t)(c0[e] ^ c1[e] ^ c2[e] ^ c3[e]);
    out[blockIdx.x * 256 + threadIdx.x] = r;
    return;
  }
  uint32_t a[16];
  uint64_t w[16];
  double f[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = threadIdx.x + c;
    w[c] = threadIdx.x * 3u + c;
    f[c] = threadIdx.x + c * 0.5;
  }
  const uint32_t b = s ^ threadIdx.x;
  const double fb = 0.999 + threadIdx.x * 1e-9;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if constexpr (K == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
      if constexpr (K == 1) asm volatile("v_min_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
      if constexpr (K == 2) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
      if constexpr (K == 3) {
        uint64_t cy;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[c]), "=s"(cy) : "v"(a[c]), "v"(b));
      }
      if constexpr (K == 4) asm volatile("v_fma_f64 %0, %0, %1, 1.0" : "+v"(f[c]) : "v"(fb));
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) r += a[c] + (uint32_t)w[c] + (uint32_t)f[c];
  out[blockIdx.x * 256 + threadIdx.x] = r;
}

void launch_issue_rate(int kind, uint32_t* out, int blocks, int iters, hipStream_t s) {
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_issue_rate<0>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
    case 1: hipLaunchKernelGGL(k_issue_rate<1>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
    case 2: hipLaunchKernelGGL(k_issue_rate<2>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
    case 3: hipLaunchKernelGGL(k_issue_rate<3>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
    case 4: hipLaunchKernelGGL(k_issue_rate<4>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
    default: hipLaunchKernelGGL(k_issue_rate<5>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
  }
}

// Word-by-word comparison of the row statistics a call's scan produced with
// the ones its reused plans were made from; any difference sets *flag.
__global__ __launch_bounds__(256) void k_stats_check(const int32_t* got, const int32_t* want, long long n,
                                                     int* flag) {
  bool diff = false;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    diff |= got[i] != want[i];
  if (__ballot(diff) != 0ull && (threadIdx.x & 63) == 0) *flag = 1;
}

// Word copy from pinned host memory, read through its device mapping, to
// device memory: the call's metadata upload as a kernel on the compute queue
// (no hand-off to a copy engine between two kernels of the same call).
__global__ __launch_bounds__(256) void k_upload(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void launch_upload(const uint32_t* src_mapped, uint32_t* dst, long long words, hipStream_t s) {
  const long long blocks = std::min<long long>((words + 255) / 256, 256);
  if (blocks > 0) hipLaunchKernelGGL(k_upload, dim3((unsigned)blocks), dim3(256), 0, s, src_mapped, dst, words);
}

void launch_stats_check(const int32_t* got, const int32_t* want, long long n, int* flag, hipStream_t s) {
  const long long blocks = std::min<long long>((n + 255) / 256, 1024);
  if (blocks > 0) hipLaunchKernelGGL(k_stats_check, dim3((unsigned)blocks), dim3(256), 0, s, got, want, n, flag);
}

void launch_scan(const ScanTask* tasks, const int4* bmap, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(nblocks), dim3(64), 0, s, tasks, bmap);
}

void launch_transpose(const uint32_t* src, uint32_t* dst, int rows, int cols, int L, hipStream_t s) {
  size_t total = (size_t)rows * cols * L;
  if (!total) return;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, rows, cols, L);
}

void launch_reduce(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_primes, TablesDev tab,
                   hipStream_t s) {
  dim3 grid(nblocks, (max_primes + KT - 1) / KT);
  hipLaunchKernelGGL(k_reduce, grid, dim3(64), 0, s, jobs, starts, nj, tab);
}

int eval_elim_block() { return 64; }

size_t eval_elim_lds_bytes(int words, int res) {
  (void)res;  // residues are read through the scalar cache
  return (size_t)words * 64 * sizeof(uint32_t);
}

void launch_eval_elim(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_words, int max_res,
                      TablesDev tab, hipStream_t s) {
  hipLaunchKernelGGL(k_eval_elim<64>, dim3(nblocks), dim3(64), eval_elim_lds_bytes(max_words, max_res), s, jobs,
                     starts, nj, tab);
}

int eval_elim_rg_capacity(int m, int n) {
  if (m < 1 || n < 1) return 0;
  const int d = std::max(m, n);
  return d < 24 ? 24 : d < 32 ? 32 : d < 64 ? 64 : 0;
}

void launch_eval_elim_rg(int C, const JobDev* jobs, const int* starts, int nj, int nblocks, int max_deg,
                         int max_words, int* fb_count, int* fb_queue, TablesDev tab, hipStream_t s) {
  const size_t lds = (size_t)(max_deg + 1) * 64 * sizeof(uint32_t);
  if (C == 24)
    hipLaunchKernelGGL(k_eval_elim_rg24, dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, tab, fb_count, fb_queue);
  else if (C == 32)
    hipLaunchKernelGGL(k_eval_elim_rg32, dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, tab, fb_count, fb_queue);
  else
    hipLaunchKernelGGL(k_eval_elim_rg64, dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, tab, fb_count, fb_queue);
  hipLaunchKernelGGL(k_eval_elim_fb, dim3(std::min(nblocks, 256)), dim3(64), eval_elim_lds_bytes(max_words, 0), s,
                     jobs, starts, nj, tab, fb_count, fb_queue);
}

int schur_rows_per_lane(int m, int n) {
  if (m < 1 || n < 1) return 0;
  return m + n <= 64 ? 1 : m + n <= 128 ? 2 : 0;
}

void launch_schur(int NR, const JobDev* jobs, const int* starts, int nj, int nblocks, int max_words, int* fallbacks,
                  TablesDev tab, hipStream_t s) {
  const size_t lds = (size_t)max_words * sizeof(uint32_t);
  if (NR == 1)
    hipLaunchKernelGGL(k_schur<1>, dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, tab, fallbacks);
  else
    hipLaunchKernelGGL(k_schur<2>, dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, tab, fallbacks);
}

void launch_interp(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_points, TablesDev tab,
                   const uint32_t* W, const uint32_t* Q, int tab_blocks, hipStream_t s) {
  size_t lds = interp_lds_words(max_points) * sizeof(uint32_t);
  InterpTab it;
  it.W = W;
  it.Q = Q;
  it.nb = tab_blocks;
  hipLaunchKernelGGL(k_interp, dim3(nblocks), dim3(256), lds, s, jobs, starts, nj, tab, it);
}

int interp_table_blocks(int max_points) { return (max_points + KB - 1) / KB; }

size_t interp_table_words(int blocks, int primes, size_t* q_offset) {
  *q_offset = (size_t)primes * blocks * KB * KB;
  return *q_offset + (size_t)primes * blocks * (KB + 1);
}

void launch_interp_tables(int blocks, int primes, TablesDev tab, uint32_t* W, uint32_t* Q, hipStream_t s) {
  hipLaunchKernelGGL(k_interp_tables, dim3(blocks, primes), dim3(64), 0, s, blocks, tab, W, Q);
}

size_t vinv_bytes(int Dp, int P) { return (size_t)4 * Dp * Dp * P; }

void launch_vinv(int D, int Dp, int P, TablesDev tab, int8_t* Ap, hipStream_t s) {
  hipLaunchKernelGGL(k_vinv, dim3(P), dim3(256), (size_t)2 * (D + 1) * sizeof(uint32_t), s, D, Dp, tab, Ap);
}

void launch_interp_mfma(uint32_t* const* gco, int N, int D, int P, const int8_t* Ap, const int8_t* Yp, TablesDev tab,
                        hipStream_t s) {
  const int Dp = (D + 31) & ~31, Np = (N + 31) & ~31;
  const int nbr = (Dp / 32 + 1) / 2, nbc = (Np / 32 + 1) / 2;
  hipLaunchKernelGGL(k_interp_mfma, dim3(nbr * nbc * P), dim3(256), interp_mfma_lds_bytes(), s, gco, N, Np, D, Dp,
                     Ap, Yp, tab);
}

void launch_mrc(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_primes, TablesDev tab,
                hipStream_t s) {
  hipLaunchKernelGGL(k_mrc, dim3(nblocks), dim3(64), (size_t)2 * max_primes * sizeof(uint32_t), s, jobs, starts, nj,
                     tab);
}

bool crt_ok(int max_primes) { return max_primes <= CRT_MAXP; }

int crt_row_stride(int max_lcap) { return max_lcap | 1; }

// Stride of the per-prime constants (even, so that the doubles stay aligned)
// and the words of M for a prime count (M < 2^(32 P) has at most P words),
// rounded up to whole column tiles, both sized by the batch's largest prime
// count rather than CRT_MAXP, which keeps the blocks small.
int crt_const_stride(int max_primes) { return (max_primes + 1) & ~1; }
static int crt_max_words(int max_primes) { return 8 * ((4 * (max_primes + 1) + 4 + 31) / 32); }

// Coefficients per block: two row tiles while the left operands of both fit
// in registers (up to 48 primes), one above.
int crt_rows_per_block(int max_primes) { return max_primes <= 48 ? 64 : 32; }

size_t crt_lds_bytes_rows(int max_lcap, int max_primes, int R) {
  // accumulator tiles, limb rows (an even word count), prime constants
  const size_t rows = (size_t)R * crt_row_stride(max_lcap);
  return (size_t)(R * 33 + rows + 5 * crt_const_stride(max_primes) + crt_max_words(max_primes)) * sizeof(uint32_t);
}

size_t crt_lds_bytes(int max_lcap, int max_primes) {
  return crt_lds_bytes_rows(max_lcap, max_primes, crt_rows_per_block(max_primes));
}

void launch_crt(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_primes, int max_lcap,
                TablesDev tab, hipStream_t s) {
  const int sld = crt_row_stride(max_lcap);
  const int cps = crt_const_stride(max_primes);
  const size_t lds = crt_lds_bytes(max_lcap, max_primes);
  const int ks = (max_primes + 7) / 8;
#define BIRES_CRT_LAUNCH(K, NT) \
  hipLaunchKernelGGL((k_crt_mfma<K, NT>), dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, sld, cps, tab)
  // two row tiles exactly when crt_rows_per_block(max_primes) is 64 (ks <= 6)
  if (ks <= 2)
    BIRES_CRT_LAUNCH(2, 2);
  else if (ks <= 4)
    BIRES_CRT_LAUNCH(4, 2);
  else if (ks <= 6)
    BIRES_CRT_LAUNCH(6, 2);
  else if (ks <= 8)
    BIRES_CRT_LAUNCH(8, 1);
  else if (ks <= 12)
    BIRES_CRT_LAUNCH(12, 1);
  else
    BIRES_CRT_LAUNCH(16, 1);
#undef BIRES_CRT_LAUNCH
}

void launch_limbs_sum(const JobDev* jobs, const int* starts, int nj, int nblocks, TablesDev tab, hipStream_t s) {
  hipLaunchKernelGGL(k_limbs_sum, dim3(nblocks), dim3(256), 0, s, jobs, starts, nj, tab);
}

void launch_limbs_carry(const JobDev* jobs, const int* starts, int nj, int nblocks, int max_lcap, hipStream_t s) {
  const int stage_ld = max_lcap <= CARRY_STAGE_MAXL ? max_lcap + 1 : 0;
  const size_t lds = (size_t)64 * stage_ld * sizeof(uint32_t);
  hipLaunchKernelGGL(k_limbs_carry, dim3(nblocks), dim3(64), lds, s, jobs, starts, nj, stage_ld);
}

}  // namespace bires
