// HIP kernels (gfx950) of the multi-modular resultant: the steps (a)-(e) of
// Collins' scheme as summarised in Section 5.1 ("Computing resultants in
// Z[x,y]"), all on the device.
//
//   k_scan        per-row degree / bit-length statistics of an input (planning)
//   k_transpose   exchange x and y in a limb rectangle (res_x, disc_x)
//   k_reduce      (a) coefficients modulo each prime, Montgomery form
//   k_eval_elim   (b)+(c) evaluate at x = a and take the univariate resultant
//                 over F_p, one lane per (prime, point)
//   k_interp      (d) Newton interpolation per prime, nodes a = 0..D-1
//   k_mrc         (e) mixed-radix (Garner) digits per coefficient
//   k_limbs_sum / k_limbs_carry   (e) digits -> two's-complement limbs
//
// Every kernel is batch-native: a block map (int4 per block) names the job and
// the slice of it the block works on, so a single job is a batch of one.
#include <hip/hip_runtime.h>

#include "job.hpp"
#include "kernels.hpp"

namespace bires {

// ---------------------------------------------------------------------------
// planning statistics: for each row j of a rectangle, the x-degree, the
// largest bit length of |c| and the number of non-zero coefficients.

__global__ void k_scan(const ScanTask* tasks, const int4* bmap) {
  int4 bm = bmap[blockIdx.x];
  const ScanTask& T = tasks[bm.x];
  int j = bm.y + threadIdx.x;
  if (j >= T.rows) return;
  int deg = -1, bits = 0, cnt = 0;
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
    }
  }
  T.out[3 * j + 0] = deg;
  T.out[3 * j + 1] = bits;
  T.out[3 * j + 2] = cnt;
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
// (a) reduction modulo the primes.  Block map: x = job, y = 0 (f) / 1 (g),
// z = first coefficient; blockIdx.y selects a tile of KT primes.  A coefficient
// with limbs w_0..w_{L-1} (two's complement) has value sum w_l 2^{32l} - s 2^{32L};
// its Montgomery residue is built by Horner over the limbs with one two-product
// reduction per limb, then the sign term (R^L)_M is subtracted.

constexpr int KT = 16;

__global__ void k_reduce(const JobDev* jobs, const int4* bmap, TablesDev tab) {
  int4 bm = bmap[blockIdx.x];
  const JobDev& J = jobs[bm.x];
  const bool isg = bm.y != 0;
  const int T = isg ? J.Tg : J.Tf;
  const int t = bm.z + threadIdx.x;
  const int k0 = blockIdx.y * KT;
  if (t >= T || k0 >= J.P) return;
  const uint32_t* src;
  int L;
  uint32_t mult = 0;  // 0: none; else the derivative factor j+1
  if (!isg) {
    src = J.limbs_f + (size_t)t * J.Lf;
    L = J.Lf;
  } else if (J.disc) {
    int j = t / J.ldf;
    src = J.limbs_f + (size_t)(t + J.ldf) * J.Lf;  // coefficient (j+1, i) of f
    L = J.Lf;
    mult = (uint32_t)(j + 1);
  } else {
    src = J.limbs_g + (size_t)t * J.Lg;
    L = J.Lg;
  }
  const bool negv = (src[L - 1] >> 31) != 0u;
  uint32_t* dst = (isg ? J.res_g : J.res_f) + t;
  const int k1 = min(J.P, k0 + KT);
  for (int k = k0; k < k1; ++k) {
    const ModP q = tab.primes[k];
    uint32_t x = 0;
    for (int l = L - 1; l >= 0; --l) x = mdot2(x, q.r2, reduce32(src[l], q.p), q.r2, q);
    if (negv) x = msub(x, mpow(q.r2, (uint32_t)L, q), q.p);
    if (mult) x = mmul(x, to_mont(mult, q), q);
    dst[(size_t)k * T] = x;
  }
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
  for (;;) {
    if (b == 0) {
      num = mmul(num, mpow(B[0], (uint32_t)a, q), q);
      break;
    }
    const uint32_t lb = B[b * W];
    const int a0 = a;
    int kk = 0;
    while (a >= b) {
      const uint32_t nla = mneg(A[a * W], q.p);
      const int s = a - b;
      for (int t = 0; t < s; ++t) A[t * W] = mmul(lb, A[t * W], q);
      for (int t = s; t < a; ++t) A[t * W] = mdot2(lb, A[t * W], nla, B[(t - s) * W], q);
      --a;
      ++kk;
      while (a >= 0 && A[a * W] == 0u) --a;
    }
    if (a < 0) return 0u;
    neg ^= ((a0 * b) & 1) != 0;
    const int e = a0 - a - kk * b;
    if (e > 0) num = mmul(num, mpow(lb, (uint32_t)e, q), q);
    else if (e < 0) den = mmul(den, mpow(lb, (uint32_t)(-e), q), q);
    uint32_t* T = A; A = B; B = T;
    int t = a; a = b; b = t;
  }
  uint32_t r = (den == q.one) ? num : mmul(num, minv(den, q), q);
  return neg ? mneg(r, q.p) : r;
}

// (b)+(c): block map x = job, y = prime index k, z = first point; one lane per
// point a = z + lane.  The prime is uniform over the block, so its constants
// and the residue rows are scalar loads.
template <int W>
__global__ __launch_bounds__(W) void k_eval_elim(const JobDev* jobs, const int4* bmap, TablesDev tab) {
  extern __shared__ uint32_t lds[];
  const int4 bm = bmap[blockIdx.x];
  const JobDev& J = jobs[bm.x];
  const int k = bm.y;
  const int pt = bm.z + (int)threadIdx.x;
  if (pt >= J.D) return;
  const ModP q = tab.primes[k];
  uint32_t* A = lds + threadIdx.x;
  uint32_t* B = A + (J.m + 1) * W;
  const uint32_t aM = to_mont((uint32_t)pt, q);
  const uint32_t* rf = J.res_f + (size_t)k * J.Tf;
  for (int j = 0; j <= J.m; ++j) {
    const uint32_t* row = rf + j * J.ldf;
    uint32_t acc = 0;
    for (int i = J.rowdeg_f[j]; i >= 0; --i) acc = madd(mmul(acc, aM, q), row[i], q.p);
    A[j * W] = acc;
  }
  const uint32_t* rg = J.res_g + (size_t)k * J.Tg;
  const int ldg = J.disc ? J.ldf : J.ldg;
  for (int j = 0; j <= J.n; ++j) {
    const uint32_t* row = rg + j * ldg;
    uint32_t acc = 0;
    for (int i = J.rowdeg_g[j]; i >= 0; --i) acc = madd(mmul(acc, aM, q), row[i], q.p);
    B[j * W] = acc;
  }
  const uint32_t r = uni_resultant<W>(A, B, J.m, J.n, q);
  J.vals[(size_t)k * J.D + pt] = from_mont(r, q);
}

// ---------------------------------------------------------------------------
// (d) interpolation per prime.  Nodes a_i = i, so the divided differences are
// c_j <- (c_j - c_{j-1}) / s at stage s; then the Newton form
// sum_s c_s prod_{t<s} (x - t) is expanded by Horner from the top:
// P <- P (x - s) + c_s.  Block map: x = job, y = prime index.

__global__ __launch_bounds__(256) void k_interp(const JobDev* jobs, const int4* bmap, TablesDev tab) {
  extern __shared__ uint32_t lds[];
  const int4 bm = bmap[blockIdx.x];
  const JobDev& J = jobs[bm.x];
  const int k = bm.y;
  const int D = J.D;
  const ModP q = tab.primes[k];
  uint32_t* c0 = lds;
  uint32_t* c1 = lds + D;
  uint32_t* inv = lds + 2 * D;  // Montgomery form of 1/s
  const uint32_t* v = J.vals + (size_t)k * D;
  for (int j = threadIdx.x; j < D; j += blockDim.x) {
    c0[j] = v[j];
    inv[j] = j ? minv(to_mont((uint32_t)j, q), q) : 0u;
  }
  __syncthreads();
  for (int s = 1; s < D; ++s) {
    const uint32_t is = inv[s];
    for (int j = threadIdx.x; j < D; j += blockDim.x)
      c1[j] = j >= s ? mmul(msub(c0[j], c0[j - 1], q.p), is, q) : c0[j];
    __syncthreads();
    uint32_t* t = c0; c0 = c1; c1 = t;
  }
  // c0 holds the Newton coefficients; expand into c1 (then ping-pong), keeping
  // the Newton coefficients in inv[] (no longer needed as inverses).
  for (int j = threadIdx.x; j < D; j += blockDim.x) {
    inv[j] = c0[j];
    c1[j] = j == 0 ? c0[D - 1] : 0u;
  }
  __syncthreads();
  uint32_t* a0 = c1;
  uint32_t* a1 = c0;
  for (int s = D - 2; s >= 0; --s) {
    const uint32_t sM = to_mont((uint32_t)s, q);
    const uint32_t cs = inv[s];
    for (int j = threadIdx.x; j < D; j += blockDim.x) {
      uint32_t x = msub(j ? a0[j - 1] : 0u, mmul(a0[j], sM, q), q.p);
      a1[j] = j ? x : madd(x, cs, q.p);
    }
    __syncthreads();
    uint32_t* t = a0; a0 = a1; a1 = t;
  }
  uint32_t* out = J.coefs + (size_t)k * D;
  for (int j = threadIdx.x; j < D; j += blockDim.x) out[j] = a0[j];
}

// ---------------------------------------------------------------------------
// (e) mixed-radix conversion (Garner).  With primes p_0 > p_1 > ... the value
// is sum_j v_j prod_{i<j} p_i, v_j in [0, p_j).  Lane k keeps
// acc_k = sum_{j<k} v_j prod_{i<j} p_i mod p_k; when j reaches k,
// v_k = (x_k - acc_k) (prod_{i<k} p_i)^{-1} mod p_k.  One wave per coefficient;
// lanes cover primes k = lane + 64 t.  The symmetric lift is negative exactly
// when the digit vector exceeds ((p_k - 1)/2)_k lexicographically from the top,
// because sum_k (p_k - 1)/2 prod_{i<k} p_i = (M - 1)/2.

__global__ __launch_bounds__(64) void k_mrc(const JobDev* jobs, const int4* bmap, TablesDev tab) {
  extern __shared__ uint32_t lds[];
  const int4 bm = bmap[blockIdx.x];
  const JobDev& J = jobs[bm.x];
  const int c = bm.y;
  const int P = J.P;
  const int lane = threadIdx.x;
  uint32_t* x = lds;        // residues, then digits
  uint32_t* acc = lds + P;  // running prefix values
  for (int kk = lane; kk < P; kk += 64) {
    x[kk] = J.coefs[(size_t)kk * J.D + c];
    acc[kk] = 0u;
  }
  uint32_t* dig = J.digits + (size_t)c * P;
  for (int j = 0; j < P; ++j) {
    const int owner = j & 63;
    uint32_t v = 0;
    if (lane == owner) {
      const ModP qj = tab.primes[j];
      v = mmul(msub(x[j], acc[j], qj.p), tab.cm[j], qj);
      x[j] = v;
      dig[j] = v;
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
  __syncthreads();
  if (lane == 0) {
    int neg = 0;
    for (int kk = P - 1; kk >= 0; --kk) {
      const uint32_t h = (tab.primes[kk].p - 1u) >> 1;
      if (x[kk] != h) {
        neg = x[kk] > h ? 1 : 0;
        break;
      }
    }
    J.negflag[c] = neg;
  }
}

// (e) limb assembly, pass 1: one thread per (coefficient, limb l) forms the
// 96-bit column sum S_l = sum_k d_k limb_l(prod_{i<k} p_i), with d_k the digit
// (non-negative lift) or p_k - 1 - digit (negative lift: then
// M - v - 1 = sum (p_k - 1 - v_k) prod_{i<k} p_i).  Block map: x = job,
// z = first flat index c * Lacc + l.
__global__ void k_limbs_sum(const JobDev* jobs, const int4* bmap, TablesDev tab) {
  const int4 bm = bmap[blockIdx.x];
  const JobDev& J = jobs[bm.x];
  const int idx = bm.z + threadIdx.x;
  if (idx >= J.D * J.Lacc) return;
  const int c = idx / J.Lacc;
  const int l = idx - c * J.Lacc;
  const int neg = J.negflag[c];
  const uint32_t* dig = J.digits + (size_t)c * J.P;
  uint64_t lo = 0;
  uint32_t hi = 0;
  for (int k = l; k < J.P; ++k) {
    uint32_t d = dig[k];
    if (neg) d = tab.primes[k].p - 1u - d;
    const uint64_t prod = (uint64_t)d * tab.pi[(size_t)k * (k + 1) / 2 + l];
    lo += prod;
    hi += (lo < prod) ? 1u : 0u;
  }
  J.acc_lo[idx] = lo;
  J.acc_hi[idx] = hi;
}

// (e) limb assembly, pass 2: one thread per output coefficient propagates the
// carries; a negative lift writes the bitwise complement (two's complement of
// -(C + 1) is ~C).  Overflow of the caller's limb count sets err.
__global__ void k_limbs_carry(const JobDev* jobs, const int4* bmap) {
  const int4 bm = bmap[blockIdx.x];
  const JobDev& J = jobs[bm.x];
  const int c = bm.z + threadIdx.x;
  if (c > J.degcap) return;
  uint32_t* o = J.out + (size_t)c * J.Lcap;
  if (c >= J.D) {
    for (int l = 0; l < J.Lcap; ++l) o[l] = 0u;
    return;
  }
  const int neg = J.negflag[c];
  const uint32_t flip = neg ? 0xFFFFFFFFu : 0u;
  uint64_t carry = 0;  // < 2^50
  bool nz = neg != 0;
  uint32_t last = 0;
  for (int l = 0; l < J.Lcap; ++l) {
    uint64_t lo = 0;
    uint32_t hi = 0;
    if (l < J.Lacc) {
      lo = J.acc_lo[(size_t)c * J.Lacc + l];
      hi = J.acc_hi[(size_t)c * J.Lacc + l];
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
  if (nz) atomicMax(J.deg_out, c);
}

// ---------------------------------------------------------------------------
// launchers

void launch_scan(const ScanTask* tasks, const int4* bmap, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(nblocks), dim3(64), 0, s, tasks, bmap);
}

void launch_transpose(const uint32_t* src, uint32_t* dst, int rows, int cols, int L, hipStream_t s) {
  size_t total = (size_t)rows * cols * L;
  if (!total) return;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, rows, cols, L);
}

void launch_reduce(const JobDev* jobs, const int4* bmap, int nblocks, int max_primes, TablesDev tab,
                   hipStream_t s) {
  dim3 grid(nblocks, (max_primes + KT - 1) / KT);
  hipLaunchKernelGGL(k_reduce, grid, dim3(64), 0, s, jobs, bmap, tab);
}

int eval_elim_block() { return 64; }

void launch_eval_elim(const JobDev* jobs, const int4* bmap, int nblocks, int max_words, TablesDev tab,
                      hipStream_t s) {
  size_t lds = (size_t)max_words * 64 * sizeof(uint32_t);
  hipLaunchKernelGGL(k_eval_elim<64>, dim3(nblocks), dim3(64), lds, s, jobs, bmap, tab);
}

void launch_interp(const JobDev* jobs, const int4* bmap, int nblocks, int max_points, TablesDev tab,
                   hipStream_t s) {
  size_t lds = (size_t)3 * max_points * sizeof(uint32_t);
  hipLaunchKernelGGL(k_interp, dim3(nblocks), dim3(256), lds, s, jobs, bmap, tab);
}

void launch_mrc(const JobDev* jobs, const int4* bmap, int nblocks, int max_primes, TablesDev tab,
                hipStream_t s) {
  size_t lds = (size_t)2 * max_primes * sizeof(uint32_t);
  hipLaunchKernelGGL(k_mrc, dim3(nblocks), dim3(64), lds, s, jobs, bmap, tab);
}

void launch_limbs_sum(const JobDev* jobs, const int4* bmap, int nblocks, TablesDev tab, hipStream_t s) {
  hipLaunchKernelGGL(k_limbs_sum, dim3(nblocks), dim3(256), 0, s, jobs, bmap, tab);
}

void launch_limbs_carry(const JobDev* jobs, const int4* bmap, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_limbs_carry, dim3(nblocks), dim3(64), 0, s, jobs, bmap);
}

}  // namespace bires
