// gcd in Z[x] by Brown's modular method (Section 5.1, "Computing gcds in Z[x]":
// reduce modulo many primes, gcd in F_p[x], Chinese remaindering).
//
// With beta = gcd(lc a, lc b), every prime p not dividing lc(a) lc(b) gives the
// monic gcd g_p of a mod p and b mod p; the primes of minimal deg g_p are kept.
// The kernels also return the exact quotients a/g_p, b/g_p.  Reconstructed
// from the kept primes (mixed radix, symmetric lift) are
//     F  = beta g,   Qa = (lc a / beta) a/g,   Qb = (lc b / beta) b/g,
// whose images satisfy F Qa = lc(a) a and F Qb = lc(b) b modulo every kept
// prime.  Certificate: if ||F||_1 ||Qa||_1 < M/2 and |lc a| ||a||_inf < M/2
// (M the product of the kept primes), both sides are integers below M/2 in
// every coefficient, so F Qa = lc(a) a over Z; likewise for b.  Then pp(F)
// divides a and b (Gauss's lemma), and deg F = min deg g_p >= deg gcd, so
// pp(F) is the primitive gcd.  A failed certificate doubles the prime count.
// The result is gcd(cont a, cont b) pp(F) with positive leading coefficient.
#include "gcd.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "bigint.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace bires {

namespace {

struct DevBuf {
  Pool* pool;
  void* p = nullptr;
  DevBuf(Pool* pl, size_t n) : pool(pl) { p = n ? pl->alloc(n) : nullptr; }
  ~DevBuf() { pool->release(p); }
  template <class T>
  T* as(size_t byte_off = 0) const {
    return (T*)((uint8_t*)p + byte_off);
  }
};

struct Layout {
  size_t bytes = 0;
  size_t take(size_t n) {
    const size_t o = (bytes + 255) & ~(size_t)255;
    bytes = o + n;
    return o;
  }
};

using Poly = std::vector<BigInt>;

void trim_poly(Poly& v) {
  while (!v.empty() && v.back().is_zero()) v.pop_back();
}

int read_upoly(const bires_upoly& u, int mem, hipStream_t st, Poly& out) {
  if (u.degree < -1 || u.limbs < 1 || (u.degree >= 0 && !u.c)) return BIRES_EINVAL;
  out.clear();
  if (u.degree < 0) return BIRES_OK;
  const size_t n = (size_t)u.degree + 1, L = (size_t)u.limbs;
  std::vector<uint32_t> buf(n * L);
  if (mem == BIRES_MEM_HOST) {
    std::memcpy(buf.data(), u.c, n * L * 4);
  } else {
    if (hipMemcpyAsync(buf.data(), u.c, n * L * 4, hipMemcpyDeviceToHost, st) != hipSuccess) return BIRES_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return BIRES_EDEVICE;
  }
  out.resize(n);
  for (size_t i = 0; i < n; ++i) out[i] = BigInt::from_twos(buf.data() + i * L, (int)L);
  trim_poly(out);
  return BIRES_OK;
}

int write_upoly(const Poly& v, bires_upoly* out, int mem, hipStream_t st) {
  const int deg = (int)v.size() - 1;
  int bits = 0;
  for (const auto& c : v) bits = std::max(bits, c.bits());
  const int need_limbs = bits / 32 + 1;  // magnitude bits plus a sign bit
  if (out->degree < std::max(deg, 0) || out->limbs < need_limbs) {
    out->degree = std::max(out->degree, std::max(deg, 0));
    out->limbs = std::max(out->limbs, need_limbs);
    return BIRES_EBUFSIZE;
  }
  const size_t n = (size_t)out->degree + 1, L = (size_t)out->limbs;
  std::vector<uint32_t> buf(n * L, 0u);
  for (size_t i = 0; i < v.size(); ++i) v[i].to_twos(buf.data() + i * L, (int)L);
  if (mem == BIRES_MEM_HOST) {
    std::memcpy(out->c, buf.data(), n * L * 4);
  } else {
    if (hipMemcpyAsync(out->c, buf.data(), n * L * 4, hipMemcpyHostToDevice, st) != hipSuccess) return BIRES_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return BIRES_EDEVICE;
  }
  out->degree = deg;
  return BIRES_OK;
}

BigInt content(const Poly& v) {
  BigInt g;
  for (const auto& c : v) {
    g = big_gcd(g, c);
    if (g.mag.size() == 1 && g.mag[0] == 1u) break;
  }
  return g;
}

// x with positive leading coefficient
void make_positive(Poly& v) {
  if (!v.empty() && v.back().neg)
    for (auto& c : v) c.neg = !c.neg && !c.is_zero();
}

int max_bits(const Poly& v) {
  int b = 0;
  for (const auto& c : v) b = std::max(b, c.bits());
  return b;
}

int limbs_of(const Poly& v) { return max_bits(v) / 32 + 1; }

// Pack a polynomial as [(deg+1)][L] two's-complement limbs.
void pack(const Poly& v, int L, uint32_t* dst) {
  for (size_t i = 0; i < v.size(); ++i) v[i].to_twos(dst + i * L, L);
}

}  // namespace

int gcd_bounds(const bires_upoly* a, const bires_upoly* b, int32_t* max_degree, int32_t* max_limbs) {
  if (!a || !b || a->degree < -1 || b->degree < -1 || a->limbs < 1 || b->limbs < 1) return BIRES_EINVAL;
  int deg, bits;
  if (a->degree < 0 && b->degree < 0) {
    deg = 0;
    bits = 1;
  } else if (a->degree < 0 || b->degree < 0) {
    const bires_upoly* x = a->degree < 0 ? b : a;
    deg = x->degree;
    bits = 32 * x->limbs + 1;  // |x| may need one more bit than x
  } else {
    // Landau-Mignotte: a divisor of x of degree <= d has |coefficients| <= 2^d ||x||_2
    deg = std::min(a->degree, b->degree);
    auto mig = [&](const bires_upoly* x) {
      return deg + 32 * x->limbs + (int)std::ceil(0.5 * std::log2((double)x->degree + 1.0)) + 1;
    };
    bits = std::min(mig(a), mig(b));
  }
  if (max_degree) *max_degree = deg;
  if (max_limbs) *max_limbs = bits / 32 + 1;
  return BIRES_OK;
}

namespace {

// Reduction and per-prime gcds for primes 0..P-1; F/QA/QB stay in `ws`.
int modular_phase(Context* cx, const Poly& A, const Poly& B, const BigInt& beta, int P, hipStream_t st,
                  DevBuf& ws, size_t& o_F, size_t& o_QA, size_t& o_QB, std::vector<int32_t>& gdeg) {
  const HostTables& T = host_tables();
  const int da = (int)A.size() - 1, db = (int)B.size() - 1, mn = std::min(da, db);
  const int La = limbs_of(A), Lb = limbs_of(B);
  BigInt qa, qb;
  big_divexact(A.back(), beta, qa);
  big_divexact(B.back(), beta, qb);
  Layout L;
  const size_t o_la = L.take((size_t)(da + 1) * La * 4);
  const size_t o_lb = L.take((size_t)(db + 1) * Lb * 4);
  const size_t o_sc = L.take((size_t)P * 3 * 4);
  const size_t o_job = L.take(sizeof(JobDev));
  const size_t o_st = L.take(2 * sizeof(int));
  const size_t up_end = L.bytes;  // everything above is uploaded
  const size_t o_ra = L.take((size_t)P * (da + 1) * 4);
  const size_t o_rb = L.take((size_t)P * (db + 1) * 4);
  o_F = L.take((size_t)P * (mn + 1) * 4);
  o_QA = L.take((size_t)P * (da + 1) * 4);
  o_QB = L.take((size_t)P * (db + 1) * 4);
  const size_t o_gd = L.take((size_t)P * 4);
  DevBuf dev(&cx->dev, L.bytes);
  DevBuf host(&cx->host, up_end);
  if (!dev.p || !host.p) return BIRES_ENOMEM;
  uint8_t* H = host.as<uint8_t>();
  std::memset(H, 0, up_end);
  pack(A, La, (uint32_t*)(H + o_la));
  pack(B, Lb, (uint32_t*)(H + o_lb));
  uint32_t* sc = (uint32_t*)(H + o_sc);
  for (int k = 0; k < P; ++k) {
    const uint32_t p = T.primes[k].p;
    sc[3 * k] = big_mod_small(beta, p);
    sc[3 * k + 1] = big_mod_small(qa, p);
    sc[3 * k + 2] = big_mod_small(qb, p);
  }
  JobDev J{};
  J.limbs_f = dev.as<uint32_t>(o_la);
  J.limbs_g = dev.as<uint32_t>(o_lb);
  J.Lf = La;
  J.Lg = Lb;
  J.ldf = da + 1;
  J.ldg = db + 1;
  J.P = P;
  J.lpf = da + 1;
  J.lpg = db + 1;
  J.Tf = da + 1;
  J.Tg = db + 1;
  J.res_f = dev.as<uint32_t>(o_ra);
  J.res_g = dev.as<uint32_t>(o_rb);
  std::memcpy(H + o_job, &J, sizeof J);
  int* starts = (int*)(H + o_st);
  starts[0] = 0;
  starts[1] = (J.Tf + 63) / 64 + (J.Tg + 63) / 64;
  if (hipMemcpyAsync(dev.p, H, up_end, hipMemcpyHostToDevice, st) != hipSuccess) return BIRES_EDEVICE;
  launch_reduce(dev.as<JobDev>(o_job), dev.as<int>(o_st), 1, starts[1], P, cx->tab, st);
  GcdDev G{};
  G.res_a = J.res_f;
  G.res_b = J.res_g;
  G.da = da;
  G.db = db;
  G.P = P;
  G.sc = dev.as<uint32_t>(o_sc);
  G.F = dev.as<uint32_t>(o_F);
  G.QA = dev.as<uint32_t>(o_QA);
  G.QB = dev.as<uint32_t>(o_QB);
  G.gdeg = dev.as<int32_t>(o_gd);
  launch_gcd_p(G, cx->tab, st);
  if (hipGetLastError() != hipSuccess) return BIRES_EDEVICE;
  gdeg.resize(P);
  if (hipMemcpyAsync(gdeg.data(), G.gdeg, (size_t)P * 4, hipMemcpyDeviceToHost, st) != hipSuccess)
    return BIRES_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return BIRES_EDEVICE;
  std::swap(ws.p, dev.p);  // hand the workspace (F, QA, QB) to the caller
  return BIRES_OK;
}

// Mixed-radix reconstruction of `rows` of `src` arrays (row stride ld[j],
// n[j] coefficients each) over the prime subset S, as symmetric integers.
int reconstruct(Context* cx, const std::vector<int>& S, const std::vector<const uint32_t*>& src,
                const std::vector<int>& ld, const std::vector<int>& n, hipStream_t st, std::vector<Poly>& out) {
  const HostTables& T = host_tables();
  const int nj = (int)src.size(), P = (int)S.size();
  std::vector<ModP> primes(P);
  for (int i = 0; i < P; ++i) primes[i] = T.primes[S[i]];
  std::vector<uint32_t> gm, cm, pm, pi;
  mrc_tables(primes, gm, cm, pm, pi);
  const int Lcap = P + 1, Lacc = P + 1;
  Layout L;
  const size_t o_pr = L.take(primes.size() * sizeof(ModP));
  const size_t o_gm = L.take(gm.size() * 4);
  const size_t o_cm = L.take(cm.size() * 4);
  const size_t o_pm = L.take(pm.size() * 4);
  const size_t o_pi = L.take(pi.size() * 4);
  const size_t o_idx = L.take((size_t)P * 4);
  const size_t o_jobs = L.take(sizeof(JobDev) * nj);
  const size_t o_st = L.take(sizeof(int) * 3 * (nj + 1));
  const size_t o_flags = L.take(sizeof(int) * 2 * nj);
  const size_t up_end = L.bytes;
  std::vector<size_t> o_c(nj), o_d(nj), o_n(nj), o_lo(nj), o_hi(nj), o_o(nj);
  for (int j = 0; j < nj; ++j) {
    o_c[j] = L.take((size_t)P * n[j] * 4);
    o_d[j] = L.take((size_t)P * n[j] * 4);
    o_n[j] = L.take((size_t)n[j] * 4);
    o_lo[j] = L.take((size_t)n[j] * Lacc * 8);
    o_hi[j] = L.take((size_t)n[j] * Lacc * 4);
    o_o[j] = L.take((size_t)n[j] * Lcap * 4);
  }
  DevBuf dev(&cx->dev, L.bytes), host(&cx->host, L.bytes);
  if (!dev.p || !host.p) return BIRES_ENOMEM;
  uint8_t* H = host.as<uint8_t>();
  std::memcpy(H + o_pr, primes.data(), primes.size() * sizeof(ModP));
  std::memcpy(H + o_gm, gm.data(), gm.size() * 4);
  std::memcpy(H + o_cm, cm.data(), cm.size() * 4);
  std::memcpy(H + o_pm, pm.data(), pm.size() * 4);
  std::memcpy(H + o_pi, pi.data(), pi.size() * 4);
  std::memcpy(H + o_idx, S.data(), (size_t)P * 4);
  JobDev* J = (JobDev*)(H + o_jobs);
  int* st3 = (int*)(H + o_st);
  int32_t* flags = (int32_t*)(H + o_flags);
  st3[0] = st3[nj + 1] = st3[2 * (nj + 1)] = 0;
  for (int j = 0; j < nj; ++j) {
    J[j] = JobDev{};
    J[j].P = P;
    J[j].D = n[j];
    J[j].coefs = dev.as<uint32_t>(o_c[j]);
    J[j].digits = dev.as<uint32_t>(o_d[j]);
    J[j].negflag = dev.as<int32_t>(o_n[j]);
    J[j].acc_lo = dev.as<uint64_t>(o_lo[j]);
    J[j].acc_hi = dev.as<uint32_t>(o_hi[j]);
    J[j].Lacc = Lacc;
    J[j].out = dev.as<uint32_t>(o_o[j]);
    J[j].Lcap = Lcap;
    J[j].degcap = n[j] - 1;
    J[j].deg_out = dev.as<int32_t>(o_flags) + 2 * j;
    J[j].err = dev.as<int32_t>(o_flags) + 2 * j + 1;
    flags[2 * j] = -1;
    flags[2 * j + 1] = 0;
    st3[j + 1] = st3[j] + n[j];  // mrc
    st3[nj + 1 + j + 1] = st3[nj + 1 + j] + (n[j] * Lacc + 255) / 256;  // limbs_sum
    st3[2 * (nj + 1) + j + 1] = st3[2 * (nj + 1) + j] + (n[j] + 63) / 64;  // limbs_carry
  }
  if (hipMemcpyAsync(dev.p, H, up_end, hipMemcpyHostToDevice, st) != hipSuccess) return BIRES_EDEVICE;
  for (int j = 0; j < nj; ++j)
    launch_gather_rows(src[j], ld[j], dev.as<int>(o_idx), P, n[j], dev.as<uint32_t>(o_c[j]), st);
  TablesDev tab{};
  tab.primes = dev.as<ModP>(o_pr);
  tab.gm = dev.as<uint32_t>(o_gm);
  tab.cm = dev.as<uint32_t>(o_cm);
  tab.pm = dev.as<uint32_t>(o_pm);
  tab.pi = dev.as<uint32_t>(o_pi);
  tab.K = P;
  const int* dst = dev.as<int>(o_st);
  const JobDev* dj = dev.as<JobDev>(o_jobs);
  launch_mrc(dj, dst, nj, st3[nj], P, tab, st);
  launch_limbs_sum(dj, dst + nj + 1, nj, st3[2 * nj + 1], tab, st);
  launch_limbs_carry(dj, dst + 2 * (nj + 1), nj, st3[3 * nj + 2], Lcap, st);
  if (hipGetLastError() != hipSuccess) return BIRES_EDEVICE;
  for (int j = 0; j < nj; ++j)
    if (hipMemcpyAsync(H + o_o[j], dev.as<uint8_t>(o_o[j]), (size_t)n[j] * Lcap * 4, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return BIRES_EDEVICE;
  if (hipMemcpyAsync(H + o_flags, dev.as<uint8_t>(o_flags), sizeof(int) * 2 * nj, hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return BIRES_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return BIRES_EDEVICE;
  out.assign(nj, Poly());
  for (int j = 0; j < nj; ++j) {
    if (flags[2 * j + 1]) return BIRES_ECHECK;
    const uint32_t* o = (const uint32_t*)(H + o_o[j]);
    out[j].resize(n[j]);
    for (int i = 0; i < n[j]; ++i) out[j][i] = BigInt::from_twos(o + (size_t)i * Lcap, Lcap);
    trim_poly(out[j]);
  }
  return BIRES_OK;
}

}  // namespace

namespace {

// The modular core for A, B of degree >= 1: G = pp(F) with positive leading
// coefficient and, when CA / CB are given, the exact cofactors A / G and
// B / G.  From F Qa = lc(A) A (certified over Z): A / pp(F) = cont(F) Qa /
// lc(A), an exact division per coefficient.
int gcd_core(Context* cx, const Poly& A, const Poly& B, hipStream_t st, Poly& G, Poly* CA, Poly* CB) {
  const int da = (int)A.size() - 1, db = (int)B.size() - 1;
  if (std::max(da, db) > MAX_GCD_DEGREE) return BIRES_ETOOBIG;
  if (gcd_lds_bytes(da, db) > cx->lds_per_block) return BIRES_ETOOBIG;
  const BigInt beta = big_gcd(A.back(), B.back());
  const int ba = max_bits(A), bb = max_bits(B);
  const HostTables& T = host_tables();
  int need = std::max(A.back().bits() + ba, B.back().bits() + bb) + beta.bits() + 64;
  std::vector<Poly> rec;
  for (int attempt = 0;; ++attempt) {
    int P = 0;
    while (P < T.K && T.cumlog[P] < need) ++P;
    P = std::min(T.K, P + 4);  // spares for primes dividing lc(a) lc(b) or unlucky ones
    if (attempt > 8 || T.cumlog[P] < need) return BIRES_ETOOBIG;
    DevBuf ws(&cx->dev, 0);
    size_t o_F = 0, o_QA = 0, o_QB = 0;
    std::vector<int32_t> gdeg;
    int e = modular_phase(cx, A, B, beta, P, st, ws, o_F, o_QA, o_QB, gdeg);
    if (e) return e;
    int d = 1 << 30;
    for (int k = 0; k < P; ++k) {
      if (gdeg[k] == -3) return BIRES_ECHECK;
      if (gdeg[k] >= 0) d = std::min(d, (int)gdeg[k]);
    }
    if (d == (1 << 30)) {
      need *= 2;
      continue;
    }
    std::vector<int> S;
    for (int k = 0; k < P; ++k)
      if (gdeg[k] == d) S.push_back(k);
    const int mn = std::min(da, db);
    rec.clear();
    e = reconstruct(cx, S, {ws.as<uint32_t>(o_F), ws.as<uint32_t>(o_QA), ws.as<uint32_t>(o_QB)},
                    {mn + 1, da + 1, db + 1}, {d + 1, da - d + 1, db - d + 1}, st, rec);
    if (e) return e;
    double log2M = 0.0;
    for (int k : S) log2M += T.log2p[k];
    auto n1 = [](const Poly& v) { return max_bits(v) + std::log2((double)v.size() + 1.0); };
    const bool ok_a = n1(rec[0]) + n1(rec[1]) < log2M - 2.0 && A.back().bits() + ba < log2M - 2.0;
    const bool ok_b = n1(rec[0]) + n1(rec[2]) < log2M - 2.0 && B.back().bits() + bb < log2M - 2.0;
    if (ok_a && ok_b && (int)rec[0].size() == d + 1) break;
    need = (int)std::ceil(std::max<double>(need, n1(rec[0]) + std::max(n1(rec[1]), n1(rec[2])) + 8.0)) * 2;
  }
  const Poly& Fs = rec[0];
  const BigInt cf = content(Fs);
  G.assign(Fs.size(), BigInt());
  for (size_t i = 0; i < Fs.size(); ++i)
    if (!big_divexact(Fs[i], cf, G[i])) return BIRES_ECHECK;
  const bool flip = G.back().neg;
  make_positive(G);
  if (G.size() == 1) {  // coprime: the cofactors are A and B
    if (CA) *CA = A;
    if (CB) *CB = B;
    return BIRES_OK;
  }
  for (int w = 0; w < 2; ++w) {
    Poly* C = w ? CB : CA;
    if (!C) continue;
    const Poly& Q = rec[1 + w];
    // cont(F) Q / lc with the common factor of cont(F) and lc cancelled
    // first, so that a unit divisor leaves only products
    const BigInt& lc = w ? B.back() : A.back();
    const BigInt h = big_gcd(cf, lc);
    BigInt num, den;
    if (!big_divexact(cf, h, num) || !big_divexact(lc, h, den)) return BIRES_ECHECK;
    const bool unit = den.mag.size() == 1 && den.mag[0] == 1u;
    const bool neg = den.neg != flip;
    den.neg = false;
    C->assign(Q.size(), BigInt());
    for (size_t i = 0; i < Q.size(); ++i) {
      const BigInt t = (num.mag.size() == 1 && num.mag[0] == 1u && !num.neg) ? Q[i] : big_mul(num, Q[i]);
      if (unit) {
        (*C)[i] = t;
      } else if (!big_divexact(t, den, (*C)[i])) {
        return BIRES_ECHECK;
      }
      if (neg) (*C)[i].neg = !(*C)[i].neg && !(*C)[i].is_zero();
    }
    trim_poly(*C);
  }
  return BIRES_OK;
}

// gcd with exact cofactors for any A, B (G primitive when A or B is
// primitive): G = 1 when either is a non-zero constant, G = pp(A) when B = 0.
int gcd_cofactors(Context* cx, const Poly& A, const Poly& B, hipStream_t st, Poly& G, Poly& CA, Poly& CB) {
  if (B.empty()) {
    if (A.empty()) return BIRES_EINVAL;
    const BigInt c = content(A);
    G.assign(A.size(), BigInt());
    for (size_t i = 0; i < A.size(); ++i)
      if (!big_divexact(A[i], c, G[i])) return BIRES_ECHECK;
    BigInt u = c;
    if (G.back().neg) u.neg = true;
    make_positive(G);
    CA = Poly{u};
    CB.clear();
    return BIRES_OK;
  }
  if (A.size() == 1 || B.size() == 1) {
    G = Poly{BigInt::from_u64(1)};
    CA = A;
    CB = B;
    return BIRES_OK;
  }
  return gcd_core(cx, A, B, st, G, &CA, &CB);
}

Poly derivative(const Poly& v) {
  Poly d;
  for (size_t i = 1; i < v.size(); ++i) d.push_back(big_mul(v[i], BigInt::from_u64(i)));
  trim_poly(d);
  return d;
}

Poly poly_sub(const Poly& a, const Poly& b) {
  Poly r(std::max(a.size(), b.size()));
  for (size_t i = 0; i < r.size(); ++i) {
    BigInt nb = i < b.size() ? b[i] : BigInt();
    nb.neg = !nb.neg && !nb.is_zero();
    r[i] = big_add(i < a.size() ? a[i] : BigInt(), nb);
  }
  trim_poly(r);
  return r;
}

}  // namespace

int run_gcd(Context* cx, const bires_upoly& a, const bires_upoly& b, bires_upoly* out, int mem, hipStream_t st) {
  if (mem != BIRES_MEM_HOST && mem != BIRES_MEM_DEVICE) return BIRES_EINVAL;
  if (!out || out->degree < 0 || out->limbs < 1 || !out->c) return BIRES_EINVAL;
  Poly A, B;
  int e = read_upoly(a, mem, st, A);
  if (e) return e;
  if ((e = read_upoly(b, mem, st, B))) return e;
  if (A.empty() && B.empty()) return write_upoly(Poly(), out, mem, st);
  if (A.empty() || B.empty()) {
    Poly G = A.empty() ? B : A;
    make_positive(G);
    return write_upoly(G, out, mem, st);
  }
  const BigInt c = big_gcd(content(A), content(B));
  if (A.size() == 1 || B.size() == 1) return write_upoly(Poly{c}, out, mem, st);
  Poly G;
  if ((e = gcd_core(cx, A, B, st, G, nullptr, nullptr))) return e;
  // primitive gcd times the gcd of the contents
  for (auto& x : G) x = big_mul(x, c);
  return write_upoly(G, out, mem, st);
}

int run_squarefree(Context* cx, const bires_upoly& r, bires_upoly* unit, bires_upoly* factors, int32_t max_factors,
                   int32_t* count, int mem, hipStream_t st) {
  if (mem != BIRES_MEM_HOST && mem != BIRES_MEM_DEVICE) return BIRES_EINVAL;
  if (!unit || !count || max_factors < 0 || (max_factors > 0 && !factors)) return BIRES_EINVAL;
  Poly R;
  int e = read_upoly(r, mem, st, R);
  if (e) return e;
  std::vector<Poly> out;
  BigInt u;  // signed content
  if (R.size() >= 2) {
    u = content(R);
    if (R.back().neg) u.neg = true;
    Poly Rp(R.size());
    for (size_t i = 0; i < R.size(); ++i)
      if (!big_divexact(R[i], u, Rp[i])) return BIRES_ECHECK;
    // Yun: b_1 = R / g, d_1 = R' / g - b_1' with g = gcd(R, R'); then
    // a_i = gcd(b_i, d_i), b_{i+1} = b_i / a_i, d_{i+1} = d_i / a_i - b_{i+1}'
    Poly g, b, c;
    if ((e = gcd_cofactors(cx, Rp, derivative(Rp), st, g, b, c))) return e;
    Poly d = poly_sub(c, derivative(b));
    while (b.size() >= 2) {
      Poly a, b2, c2;
      if ((e = gcd_cofactors(cx, b, d, st, a, b2, c2))) return e;
      out.push_back(a);
      b = b2;
      d = poly_sub(c2, derivative(b));
    }
  } else if (R.size() == 1) {
    u = R[0];
  }
  *count = (int32_t)out.size();
  int first = BIRES_OK;
  const Poly U = u.is_zero() ? Poly() : Poly{u};
  if ((e = write_upoly(U, unit, mem, st)) && first == BIRES_OK) first = e;
  if ((int)out.size() > max_factors) return BIRES_EBUFSIZE;
  for (size_t i = 0; i < out.size(); ++i)
    if ((e = write_upoly(out[i], &factors[i], mem, st)) && first == BIRES_OK) first = e;
  return first;
}

}  // namespace bires
