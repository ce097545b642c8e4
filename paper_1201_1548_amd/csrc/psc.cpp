// Principal subresultant coefficients modulo one prime and the N^- / N^+
// test of Section 3.2.2 ("Computation of N^+", "(Exact) Computation of N",
// "Computation of N^-").
//
// psc: the inputs are reduced modulo the prime (k_reduce), every point
// a = 0..D-1 runs the subresultant recurrence in one lane (k_psc), and each
// index i is interpolated on the nodes 0..D-1 (k_interp, one block per
// index).  D is the resultant's point count: sr_i is a minor of the Sylvester
// matrix's rows (n - i rows of f, m - i of g), so the degree bound of R bounds
// it too.  The prime must be one of the library's table primes (the largest
// below 2^32 / 3), whose tables the kernels index; the kernels see the table
// shifted so that the prime is index 0.
//
// Fiber bounds: with the psc's of (f, f_y) and Q = res(f_x, f_y; y) modulo p
// on the device, one block (k_fiber_chain) runs the gcd chain S_i and the
// common part of R* and Q over F_p.  The host adds up
//   N^- = sum_{i >= 1} (n_y - i) (deg S_{i-1} - deg S_i)      (eq. lower-bound),
//   N^+ = deg R* n_y - deg R + deg gcd(R^inf mod p, Q mod p)   (eq. up-bound).
#include <algorithm>
#include <cstring>

#include "engine.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace bires {

namespace {

struct Layout {
  size_t bytes = 0;
  size_t take(size_t n) {
    const size_t o = (bytes + 255) & ~(size_t)255;
    bytes = o + n;
    return o;
  }
};

struct DevBuf {
  Pool* pool = nullptr;
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void take(Pool* pl, size_t n) {
    pool = pl;
    p = n ? pl->alloc(n) : nullptr;
  }
  ~DevBuf() {
    if (pool) pool->release(p);
  }
  template <class T>
  T* as(size_t off = 0) const {
    return (T*)((uint8_t*)p + off);
  }
};

#define DEV(x)                                   \
  do {                                           \
    if ((x) != hipSuccess) return BIRES_EDEVICE; \
  } while (0)

// Index of p in the prime table (descending), or -1.
int table_index(uint32_t p) {
  const HostTables& t = host_tables();
  int lo = 0, hi = (int)t.primes.size() - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) / 2;
    const uint32_t v = t.primes[mid].p;
    if (v == p) return mid;
    if (v > p) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

TablesDev shifted(const TablesDev& t, int k) {
  TablesDev s = t;
  s.primes += k;
  s.invfact += (size_t)k * t.dmax;
  s.inv_p += k;
  s.K -= k;
  return s;
}

// The psc's of one planned job on the device: coefficients [K][D] (plain) at
// *coefs inside `ws`, which the caller keeps.
struct PscRun {
  DevBuf ws;
  const uint32_t* coefs = nullptr;
  int K = 0, D = 0, m = -1, n = -1;
};

}  // namespace

int psc_count(int m, int n) {
  if (m < 0 || n < 0) return 0;
  return std::min(m, n) + 1 - (m == n ? 1 : 0);
}

static int psc_device(Context* cx, const HostJob& h, int kind, int kp, int kmax, hipStream_t st, PscRun& r) {
  const Plan& pl = h.pl;
  if (pl.m < 0 || pl.n < 0) return BIRES_EINVAL;  // not formed for a zero polynomial
  r.m = pl.m;
  r.n = pl.n;
  r.D = pl.D;
  r.K = psc_count(pl.m, pl.n);
  if (kmax > 0) r.K = std::min(r.K, kmax);
  if (r.K == 0) return BIRES_OK;
  const int D = pl.D, K = r.K;
  if (D > MAX_POINTS || psc_lds_bytes(pl.m, pl.n) > cx->lds_per_block ||
      interp_lds_words(D) * 4 > cx->lds_per_block)
    return BIRES_ETOOBIG;
  const bool derived = kind != BIRES_KIND_RESULTANT;
  const int ldg = derived ? h.ld_f : h.ld_g;
  const int lpf = pad4(h.ld_f), lpg = pad4(ldg);
  const int Tf = (pl.m + 1) * lpf, Tg = (pl.n + 1) * lpg;
  Layout L;
  const size_t o_lf = L.take(h.f.size() * 4);
  const size_t o_lg = L.take(h.g.size() * 4);
  const size_t o_rd = L.take((size_t)(pl.m + pl.n + 2) * 4);
  const size_t o_job = L.take(sizeof(JobDev));
  const size_t o_st = L.take(2 * sizeof(int));
  const size_t o_ij = L.take(sizeof(JobDev) * K);
  const size_t o_is = L.take(sizeof(int) * (K + 1));
  const size_t up_end = L.bytes;
  const size_t o_rf = L.take((size_t)Tf * 4 + 256);  // whole-chunk loads read past a short row
  const size_t o_rg = L.take((size_t)Tg * 4 + 256);
  const size_t o_num = L.take((size_t)K * D * 4);
  const size_t o_den = L.take((size_t)K * D * 4);
  const size_t o_co = L.take((size_t)K * D * 4);
  r.ws.take(&cx->dev, L.bytes);
  DevBuf host;
  host.take(&cx->host, up_end);
  if (!r.ws.p || !host.p) return BIRES_ENOMEM;
  uint8_t* H = host.as<uint8_t>();
  std::memset(H, 0, up_end);
  std::memcpy(H + o_lf, h.f.data(), h.f.size() * 4);
  if (!h.g.empty()) std::memcpy(H + o_lg, h.g.data(), h.g.size() * 4);
  int32_t* rd = (int32_t*)(H + o_rd);
  for (int j = 0; j <= pl.m; ++j) rd[j] = h.stf.deg(j);
  for (int j = 0; j <= pl.n; ++j) rd[pl.m + 1 + j] = h.stg.deg(j);
  JobDev J{};
  J.limbs_f = r.ws.as<uint32_t>(o_lf);
  J.limbs_g = derived ? nullptr : r.ws.as<uint32_t>(o_lg);
  J.Lf = h.L_f;
  J.Lg = derived ? h.L_f : h.L_g;
  J.ldf = h.ld_f;
  J.ldg = ldg;
  J.m = pl.m;
  J.n = pl.n;
  J.kind = kind;
  J.P = 1;
  J.D = D;
  J.lpf = lpf;
  J.lpg = lpg;
  J.Tf = Tf;
  J.Tg = Tg;
  J.rowdeg_f = r.ws.as<int32_t>(o_rd);
  J.rowdeg_g = r.ws.as<int32_t>(o_rd) + pl.m + 1;
  J.res_f = r.ws.as<uint32_t>(o_rf);
  J.res_g = r.ws.as<uint32_t>(o_rg);
  std::memcpy(H + o_job, &J, sizeof J);
  int* st2 = (int*)(H + o_st);
  st2[0] = 0;
  st2[1] = (Tf + 63) / 64 + (Tg + 63) / 64;
  JobDev* IJ = (JobDev*)(H + o_ij);
  int* is = (int*)(H + o_is);
  for (int i = 0; i < K; ++i) {
    IJ[i] = JobDev{};
    IJ[i].P = 1;
    IJ[i].D = D;
    IJ[i].vals = r.ws.as<uint32_t>(o_num) + (size_t)i * D;
    IJ[i].coefs = r.ws.as<uint32_t>(o_co) + (size_t)i * D;
    is[i] = i;
  }
  is[K] = K;
  const TablesDev tab = shifted(cx->tab, kp);
  DEV(hipMemcpyAsync(r.ws.p, H, up_end, hipMemcpyHostToDevice, st));
  launch_reduce(r.ws.as<JobDev>(o_job), r.ws.as<int>(o_st), 1, st2[1], 1, tab, st);
  launch_psc(J, tab, r.ws.as<uint32_t>(o_num), r.ws.as<uint32_t>(o_den), K, st);
  launch_interp(r.ws.as<JobDev>(o_ij), r.ws.as<int>(o_is), K, K, D, tab, nullptr, nullptr, 0, st);
  DEV(hipGetLastError());
  // the staging block is read by the copy: it must outlive it
  DEV(hipStreamSynchronize(st));
  r.coefs = r.ws.as<uint32_t>(o_co);
  return BIRES_OK;
}

int run_psc(Context* cx, const JobIn& jb, uint32_t p, uint32_t* out, int64_t capacity, int32_t* count,
            int32_t* points, hipStream_t st) {
  const int kp = table_index(p);
  if (kp < 0) return BIRES_EINVAL;
  HostJob h;
  int e = host_job(jb, h);
  if (e) return e;
  if (h.pl.m < 0 || h.pl.n < 0) return BIRES_EINVAL;
  const int K = psc_count(h.pl.m, h.pl.n), D = h.pl.D;
  if (count) *count = K;
  if (points) *points = D;
  if ((int64_t)K * D > capacity) return BIRES_EBUFSIZE;
  if (K == 0) return BIRES_OK;
  PscRun r;
  if ((e = psc_device(cx, h, jb.kind, kp, 0, st, r))) return e;
  DEV(hipMemcpyAsync(out, r.coefs, (size_t)K * D * 4, hipMemcpyDeviceToHost, st));
  DEV(hipStreamSynchronize(st));
  return BIRES_OK;
}

int run_fiber_bounds(Context* cx, const bires_bipoly& f, int var, const bires_upoly& rstar, int32_t deg_r,
                     uint32_t p, int64_t* n_minus, int64_t* n_plus, int32_t* flags, hipStream_t st) {
  const int kp = table_index(p);
  if (kp < 0 || rstar.limbs < 1 || rstar.degree < 0 || !rstar.c || deg_r < 0) return BIRES_EINVAL;
  // R* trimmed (host memory), the degree the test counts with
  const int L = rstar.limbs;
  int dr = rstar.degree;
  auto zero = [&](int i) {
    for (int l = 0; l < L; ++l)
      if (rstar.c[(size_t)i * L + l]) return false;
    return true;
  };
  while (dr >= 0 && zero(dr)) --dr;
  if (dr < 0) return BIRES_EINVAL;
  JobIn jd;
  jd.f = f;
  jd.g = f;
  jd.var = var;
  jd.kind = BIRES_KIND_DISCRIMINANT;
  HostJob hd;
  int e = host_job(jd, hd);
  if (e) return e;
  JobIn jq = jd;
  jq.kind = BIRES_KIND_POLAR;
  HostJob hq;
  if ((e = host_job(jq, hq))) return e;
  const int ny = hd.pl.m;
  int32_t fl = 0;
  // the lemma's condition: p divides neither lc_y f nor lc_y f_y (n_y lc_y f, n_y < p)
  {
    const int ld = hd.ld_f, Lf = hd.L_f;
    const ModP& q = host_tables().primes[kp];
    bool all_zero = true;
    for (int i = 0; i < ld && all_zero; ++i) {
      const uint32_t* c = hd.f.data() + ((size_t)ny * ld + i) * Lf;
      // two's-complement limbs modulo p, top limb first
      const bool neg = (c[Lf - 1] >> 31) != 0u;
      uint64_t v = 0;
      for (int l = Lf - 1; l >= 0; --l) v = ((v << 32) | c[l]) % q.p;
      if (neg) {
        uint64_t two = 1;
        for (int l = 0; l < Lf; ++l) two = (two << 32) % q.p;
        v = (v + q.p - two) % q.p;
      }
      all_zero = v == 0;
    }
    if (all_zero) fl |= 1;
  }
  PscRun rd, rq;
  if ((e = psc_device(cx, hd, BIRES_KIND_DISCRIMINANT, kp, 0, st, rd))) return e;
  const bool q_zero = hq.pl.m < 0;  // f_x = 0
  if (!q_zero && (e = psc_device(cx, hq, BIRES_KIND_POLAR, kp, 1, st, rq))) return e;
  // R* mod p: a one-row rectangle through k_reduce
  Layout Lo;
  const size_t o_l = Lo.take((size_t)(dr + 1) * L * 4);
  const size_t o_job = Lo.take(sizeof(JobDev));
  const size_t o_st = Lo.take(2 * sizeof(int));
  const size_t o_cd = Lo.take(sizeof(ChainDev));
  const size_t o_z = Lo.take(4);  // Q = 0 when f_x = 0
  const size_t up_end = Lo.bytes;
  const size_t o_r = Lo.take((size_t)pad4(dr + 1) * 4 + 256);
  const size_t o_out = Lo.take((size_t)(rd.K + 2) * 4);
  DevBuf ws, host;
  ws.take(&cx->dev, Lo.bytes);
  host.take(&cx->host, up_end);
  if (!ws.p || !host.p) return BIRES_ENOMEM;
  uint8_t* H = host.as<uint8_t>();
  std::memset(H, 0, up_end);
  std::memcpy(H + o_l, rstar.c, (size_t)(dr + 1) * L * 4);
  JobDev J{};
  J.limbs_f = ws.as<uint32_t>(o_l);
  J.Lf = L;
  J.Lg = L;
  J.ldf = dr + 1;
  J.ldg = dr + 1;
  J.m = 0;
  J.n = -1;
  J.P = 1;
  J.lpf = pad4(dr + 1);
  J.lpg = pad4(dr + 1);
  J.Tf = J.lpf;
  J.Tg = 0;
  J.res_f = ws.as<uint32_t>(o_r);
  std::memcpy(H + o_job, &J, sizeof J);
  int* st2 = (int*)(H + o_st);
  st2[0] = 0;
  st2[1] = (J.Tf + 63) / 64;
  ChainDev C{};
  C.rstar = J.res_f;
  C.dr = dr;
  C.srs = rd.coefs;
  C.K = rd.K;
  C.D = rd.D;
  C.qpol = q_zero ? ws.as<uint32_t>(o_z) : rq.coefs;
  C.Dq = q_zero ? 1 : rq.D;
  C.out = ws.as<int32_t>(o_out);
  if (fiber_chain_lds_bytes(C.dr, C.D, C.Dq) > cx->lds_per_block) return BIRES_ETOOBIG;
  std::memcpy(H + o_cd, &C, sizeof C);
  const TablesDev tab = shifted(cx->tab, kp);
  DEV(hipMemcpyAsync(ws.p, H, up_end, hipMemcpyHostToDevice, st));
  launch_reduce(ws.as<JobDev>(o_job), ws.as<int>(o_st), 1, st2[1], 1, tab, st);
  launch_fiber_chain(C, tab, st);
  DEV(hipGetLastError());
  std::vector<int32_t> out(rd.K + 2);
  DEV(hipMemcpyAsync(out.data(), C.out, out.size() * 4, hipMemcpyDeviceToHost, st));
  DEV(hipStreamSynchronize(st));
  if (out[0] != dr) fl |= 2;          // p divides lc(R*)
  if (q_zero || out[rd.K + 1]) fl |= 4;  // Q = 0 mod p
  int64_t nm = 0;
  for (int i = 1; i <= rd.K; ++i) {
    const int64_t prev = out[i - 1], cur = i < rd.K ? out[i] : 0;
    nm += (int64_t)(ny - i) * (prev - cur);
  }
  const int64_t np = (int64_t)dr * ny - deg_r + out[rd.K];
  if (n_minus) *n_minus = nm;
  if (n_plus) *n_plus = np;
  if (flags) *flags = fl;
  return BIRES_OK;
}

}  // namespace bires
