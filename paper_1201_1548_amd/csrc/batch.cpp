// The batched pipeline: plan every job, lay out one device workspace, launch
// each kernel once for all jobs, copy the results back.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <type_traits>

#include "engine.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace bires {

namespace {

struct Shape {
  int rows = 0, ld = 0, L = 1;
};

Shape shape_of(const bires_bipoly& p, int var) {
  Shape s;
  s.L = p.limbs;
  if (p.deg_y < 0) return s;
  s.rows = var == BIRES_VAR_Y ? p.deg_y + 1 : p.deg_x + 1;
  s.ld = var == BIRES_VAR_Y ? p.deg_x + 1 : p.deg_y + 1;
  return s;
}

void pack_rect(const bires_bipoly& p, int var, uint32_t* dst) {
  const size_t n = (size_t)(p.deg_y + 1) * (p.deg_x + 1) * p.limbs;
  if (var == BIRES_VAR_Y) {
    std::memcpy(dst, p.c, n * sizeof(uint32_t));
    return;
  }
  const int rows = p.deg_y + 1, cols = p.deg_x + 1, L = p.limbs;
  for (int j = 0; j < rows; ++j)
    for (int i = 0; i < cols; ++i)
      for (int l = 0; l < L; ++l) dst[((size_t)i * rows + j) * L + l] = p.c[((size_t)j * cols + i) * L + l];
}

struct Layout {
  size_t bytes = 0;
  size_t take(size_t n) {
    const size_t o = (bytes + 255) & ~(size_t)255;
    bytes = o + n;
    return o;
  }
};

struct Work {
  Shape sf, sg;
  int kind = BIRES_KIND_RESULTANT;
  bool derived = false;  // both operands formed from f (discriminant, polar)
  RowStats stf, stg;
  Plan pl;
  int status = BIRES_OK;
  bool active = false;  // goes through the kernels
  int Lout = 1, degcap = 0, Tf = 0, Tg = 0, ldg = 0, Lacc = 1;
  const uint32_t* dev_f = nullptr;
  const uint32_t* dev_g = nullptr;
  size_t o_in[2] = {0, 0}, o_scan[2] = {0, 0};
  size_t o_res_f = 0, o_res_g = 0, o_vals = 0, o_coefs = 0, o_digits = 0, o_neg = 0, o_acc_lo = 0, o_acc_hi = 0;
  size_t o_out = 0, o_hout = 0, o_rowdeg = 0;
};

// Holder of one pool block (given back when the holder goes).
struct Held {
  Pool* pool = nullptr;
  void* p = nullptr;
  Held() = default;
  Held(const Held&) = delete;
  Held& operator=(const Held&) = delete;
  void take(Pool* pl, size_t n) {
    pool = pl;
    p = n ? pl->alloc(n) : nullptr;
  }
  ~Held() {
    if (pool) pool->release(p);
  }
  uint8_t* b() const { return (uint8_t*)p; }
};

}  // namespace

// Operand statistics of the kinds formed from f alone: g = df/dy for the
// discriminant; f <- df/dx and g = df/dy for the polar resultant.  Both need
// deg_y f >= 1.  On entry f holds the statistics of the input.
static int derive_operand_stats(int kind, RowStats& f, RowStats& g) {
  int top = -1;
  for (int j = 0; j < f.rows(); ++j)
    if (f.cnt(j)) top = j;
  if (top < 1) return BIRES_EINVAL;
  g = derive_stats(f);
  if (kind == BIRES_KIND_POLAR) f = derive_stats_x(f);
  return BIRES_OK;
}

static SpecKey key_of(const JobIn& jb) {
  SpecKey k;
  std::memset(&k, 0, sizeof k);
  k.f[0] = jb.f.deg_x, k.f[1] = jb.f.deg_y, k.f[2] = jb.f.limbs;
  k.g[0] = jb.g.deg_x, k.g[1] = jb.g.deg_y, k.g[2] = jb.g.limbs;
  k.kind = jb.kind;
  k.var = jb.var;
  k.odeg = jb.out ? jb.out->degree : 0;
  k.olimbs = jb.out ? jb.out->limbs : 0;
  return k;
}

static bool same_key(const SpecKey& a, const JobIn& jb) {
  const SpecKey b = key_of(jb);
  return std::memcmp(&a, &b, sizeof a) == 0;
}

static int validate(const JobIn& jb, bool need_out) {
  if (jb.kind != BIRES_KIND_RESULTANT && jb.kind != BIRES_KIND_DISCRIMINANT && jb.kind != BIRES_KIND_POLAR)
    return BIRES_EINVAL;
  if (jb.var != BIRES_VAR_X && jb.var != BIRES_VAR_Y) return BIRES_EINVAL;
  int e = check_bipoly(&jb.f, 0);
  if (e) return e;
  if (jb.kind == BIRES_KIND_RESULTANT && (e = check_bipoly(&jb.g, 0))) return e;
  if (need_out && (!jb.out || jb.out->limbs < 1 || jb.out->degree < 0 || !jb.out->c)) return BIRES_EINVAL;
  return BIRES_OK;
}

#define DEV(x)                        \
  do {                                \
    if ((x) != hipSuccess) return BIRES_EDEVICE; \
  } while (0)

namespace {
// FNV-1a hash of the arguments of a device call sequence.
struct SeqHash {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <class T>
  void one(const T& v) {
    static_assert(std::is_arithmetic<T>::value || std::is_pointer<T>::value || std::is_enum<T>::value,
                  "hash scalars and pointers only");
    bytes(&v, sizeof v);
  }
  // a plain struct of pointers and counts, value-initialised (zero padding)
  void one(const FusedPlan& F) { bytes(&F, sizeof F); }
  template <class... A>
  void add(const A&... a) {
    (one(a), ...);
  }
};

// Host time per phase of a batched call (microseconds), accumulated into the
// context when timing is enabled.
struct HostClock {
  using C = std::chrono::steady_clock;
  bool on;
  C::time_point last;
  double us[BIRES_HOST_PHASES] = {0};
  explicit HostClock(bool enable) : on(enable), last(C::now()) {}
  void mark(int phase) {
    if (!on) return;
    const C::time_point t = C::now();
    us[phase] += std::chrono::duration<double, std::micro>(t - last).count();
    last = t;
  }
  void resume() {  // not counting the time since the last mark
    if (on) last = C::now();
  }
  void commit(Context* cx) {
    if (!on) return;
    std::lock_guard<std::mutex> lk(cx->timing_mu);
    for (int k = 0; k < BIRES_HOST_PHASES; ++k) cx->host_us[k] += us[k];
    cx->host_calls += 1;
  }
};

hipEvent_t take_event(Context* cx) {
  {
    std::lock_guard<std::mutex> lk(cx->ev_mu);
    if (!cx->ev_free.empty()) {
      hipEvent_t e = cx->ev_free.back();
      cx->ev_free.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void give_event(Context* cx, hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(cx->ev_mu);
  cx->ev_free.push_back(e);
}
}  // namespace

// State of a launched call until run_batch_finish: the jobs, the per-job
// work, the pool blocks the device work reads and writes, and the event that
// marks its end.
struct PendingBatch {
  Context* cx = nullptr;
  std::vector<JobIn> jobs;
  int mem = BIRES_MEM_DEVICE;
  hipStream_t st = nullptr;
  int32_t* status = nullptr;
  bool lock_stream = false;  // a rerun takes cx->stream_mu (calls on the library stream)
  bool in_flight = true;     // device work may still use the blocks
  HostClock hc;
  int nj = 0;
  std::vector<Work> w;
  std::vector<int32_t> rowdeg;  // per active job: the m + 1 row degrees of f, then the n + 1 of g
  std::vector<int> rd_off;
  bool spec = false, spec_ok = false, fused = false, timing = false;
  std::shared_ptr<DevImage> image;  // statistics the reused plans were made from
  size_t o_scan0 = 0, scan_words = 0;
  int32_t* h_flags = nullptr;
  long long schur_instances = 0;  // (prime, point) instances on the Schur kernel
  hipEvent_t ev0 = nullptr, ev1 = nullptr, done = nullptr;
  Held d_in, h_in, d_ws, h_meta, h_out;
  // allocation-free calls: device buffers in the library's fixed scratch
  // array, host staging in ordinary memory, completion by stream sync
  bool noalloc = false;
  std::vector<uint8_t> hv_in, hv_meta, hv_out;
  uint8_t* hout_base = nullptr;  // host output staging (pinned block or hv_out)
  explicit PendingBatch(bool clock) : hc(clock) {}
};

void PendingDeleter::operator()(PendingBatch* p) const {
  if (!p) return;
  if (p->in_flight && p->st) (void)hipStreamSynchronize(p->st);  // an error after queued work
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  give_event(p->cx, p->done);
  delete p;
}

namespace {

int launch_impl(Context* cx, const std::vector<JobIn>& jobs_in, int mem, hipStream_t st, int32_t* status,
                std::vector<uint32_t>* debug_values, std::vector<int>* debug_shape, PendingPtr* pending,
                bool noalloc = false) {
  if (mem != BIRES_MEM_HOST && mem != BIRES_MEM_DEVICE) return BIRES_EINVAL;
  if (noalloc && (debug_values || !cx->scratch)) return BIRES_EINVAL;
  PendingPtr P(new PendingBatch(cx->timing && debug_values == nullptr && !noalloc));
  P->noalloc = noalloc;
  P->cx = cx;
  P->jobs = jobs_in;
  P->mem = mem;
  P->st = st;
  P->status = status;
  const std::vector<JobIn>& jobs = P->jobs;
  HostClock& hc = P->hc;
  const int nj = P->nj = (int)jobs.size();
  const bool debug = debug_values != nullptr;
  std::vector<Work>& w = P->w;
  w.resize(nj);
  for (int i = 0; i < nj; ++i) {
    const JobIn& jb = jobs[i];
    w[i].status = validate(jb, !debug);
    if (w[i].status) continue;
    w[i].kind = jb.kind;
    w[i].derived = jb.kind != BIRES_KIND_RESULTANT;
    w[i].sf = shape_of(jb.f, jb.var);
    if (!w[i].derived) w[i].sg = shape_of(jb.g, jb.var);
  }
  auto nsrc = [&](int i) { return w[i].derived ? 1 : 2; };
  auto shp = [&](int i, int which) -> const Shape& { return which ? w[i].sg : w[i].sf; };

  // ---------------- inputs on the device, row statistics
  Layout in;
  std::vector<ScanTask> tasks;
  std::vector<int4> smap;
  for (int i = 0; i < nj; ++i) {
    if (w[i].status) continue;
    for (int which = 0; which < nsrc(i); ++which) {
      const Shape& s = shp(i, which);
      const size_t bytes = (size_t)s.rows * s.ld * s.L * 4;
      if (mem == BIRES_MEM_HOST || jobs[i].var == BIRES_VAR_X) w[i].o_in[which] = in.take(bytes);
    }
  }
  // scan outputs: read by the host from the pinned staging block
  const size_t o_scan0 = in.take(0);
  size_t o_scan_end = o_scan0;
  if (mem == BIRES_MEM_DEVICE) {
    for (int i = 0; i < nj; ++i) {
      if (w[i].status) continue;
      for (int which = 0; which < nsrc(i); ++which) {
        const Shape& s = shp(i, which);
        w[i].o_scan[which] = in.bytes;
        in.bytes += (size_t)s.rows * ROWSTAT_WORDS * 4;
        for (int r0 = 0; r0 < s.rows; r0 += 64) smap.push_back(make_int4((int)tasks.size(), r0, 0, 0));
        tasks.push_back(ScanTask{});
      }
    }
  }
  o_scan_end = in.bytes;
  const size_t o_tasks = in.take(sizeof(ScanTask) * tasks.size());
  const size_t o_smap = in.take(sizeof(int4) * smap.size());
  const size_t scan_words = (o_scan_end - o_scan0) / 4;
  P->o_scan0 = o_scan0;
  P->scan_words = scan_words;
  uint8_t *din = nullptr, *hin = nullptr;
  if (noalloc) {
    if (in.bytes > cx->scratch_bytes) return BIRES_ETOOBIG;
    din = cx->scratch;
    P->hv_in.resize(in.bytes);
    hin = P->hv_in.data();
  } else {
    P->d_in.take(&cx->dev, in.bytes);
    P->h_in.take(&cx->host, in.bytes);
    if (in.bytes && (!P->d_in.p || !P->h_in.p)) return BIRES_ENOMEM;
    din = P->d_in.b();
    hin = P->h_in.b();
  }
  // Plans reused from the previous call when it had the same descriptors and
  // the statistics have repeated; the scan still runs and a device check of
  // its output against the statistics of those plans decides, at the end,
  // whether the call stands or is rerun with fresh plans.
  SpecCache& sc = cx->spec;
  const bool spec_ok = P->spec_ok = cx->plan_cache && mem == BIRES_MEM_DEVICE && !debug && !noalloc && scan_words > 0;
  bool& spec = P->spec;
  std::vector<int32_t>& rowdeg = P->rowdeg;
  std::vector<int>& rd_off = P->rd_off;
  rd_off.assign(nj, 0);
  std::vector<SpecJob> reused;
  if (spec_ok) {
    std::lock_guard<std::mutex> lk(sc.mu);
    if (sc.valid && sc.conf >= 1 && sc.dimg && sc.image.size() == scan_words && sc.keys.size() == (size_t)nj) {
      spec = true;
      // cached plans come from calls where every job was valid
      for (int i = 0; i < nj && spec; ++i) spec = w[i].status == BIRES_OK && same_key(sc.keys[i], jobs[i]);
    }
    if (spec) {
      reused = sc.plans;
      rowdeg = sc.rowdeg;
      P->image = sc.dimg;
    }
  }

  if (mem == BIRES_MEM_HOST) {
    for (int i = 0; i < nj; ++i) {
      if (w[i].status) continue;
      for (int which = 0; which < nsrc(i); ++which) {
        const Shape& s = shp(i, which);
        uint32_t* h = (uint32_t*)(hin + w[i].o_in[which]);
        if (s.rows) pack_rect(which ? jobs[i].g : jobs[i].f, jobs[i].var, h);
        (which ? w[i].stg : w[i].stf) = scan_host(h, s.rows, s.ld, s.L);
        (which ? w[i].dev_g : w[i].dev_f) = (const uint32_t*)(din + w[i].o_in[which]);
      }
    }
    hc.mark(0);
    if (in.bytes) DEV(hipMemcpyAsync(din, hin, in.bytes, hipMemcpyHostToDevice, st));
    hc.mark(1);
  } else if (!tasks.empty()) {
    // The scan reads its task list from and writes its statistics to the
    // pinned staging block through its device mapping: no copies to wait on.
    // Allocation-free calls keep both in the device scratch and copy.
    uint8_t* hmap = nullptr;
    if (noalloc)
      hmap = din;
    else
      DEV(hipHostGetDevicePointer((void**)&hmap, hin, 0));
    int t = 0;
    for (int i = 0; i < nj; ++i) {
      if (w[i].status) continue;
      for (int which = 0; which < nsrc(i); ++which) {
        const bires_bipoly& p = which ? jobs[i].g : jobs[i].f;
        const Shape& s = shp(i, which);
        const uint32_t* src = p.c;
        if (jobs[i].var == BIRES_VAR_X && s.rows) {
          uint32_t* dst = (uint32_t*)(din + w[i].o_in[which]);
          launch_transpose(p.c, dst, p.deg_y + 1, p.deg_x + 1, p.limbs, st);
          src = dst;
        }
        (which ? w[i].dev_g : w[i].dev_f) = src;
        tasks[t++] = ScanTask{src, s.rows, s.ld, s.L, (int32_t*)(hmap + w[i].o_scan[which])};
      }
    }
    std::memcpy(hin + o_tasks, tasks.data(), sizeof(ScanTask) * tasks.size());
    std::memcpy(hin + o_smap, smap.data(), sizeof(int4) * smap.size());
    if (noalloc)
      DEV(hipMemcpyAsync(din + o_tasks, hin + o_tasks, o_smap + sizeof(int4) * smap.size() - o_tasks,
                         hipMemcpyHostToDevice, st));
    hc.mark(0);
    if (!smap.empty())
      launch_scan((const ScanTask*)(hmap + o_tasks), (const int4*)(hmap + o_smap), (int)smap.size(), st);
    hc.mark(1);
    if (!spec) {
      if (noalloc && scan_words)
        DEV(hipMemcpyAsync(hin + o_scan0, din + o_scan0, scan_words * 4, hipMemcpyDeviceToHost, st));
      DEV(hipStreamSynchronize(st));
      hc.mark(2);
      for (int i = 0; i < nj; ++i) {
        if (w[i].status) continue;
        for (int which = 0; which < nsrc(i); ++which) {
          const int rows = shp(i, which).rows;
          const int32_t* v = (const int32_t*)(hin + w[i].o_scan[which]);
          RowStats& rs = which ? w[i].stg : w[i].stf;
          rs.v.assign(v, v + ROWSTAT_WORDS * (size_t)rows);
        }
      }
    }
  }

  // ---------------- plans and output capacities
  if (spec) {
    for (int i = 0; i < nj; ++i) {
      Work& x = w[i];
      const SpecJob& c = reused[i];
      x.status = c.status;
      x.active = c.active;
      x.pl = c.pl;
      x.Lout = c.Lout;
      x.degcap = c.degcap;
      x.Tf = c.Tf;
      x.Tg = c.Tg;
      x.ldg = c.ldg;
      x.Lacc = c.Lacc;
      rd_off[i] = c.rd_off;
    }
  }
  for (int i = 0; i < nj && !spec; ++i) {
    Work& x = w[i];
    if (x.status) continue;
    if (x.derived && (x.status = derive_operand_stats(x.kind, x.stf, x.stg))) continue;
    if ((x.status = make_plan(x.stf, x.stg, x.pl))) continue;
    if (x.pl.kind_special == 0 &&
        (x.pl.D > MAX_POINTS || interp_lds_words(x.pl.D) * 4 > cx->lds_per_block ||
         eval_elim_lds_bytes(x.pl.m + x.pl.n + 2, (x.pl.m + 1) * pad4(x.sf.ld) +
                                                      (x.pl.n + 1) * pad4(x.derived ? x.sf.ld : x.sg.ld)) >
             cx->lds_per_block)) {
      x.status = BIRES_ETOOBIG;
      continue;
    }
    const int need_limbs = x.pl.kind_special ? 1 : limbs_for_log2(x.pl.log2B);
    if (!debug) {
      bires_upoly* o = jobs[i].out;
      if (o->degree < x.pl.D - 1 || o->limbs < need_limbs) {
        o->degree = std::max(o->degree, x.pl.D - 1);
        o->limbs = std::max(o->limbs, need_limbs);
        x.status = BIRES_EBUFSIZE;
        continue;
      }
      x.degcap = o->degree;
      x.Lout = o->limbs;
    }
    x.active = x.pl.kind_special == 0;
    if (x.active) {
      x.ldg = x.derived ? x.sf.ld : x.sg.ld;
      x.Tf = (x.pl.m + 1) * pad4(x.sf.ld);
      x.Tg = (x.pl.n + 1) * pad4(x.ldg);
      x.Lacc = std::min(x.Lout, x.pl.P + 1);
      rd_off[i] = (int)rowdeg.size();
      for (int j = 0; j <= x.pl.m; ++j) rowdeg.push_back(x.stf.deg(j));
      for (int j = 0; j <= x.pl.n; ++j) rowdeg.push_back(x.stg.deg(j));
    }
  }

  // ---------------- workspace: device buffers, then the uploaded metadata block
  Layout ws;
  Layout hout;  // host staging of outputs (host memory space only)
  // per-kernel first block of each job (prefix sums of the per-job block counts)
  // eval_elim runs one launch per size bucket (LDS per block sized for the
  // bucket, so small jobs are not held to the occupancy of the largest)
  // jobs whose f array fits in registers (eval_elim_rg_capacity 24, 32 or 64)
  // run in three more launches
  // jobs on the Schur kernel (wave per instance; 1 or 2 generator rows per
  // lane) in two more
  enum {
    K_RED, K_IP, K_MRC, K_SUM, K_CAR, K_CRT, K_EE0, NBUCKET = 5, K_RG0 = K_EE0 + NBUCKET, NRG = 3,
    K_SC0 = K_RG0 + NRG, NSC = 2, NK = K_SC0 + NSC
  };
  const int bucket_words[NBUCKET] = {24, 40, 64, 96, 1 << 30};
  const int rg_cap[NRG] = {24, 32, 64};
  int bw[NBUCKET] = {0}, br_[NBUCKET] = {0};
  int rdeg[NRG] = {0}, rw[NRG] = {0};
  int sw[NSC] = {0};
  std::vector<int> starts[NK];
  for (auto& v : starts) v.assign(nj + 1, 0);
  // the schedule: from the autotuner's table for the batch's size key
  long long instances = 0;
  int max_r = 0, keyP = 1;
  for (int i = 0; i < nj; ++i)
    if (!w[i].status && w[i].active) {
      instances += (long long)w[i].pl.P * w[i].pl.D;
      max_r = std::max(max_r, w[i].pl.m + w[i].pl.n);
      keyP = std::max(keyP, w[i].pl.P);
    }
  const std::string key = tune_key(instances, max_r, keyP);
  {
    std::lock_guard<std::mutex> lk(cx->tune_mu);
    cx->last_key = key;
  }
  const int sched = (debug || noalloc || instances == 0) ? BIRES_SCHEDULE_STAGED : schedule_for(cx, key);
  const bool schur = cx->eval_mode == BIRES_EVAL_SCHUR || sched == BIRES_SCHEDULE_SCHUR;
  int maxP = 1, maxD = 1;
  for (int i = 0; i < nj; ++i) {
    Work& x = w[i];
    if (x.status || !x.active) continue;
    const Plan& p = x.pl;
    x.o_res_f = ws.take((size_t)p.P * x.Tf * 4);
    x.o_res_g = ws.take((size_t)p.P * x.Tg * 4);
    (void)ws.take(128);  // whole-chunk loads of the evaluation may read past the last row
    x.o_vals = ws.take((size_t)p.P * p.D * 4);
    if (!debug) {
      x.o_coefs = ws.take((size_t)p.P * p.D * 4);
      x.o_digits = ws.take((size_t)p.P * p.D * 4);
      x.o_neg = ws.take((size_t)p.D * 4);
      x.o_acc_lo = ws.take((size_t)p.D * x.Lacc * 8);
      x.o_acc_hi = ws.take((size_t)p.D * x.Lacc * 4);
      if (mem == BIRES_MEM_HOST) {
        x.o_out = ws.take((size_t)(x.degcap + 1) * x.Lout * 4);
        x.o_hout = hout.take((size_t)(x.degcap + 1) * x.Lout * 4);
      }
    }
    maxP = std::max(maxP, p.P);
    maxD = std::max(maxD, p.D);
    starts[K_RED][i + 1] = (x.Tf + 63) / 64 + (x.Tg + 63) / 64;
    const int nr = schur ? schur_rows_per_lane(p.m, p.n) : 0;
    const int rc = cx->eval_mode == BIRES_EVAL_AUTO ? eval_elim_rg_capacity(p.m, p.n) : 0;
    if (nr) {
      starts[K_SC0 + nr - 1][i + 1] = p.P * p.D;
      sw[nr - 1] = std::max(sw[nr - 1], p.m + p.n + 2);
    } else if (rc) {
      const int r = rc == rg_cap[0] ? 0 : rc == rg_cap[1] ? 1 : 2;
      starts[K_RG0 + r][i + 1] = p.P * ((p.D + 63) / 64);
      rdeg[r] = std::max(rdeg[r], std::max(p.m, p.n));
      rw[r] = std::max(rw[r], p.m + p.n + 2);
    } else {
      int bk = 0;
      while (p.m + p.n + 2 > bucket_words[bk]) ++bk;
      starts[K_EE0 + bk][i + 1] = p.P * ((p.D + 63) / 64);
      bw[bk] = std::max(bw[bk], p.m + p.n + 2);
      br_[bk] = std::max(br_[bk], x.Tf + x.Tg);
    }
    starts[K_IP][i + 1] = p.P;
    starts[K_MRC][i + 1] = p.D;  // Garner: one wave per coefficient
    starts[K_SUM][i + 1] = (p.D * x.Lacc + 255) / 256;
    starts[K_CAR][i + 1] = debug ? 0 : (x.degcap + 1 + 63) / 64;
    // coefficients below D (the blocks also write the zero ones above them);
    // divided below by the rows per block, which depend on the largest prime
    // count
    starts[K_CRT][i + 1] = debug ? 0 : std::min(p.D, x.degcap + 1);
  }
  {
    const int rows = crt_rows_per_block(maxP);
    for (int i = 0; i < nj; ++i) starts[K_CRT][i + 1] = (starts[K_CRT][i + 1] + rows - 1) / rows;
  }
  int maxLcap = 1;
  for (int i = 0; i < nj; ++i)
    if (!w[i].status && w[i].active) maxLcap = std::max(maxLcap, w[i].Lout);
  for (auto& v : starts)
    for (int i = 0; i < nj; ++i) v[i + 1] += v[i];
  const bool fused = P->fused = sched == BIRES_SCHEDULE_FUSED;
  if (!fused && !debug) P->schur_instances = (long long)starts[K_SC0][nj] + starts[K_SC0 + 1][nj];
  // explicit CRT straight to limbs when the prime counts allow
  std::vector<std::pair<const uint32_t*, int>> crt(nj, {nullptr, 0});
  bool use_crt = !debug && crt_ok(maxP);
  int lastP = -1, lastLM = 0;
  const uint32_t* lastd = nullptr;
  for (int i = 0; i < nj && use_crt; ++i) {
    if (w[i].status || !w[i].active) continue;
    if (w[i].pl.P != lastP) {  // consecutive jobs mostly share P
      lastP = w[i].pl.P;
      // allocation-free calls use only operand tables that already exist
      lastd = noalloc ? crt_device_cached(cx, lastP, &lastLM) : crt_device(cx, lastP, &lastLM);
    }
    if (!lastd) use_crt = false;
    crt[i] = {lastd, lastLM};
  }
  // (the fused launch's CRT blocks have 32 rows)
  if (use_crt && (fused ? crt_lds_bytes_rows(maxLcap, maxP, 32) : crt_lds_bytes(maxLcap, maxP)) > cx->lds_per_block)
    use_crt = false;
  // interpolation on the matrix cores when at least 32 jobs share D and P
  // (all active jobs of the batch)
  std::vector<int> group;
  int gD = 0, gP = 0;
  for (int i = 0; i < nj && !debug && !noalloc; ++i) {
    if (w[i].status || !w[i].active) continue;
    if (group.empty()) {
      gD = w[i].pl.D;
      gP = w[i].pl.P;
    } else if (w[i].pl.D != gD || w[i].pl.P != gP) {
      group.clear();
      break;
    }
    group.push_back(i);
  }
  const int8_t* vinv = nullptr;
  if ((int)group.size() >= 32 && gD <= 4096) vinv = vinv_device(cx, gD, gP, st);
  if (!vinv) group.clear();
  // the per-(job, prime) interpolation kernel reads its block tables
  const uint32_t *itW = nullptr, *itQ = nullptr;
  int itNB = 0;
  if (group.empty() && !debug && !noalloc &&
      !interp_tables_device(cx, interp_table_blocks(maxD), maxP, st, &itW, &itQ, &itNB)) {
    itW = itQ = nullptr;
    itNB = 0;
  }
  const int gDp = (gD + 31) & ~31, gNp = ((int)group.size() + 31) & ~31;
  const size_t o_yp = group.empty() ? 0 : ws.take((size_t)4 * gNp * gDp * gP);
  // persistent fused launch: the evaluation's block lists (register Euclid at
  // the batch's capacity fC, LDS kernel), the CRT's blocks of 32 rows
  int fC = 0, fKS = 6, f_rgdeg = 0, f_rgw = 0, f_eew = 0;
  std::vector<int> fst_rg, fst_ee, fst_crt;
  if (fused) {
    fst_rg.assign(nj + 1, 0);
    fst_ee.assign(nj + 1, 0);
    fst_crt.assign(nj + 1, 0);
    auto cap = [&](const Plan& p) {
      return cx->eval_mode == BIRES_EVAL_AUTO ? fused_capacity(eval_elim_rg_capacity(p.m, p.n)) : 0;
    };
    for (int i = 0; i < nj; ++i)
      if (!w[i].status && w[i].active) fC = std::max(fC, cap(w[i].pl));
    for (int i = 0; i < nj; ++i) {
      const Work& x = w[i];
      if (x.status || !x.active) continue;
      const Plan& p = x.pl;
      const int nb = p.P * ((p.D + 63) / 64);
      if (cap(p)) {
        fst_rg[i + 1] = nb;
        f_rgdeg = std::max(f_rgdeg, std::max(p.m, p.n));
        f_rgw = std::max(f_rgw, p.m + p.n + 2);
      } else {
        fst_ee[i + 1] = nb;
        f_eew = std::max(f_eew, p.m + p.n + 2);
      }
      fst_crt[i + 1] = (std::min(p.D, x.degcap + 1) + 31) / 32;
    }
    for (std::vector<int>* v : {&fst_rg, &fst_ee, &fst_crt})
      for (int i = 0; i < nj; ++i) (*v)[i + 1] += (*v)[i];
    fKS = fused_crt_steps(maxP);
  }
  const size_t o_ffbq = ws.take(sizeof(int) * (fused ? (size_t)fst_rg[nj] : 0));
  size_t o_fbq[NRG];  // queues of blocks recomputed by the LDS kernel
  for (int r = 0; r < NRG; ++r) o_fbq[r] = ws.take(sizeof(int) * (size_t)starts[K_RG0 + r][nj]);
  // metadata uploaded with one copy: descriptors, flags, row degrees, block maps
  const size_t meta_begin = ws.take(0);
  const size_t o_jobs = ws.take(sizeof(JobDev) * (size_t)nj);
  // [deg_out, err] per job, fused error, statistics mismatch of reused plans
  // per job (degree, error), then the fused error, the statistics check and
  // the Schur kernel's fallback count
  const size_t o_flags = ws.take(sizeof(int32_t) * (2 * (size_t)nj + 3));
  const size_t o_fbc = ws.take(sizeof(int) * NRG);                         // queue lengths, uploaded as zero
  for (int i = 0; i < nj; ++i)
    if (!w[i].status && w[i].active) w[i].o_rowdeg = ws.take((size_t)(w[i].pl.m + w[i].pl.n + 2) * 4);
  const size_t o_maps = ws.take(sizeof(int) * (size_t)NK * (nj + 1));
  // the group's coefs pointers
  const size_t o_gco = ws.take(sizeof(uint32_t*) * group.size());
  // the fused launch's block maps (register Euclid, LDS kernel, CRT) and its
  // claim and completion counters (uploaded as zero)
  enum { F_CTR = 6 * FUSED_STAGE_INTS };
  const size_t o_fst = ws.take(sizeof(int) * (fused ? 3 * (size_t)(nj + 1) : 0));
  const size_t o_fctr = ws.take(sizeof(int) * (fused ? F_CTR : 0));
  const size_t meta_end = ws.bytes;
  uint8_t* D0 = nullptr;
  uint8_t* H0 = nullptr;  // H0 + offset addresses the metadata image
  if (noalloc) {
    // the workspace follows the input region in the scratch array
    const size_t base = (in.bytes + 255) & ~(size_t)255;
    if (base + ws.bytes > cx->scratch_bytes) return BIRES_ETOOBIG;
    D0 = cx->scratch + base;
    P->hv_meta.resize(meta_end - meta_begin);
    P->hv_out.resize(hout.bytes);
    H0 = P->hv_meta.data() - meta_begin;
    P->hout_base = P->hv_out.data();
  } else {
    P->d_ws.take(&cx->dev, ws.bytes);
    P->h_meta.take(&cx->host, meta_end - meta_begin);
    P->h_out.take(&cx->host, hout.bytes);
    if ((ws.bytes && !P->d_ws.p) || (meta_end > meta_begin && !P->h_meta.p) || (hout.bytes && !P->h_out.p))
      return BIRES_ENOMEM;
    D0 = P->d_ws.b();
    H0 = P->h_meta.b() - meta_begin;
    P->hout_base = P->h_out.b();
  }
  uint8_t* const hob = P->hout_base;

  int32_t* h_flags = P->h_flags = (int32_t*)(H0 + o_flags);
  std::memset(H0 + o_fbc, 0, sizeof(int) * NRG);
  JobDev* h_jobs = (JobDev*)(H0 + o_jobs);
  for (int i = 0; i < nj; ++i) {
    h_flags[2 * i] = -1;
    h_flags[2 * i + 1] = 0;
    if (i == nj - 1) h_flags[2 * nj] = h_flags[2 * nj + 1] = h_flags[2 * nj + 2] = 0;
    h_jobs[i] = JobDev{};
    Work& x = w[i];
    if (x.status || !x.active) continue;
    const Plan& p = x.pl;
    JobDev& J = h_jobs[i];
    J.limbs_f = x.dev_f;
    J.limbs_g = x.derived ? nullptr : x.dev_g;
    J.Lf = x.sf.L;
    J.Lg = x.derived ? x.sf.L : x.sg.L;
    J.ldf = x.sf.ld;
    J.ldg = x.ldg;
    J.m = p.m;
    J.n = p.n;
    J.kind = x.kind;
    J.P = p.P;
    J.D = p.D;
    J.lpf = pad4(x.sf.ld);
    J.lpg = pad4(x.ldg);
    J.Tf = x.Tf;
    J.Tg = x.Tg;
    int32_t* rd = (int32_t*)(H0 + x.o_rowdeg);
    std::memcpy(rd, rowdeg.data() + rd_off[i], sizeof(int32_t) * (size_t)(p.m + p.n + 2));
    J.rowdeg_f = (const int32_t*)(D0 + x.o_rowdeg);
    J.rowdeg_g = J.rowdeg_f + p.m + 1;
    J.res_f = (uint32_t*)(D0 + x.o_res_f);
    J.res_g = (uint32_t*)(D0 + x.o_res_g);
    J.vals = (uint32_t*)(D0 + x.o_vals);
    if (!debug) {
      J.coefs = (uint32_t*)(D0 + x.o_coefs);
      J.digits = (uint32_t*)(D0 + x.o_digits);
      J.negflag = (int32_t*)(D0 + x.o_neg);
      J.acc_lo = (uint64_t*)(D0 + x.o_acc_lo);
      J.acc_hi = (uint32_t*)(D0 + x.o_acc_hi);
      J.Lacc = x.Lacc;
      J.out = mem == BIRES_MEM_HOST ? (uint32_t*)(D0 + x.o_out) : jobs[i].out->c;
      J.Lcap = x.Lout;
      J.degcap = x.degcap;
    }
    J.crt = crt[i].first;
    J.crt_LM = crt[i].second;
    J.deg_out = (int32_t*)(D0 + o_flags) + 2 * i;
    J.err = (int32_t*)(D0 + o_flags) + 2 * i + 1;
  }
  int* hm = (int*)(H0 + o_maps);
  const int* dm = (const int*)(D0 + o_maps);
  for (int kk = 0; kk < NK; ++kk) std::memcpy(hm + (size_t)kk * (nj + 1), starts[kk].data(), sizeof(int) * (nj + 1));
  auto st_of = [&](int kk) { return dm + (size_t)kk * (nj + 1); };
  if (!group.empty()) {
    uint32_t** gco = (uint32_t**)(H0 + o_gco);
    for (size_t n = 0; n < group.size(); ++n) {
      gco[n] = (uint32_t*)(D0 + w[group[n]].o_coefs);
      // the evaluation writes this job's values into column n of the digit planes
      JobDev& J = h_jobs[group[n]];
      J.yp = (int8_t*)(D0 + o_yp);
      J.ycol = (int)n;
      J.ynp = gNp;
      J.ydp = gDp;
    }
  }
  if (fused) {
    std::memcpy(H0 + o_fst, fst_rg.data(), sizeof(int) * (nj + 1));
    std::memcpy(H0 + o_fst + sizeof(int) * (nj + 1), fst_ee.data(), sizeof(int) * (nj + 1));
    std::memcpy(H0 + o_fst + sizeof(int) * 2 * (nj + 1), fst_crt.data(), sizeof(int) * (nj + 1));
    std::memset(H0 + o_fctr, 0, sizeof(int) * F_CTR);
  }
  auto nb_of = [&](int kk) { return starts[kk][nj]; };
  hc.mark(3);
  // special results of device-memory outputs are written on the stream
  // (outside any captured graph: memset nodes are not used in graphs)
  for (int i = 0; i < nj && !debug; ++i) {
    const Work& x = w[i];
    if (x.status || x.active || mem != BIRES_MEM_DEVICE) continue;
    bires_upoly* o = jobs[i].out;
    DEV(hipMemsetAsync(o->c, 0, (size_t)(x.degcap + 1) * x.Lout * 4, st));
    if (x.pl.kind_special == 2) {
      static const uint32_t one = 1u;
      DEV(hipMemcpyAsync(o->c, &one, 4, hipMemcpyHostToDevice, st));
    }
  }
  const JobDev* d_jobs = (const JobDev*)(D0 + o_jobs);
  int nb_ee = 0;
  for (int bk = 0; bk < NBUCKET + NRG + NSC; ++bk) nb_ee += nb_of(K_EE0 + bk);

  // The device sequence of the call: metadata upload, kernels, result copies.
  // seq(run, sig) hashes every argument of every call into sig and, with
  // run, issues the calls; a graph captured from one issue is valid for any
  // later call with the same hash.
  FusedPlan F{};
  size_t f_lds = 0;
  int f_blocks = 0;
  if (fused) {
    const int* fm = (const int*)(D0 + o_fst);
    F.jobs = d_jobs;
    F.nj = nj;
    F.st_rg = fm;
    F.st_ee = fm + (nj + 1);
    F.n_rg = fst_rg[nj];
    F.n_ee = fst_ee[nj];
    F.fb_count = (int*)(D0 + o_fbc);
    F.fb_queue = (int*)(D0 + o_ffbq);
    size_t block_lds;
    int demand;  // blocks that the largest stage can use
    if (!group.empty()) {
      F.im = 1;
      F.n_im = ((gDp / 32 + 1) / 2) * (gNp / 32) * gP;  // blocks of 64 coefficients x 32 jobs
      F.gco = (uint32_t* const*)(D0 + o_gco);
      F.gN = (int)group.size();
      F.gNp = gNp;
      F.gD = gD;
      F.gDp = gDp;
      F.Ap = vinv;
      F.Yp = (const int8_t*)(D0 + o_yp);
      block_lds = fused_interp_lds_bytes();
      demand = F.n_im;
    } else {
      F.st_ip = st_of(K_IP);
      F.n_ip = nb_of(K_IP);
      F.itW = itW;
      F.itQ = itQ;
      F.itNB = itNB;
      block_lds = interp_lds_words(maxD) * 4;
      demand = F.n_ip;
    }
    // LDS words of a wave's slice per wave stage (multiples of 4)
    int lw[4] = {std::max(f_rgdeg + 1, f_eew) * 64, f_rgw * 64, 0, 0};
    if (use_crt) {
      F.crt = 1;
      F.st_crt = fm + 2 * (nj + 1);
      F.n_crt = fst_crt[nj];
      F.sld = crt_row_stride(maxLcap);
      F.cps = crt_const_stride(maxP);
      lw[2] = (int)(crt_lds_bytes_rows(maxLcap, maxP, 32) / 4);
    } else {
      F.st_mrc = st_of(K_MRC);
      F.n_mrc = nb_of(K_MRC);
      F.st_sum = st_of(K_SUM);
      F.n_sum = nb_of(K_SUM);
      F.st_car = st_of(K_CAR);
      F.n_car = nb_of(K_CAR);
      F.stage_ld = maxLcap <= 128 ? maxLcap + 1 : 0;
      lw[2] = 2 * maxP;
      lw[3] = 64 * F.stage_ld;
      demand = std::max(demand, F.n_sum);
    }
    // the LDS per block that the register budget's occupancy leaves (blocks
    // per CU without LDS); each wave stage as many waves of a block as their
    // slices fit in it, at least one
    const int occ = fused_blocks_per_cu(fC, fKS, 0);
    if (occ <= 0) return BIRES_EDEVICE;
    const size_t target = (cx->lds_per_cu / occ) & ~(size_t)15;
    const int wave_tasks[4] = {F.n_rg + F.n_ee, F.n_rg, F.crt ? F.n_crt : F.n_mrc, F.n_car};
    f_lds = block_lds;
    for (int k = 0; k < 4; ++k) {
      F.lw[k] = (lw[k] + 3) & ~3;
      const size_t b = (size_t)F.lw[k] * 4;
      F.wv[k] = b ? (int)std::max<size_t>(1, std::min<size_t>(4, target / b)) : 4;
      f_lds = std::max(f_lds, F.wv[k] * b);
      demand = std::max(demand, (wave_tasks[k] + F.wv[k] - 1) / F.wv[k]);
    }
    if (f_lds > cx->lds_per_block) return BIRES_ETOOBIG;
    F.ctr = (int*)(D0 + o_fctr);
    F.err = (int*)(D0 + o_flags) + 2 * nj;
    const int per_cu = fused_blocks_per_cu(fC, fKS, f_lds);
    if (per_cu <= 0) return BIRES_EDEVICE;
    // as many blocks as the device holds at once (blocks that start late find
    // the tasks taken)
    f_blocks = std::min(per_cu * cx->compute_units, std::max(1, demand));
    // tasks per claim: about eight claims per wave (or block) and stage
    auto per_claim = [&](long long tasks, long long takers) {
      return (int)std::max<long long>(1, std::min<long long>(32, tasks / (8 * takers)));
    };
    F.kc[0] = per_claim(F.n_rg + F.n_ee, (long long)f_blocks * F.wv[0]);
    F.kc[1] = 1;
    F.kc[2] = per_claim(F.im ? F.n_im : F.n_ip, f_blocks);
    F.kc[3] = per_claim(F.crt ? F.n_crt : F.n_mrc, (long long)f_blocks * F.wv[2]);
    F.kc[4] = per_claim(F.n_sum, f_blocks);
    F.kc[5] = per_claim(F.n_car, (long long)f_blocks * F.wv[3]);
  }
  const bool use_graph = cx->graphs && !debug && !noalloc;
  const bool timing = P->timing = cx->timing && nb_ee > 0 && !use_graph;
  if (timing) {
    DEV(hipEventCreate(&P->ev0));
    DEV(hipEventCreate(&P->ev1));
  }
  const hipEvent_t ev0 = P->ev0, ev1 = P->ev1;
  const int32_t* const d_image = spec ? P->image->d : nullptr;
  const int32_t* spec_got = nullptr;
  if (spec) {
    uint8_t* hmap = nullptr;
    DEV(hipHostGetDevicePointer((void**)&hmap, hin, 0));
    spec_got = (const int32_t*)(hmap + o_scan0);
  }
  // the metadata block is uploaded by a kernel that reads it through the
  // pinned block's device mapping (all its regions are whole words)
  // (allocation-free calls copy it from ordinary host memory)
  const uint32_t* meta_mapped = nullptr;
  if (meta_end > meta_begin && !noalloc) {
    uint8_t* m = nullptr;
    DEV(hipHostGetDevicePointer((void**)&m, P->h_meta.p, 0));
    meta_mapped = (const uint32_t*)m;
  }
  auto seq = [&](bool run, SeqHash& sg) -> int {
    sg.add(st, D0, meta_begin, meta_end, (const void*)meta_mapped);
    if (run && meta_end > meta_begin) {
      if (noalloc)
        DEV(hipMemcpyAsync(D0 + meta_begin, H0 + meta_begin, meta_end - meta_begin, hipMemcpyHostToDevice, st));
      else
        launch_upload(meta_mapped, (uint32_t*)(D0 + meta_begin), (long long)((meta_end - meta_begin) / 4), st);
    }
    if (spec) {
      sg.add((const void*)spec_got, (const void*)d_image, scan_words);
      if (run)
        launch_stats_check(spec_got, d_image, (long long)scan_words, (int*)(D0 + o_flags) + 2 * nj + 1, st);
    }
    if (fused) {
      // the reduction in a launch of its own: the evaluation reads its
      // residues through the scalar cache
      sg.add(nb_of(K_RED), maxP);
      if (run && nb_of(K_RED)) launch_reduce(d_jobs, st_of(K_RED), nj, nb_of(K_RED), maxP, cx->tab, st);
      sg.add(F, fC, fKS, f_lds, f_blocks);
      if (run && timing) DEV(hipEventRecord(ev0, st));
      if (run) launch_fused(fC, fKS, F, f_lds, f_blocks, cx->tab, st);
      if (run && timing) DEV(hipEventRecord(ev1, st));
    } else {
      sg.add(nb_of(K_RED), maxP);
      if (run && nb_of(K_RED)) launch_reduce(d_jobs, st_of(K_RED), nj, nb_of(K_RED), maxP, cx->tab, st);
      if (run && timing) DEV(hipEventRecord(ev0, st));
      for (int bk = 0; bk < NBUCKET; ++bk) {
        sg.add(nb_of(K_EE0 + bk), bw[bk], br_[bk]);
        if (run && nb_of(K_EE0 + bk))
          launch_eval_elim(d_jobs, st_of(K_EE0 + bk), nj, nb_of(K_EE0 + bk), bw[bk], br_[bk], cx->tab, st);
      }
      for (int r = 0; r < NRG; ++r) {
        sg.add(nb_of(K_RG0 + r), rdeg[r], rw[r], o_fbc, o_fbq[r]);
        if (run && nb_of(K_RG0 + r))
          launch_eval_elim_rg(rg_cap[r], d_jobs, st_of(K_RG0 + r), nj, nb_of(K_RG0 + r), rdeg[r], rw[r],
                              (int*)(D0 + o_fbc) + r, (int*)(D0 + o_fbq[r]), cx->tab, st);
      }
      for (int r = 0; r < NSC; ++r) {
        sg.add(nb_of(K_SC0 + r), sw[r]);
        if (run && nb_of(K_SC0 + r))
          launch_schur(r + 1, d_jobs, st_of(K_SC0 + r), nj, nb_of(K_SC0 + r), sw[r],
                       (int*)(D0 + o_flags) + 2 * nj + 2, cx->tab, st);
      }
      if (run && timing) DEV(hipEventRecord(ev1, st));
      if (!debug) {
        sg.add((const void*)itW, (const void*)itQ, itNB);
        sg.add((int)group.size(), gD, gP, (const void*)vinv, o_yp, o_gco, nb_of(K_IP), maxD, use_crt, nb_of(K_CAR),
               nb_of(K_CRT), maxLcap, nb_of(K_MRC), nb_of(K_SUM));
        if (run) {
          if (!group.empty())
            launch_interp_mfma((uint32_t* const*)(D0 + o_gco), (int)group.size(), gD, gP, vinv,
                               (const int8_t*)(D0 + o_yp), cx->tab, st);
          else if (nb_of(K_IP))
            launch_interp(d_jobs, st_of(K_IP), nj, nb_of(K_IP), maxD, cx->tab, itW, itQ, itNB, st);
          if (use_crt) {
            // residues to limbs in one pass over the output capacity
            if (nb_of(K_CRT)) launch_crt(d_jobs, st_of(K_CRT), nj, nb_of(K_CRT), maxP, maxLcap, cx->tab, st);
          } else {
            if (nb_of(K_MRC)) launch_mrc(d_jobs, st_of(K_MRC), nj, nb_of(K_MRC), maxP, cx->tab, st);
            if (nb_of(K_SUM)) launch_limbs_sum(d_jobs, st_of(K_SUM), nj, nb_of(K_SUM), cx->tab, st);
            if (nb_of(K_CAR)) launch_limbs_carry(d_jobs, st_of(K_CAR), nj, nb_of(K_CAR), maxLcap, st);
          }
        }
      }
    }
    if (run) DEV(hipGetLastError());
    if (debug) return BIRES_OK;
    sg.add(nj, o_flags, (const void*)h_flags);
    if (run && nj)
      DEV(hipMemcpyAsync(h_flags, D0 + o_flags, sizeof(int32_t) * (2 * nj + 3), hipMemcpyDeviceToHost, st));
    for (int i = 0; i < nj; ++i) {
      const Work& x = w[i];
      if (x.status || !x.active || mem != BIRES_MEM_HOST) continue;
      sg.add(i, (const void*)hob, x.o_hout, x.o_out, x.degcap, x.Lout);
      if (run)
        DEV(hipMemcpyAsync(hob + x.o_hout, D0 + x.o_out, (size_t)(x.degcap + 1) * x.Lout * 4,
                           hipMemcpyDeviceToHost, st));
    }
    return BIRES_OK;
  };
  if (use_graph) {
    SeqHash sig;
    (void)seq(false, sig);
    bool launched = graph_launch(cx, sig.h, st);
    if (!launched) {
      // capture one issue of the sequence, then launch it as a graph
      SeqHash again;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int e = seq(true, again);
        hipGraph_t g = nullptr;
        hipGraphExec_t exec = nullptr;
        const bool ended = hipStreamEndCapture(st, &g) == hipSuccess;
        if (e == BIRES_OK && ended && g && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess)
          launched = graph_store_launch(cx, sig.h, exec, st);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
      }
    }
    if (!launched) {  // capture unavailable: issue the calls directly
      SeqHash unused;
      const int e = seq(true, unused);
      if (e) return e;
    }
  } else {
    SeqHash unused;
    const int e = seq(true, unused);
    if (e) return e;
  }

  if (debug) {
    const Work& x = w[0];
    if (x.status) return x.status;
    if (!x.active) return BIRES_EINVAL;
    debug_values->resize((size_t)x.pl.P * x.pl.D);
    debug_shape->assign({x.pl.P, x.pl.D});
    DEV(hipMemcpyAsync(debug_values->data(), D0 + x.o_vals, debug_values->size() * 4, hipMemcpyDeviceToHost, st));
    DEV(hipStreamSynchronize(st));
    P->in_flight = false;
    return BIRES_OK;
  }
  if (!noalloc) {
    P->done = take_event(cx);
    if (!P->done) return BIRES_EDEVICE;
    DEV(hipEventRecord(P->done, st));
  }
  hc.mark(4);
  *pending = std::move(P);
  return BIRES_OK;
}

}  // namespace

int run_batch_launch(Context* cx, const std::vector<JobIn>& jobs, int mem, hipStream_t st, int32_t* status,
                     PendingPtr* pending) {
  pending->reset();
  return launch_impl(cx, jobs, mem, st, status, nullptr, nullptr, pending);
}

void set_pending_stream_lock(PendingBatch* pending) {
  if (pending) pending->lock_stream = true;
}

int run_batch_finish(PendingPtr P) {
  if (!P) return BIRES_EINVAL;
  Context* cx = P->cx;
  const std::vector<JobIn>& jobs = P->jobs;
  const int mem = P->mem;
  const int nj = P->nj;
  std::vector<Work>& w = P->w;
  HostClock& hc = P->hc;
  const int32_t* h_flags = P->h_flags;
  const size_t scan_words = P->scan_words;
  SpecCache& sc = cx->spec;
  hc.resume();
  if (P->noalloc)
    DEV(hipStreamSynchronize(P->st));
  else
    DEV(hipEventSynchronize(P->done));
  P->in_flight = false;
  if (P->timing) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P->ev0, P->ev1) == hipSuccess) {
      std::lock_guard<std::mutex> lk(cx->timing_mu);
      cx->kernel_ms += ms;
      cx->kernel_launches += 1;
    }
  }
  if (P->spec) {
    if (h_flags[2 * nj + 1]) {
      // the statistics changed: drop the cache and rerun with fresh plans
      {
        std::lock_guard<std::mutex> lk(sc.mu);
        sc.valid = false;
        sc.conf = 0;
        sc.misses++;
      }
      const std::vector<JobIn> again = std::move(P->jobs);
      hipStream_t st = P->st;
      int32_t* status = P->status;
      const bool lock_stream = P->lock_stream;
      P.reset();
      if (!lock_stream) return run_batch(cx, again, mem, st, status);
      std::lock_guard<std::mutex> lk(cx->stream_mu);
      return run_batch(cx, again, mem, st, status);
    }
    std::lock_guard<std::mutex> lk(sc.mu);
    sc.hits++;
  } else if (P->spec_ok) {
    int bad = 0;
    for (int i = 0; i < nj; ++i) bad |= w[i].status;
    const int32_t* img = (const int32_t*)(P->h_in.b() + P->o_scan0);
    std::lock_guard<std::mutex> lk(sc.mu);
    bool same = sc.valid && sc.image.size() == scan_words && sc.keys.size() == (size_t)nj &&
                std::memcmp(sc.image.data(), img, scan_words * 4) == 0;
    for (int i = 0; i < nj && same; ++i) same = same_key(sc.keys[i], jobs[i]);
    if (bad) {
      sc.valid = false;  // output-size errors rewrite descriptors: plan those calls afresh
      sc.conf = 0;
    } else {
      sc.conf = same ? sc.conf + 1 : 0;
      if (!same) {
        sc.keys.resize(nj);
        for (int i = 0; i < nj; ++i) sc.keys[i] = key_of(jobs[i]);
        sc.image.assign(img, img + scan_words);
        sc.plans.resize(nj);
        for (int i = 0; i < nj; ++i) {
          const Work& x = w[i];
          sc.plans[i] =
              SpecJob{x.status, x.active, x.pl, x.Lout, x.degcap, x.Tf, x.Tg, x.ldg, x.Lacc, P->rd_off[i]};
        }
        sc.rowdeg = P->rowdeg;
        // a fresh device copy: calls in flight keep the one they check against
        std::shared_ptr<DevImage> di = std::make_shared<DevImage>();
        bool up = hipMalloc((void**)&di->d, scan_words * 4) == hipSuccess;
        if (!up) di->d = nullptr;
        up = up && hipMemcpy(di->d, img, scan_words * 4, hipMemcpyHostToDevice) == hipSuccess;
        if (!up) (void)hipGetLastError();
        sc.dimg = up ? di : nullptr;
        sc.valid = up;
        if (!up) sc.conf = 0;
      }
    }
  }
  const int fused_err = P->fused ? h_flags[2 * nj] : 0;
  if (P->schur_instances) {
    cx->schur_instances += P->schur_instances;
    cx->schur_fallbacks += h_flags[2 * nj + 2];
  }
  int first_err = BIRES_OK;
  for (int i = 0; i < nj; ++i) {
    Work& x = w[i];
    bires_upoly* o = jobs[i].out;
    if (!x.status && x.active && fused_err) x.status = BIRES_ECHECK;
    if (!x.status) {
      if (x.active) {
        if (h_flags[2 * i + 1]) {
          x.status = BIRES_ECHECK;
        } else {
          if (mem == BIRES_MEM_HOST)
            std::memcpy(o->c, P->hout_base + x.o_hout, (size_t)(x.degcap + 1) * x.Lout * 4);
          o->degree = h_flags[2 * i];
        }
      } else {
        if (mem == BIRES_MEM_HOST) {
          std::memset(o->c, 0, (size_t)(x.degcap + 1) * x.Lout * 4);
          if (x.pl.kind_special == 2) o->c[0] = 1u;
        }
        o->degree = x.pl.kind_special == 2 ? 0 : -1;
      }
    }
    if (P->status) P->status[i] = x.status;
    if (x.status && first_err == BIRES_OK) first_err = x.status;
  }
  hc.mark(5);
  hc.commit(cx);
  return first_err;
}

int run_batch(Context* cx, const std::vector<JobIn>& jobs, int mem, hipStream_t st, int32_t* status,
              std::vector<uint32_t>* debug_values, std::vector<int>* debug_shape) {
  PendingPtr p;
  const int e = launch_impl(cx, jobs, mem, st, status, debug_values, debug_shape, &p);
  if (e || !p) return e;
  return run_batch_finish(std::move(p));
}

int run_batch_noalloc(Context* cx, const std::vector<JobIn>& jobs, int mem, hipStream_t st, int32_t* status) {
  // one call at a time: every call shares the scratch array
  std::lock_guard<std::mutex> lk(cx->scratch_mu);
  PendingPtr p;
  const int e = launch_impl(cx, jobs, mem, st, status, nullptr, nullptr, &p, true);
  if (e || !p) {
    if (p) (void)hipStreamSynchronize(st);
    return e;
  }
  return run_batch_finish(std::move(p));
}

}  // namespace bires

namespace bires {

int host_job(const JobIn& jb, HostJob& h) {
  int e = validate(jb, false);
  if (e) return e;
  const Shape sf = shape_of(jb.f, jb.var);
  h.rows_f = sf.rows, h.ld_f = sf.ld, h.L_f = sf.L;
  h.f.assign((size_t)sf.rows * sf.ld * sf.L, 0u);
  if (sf.rows) pack_rect(jb.f, jb.var, h.f.data());
  h.stf = scan_host(h.f.data(), sf.rows, sf.ld, sf.L);
  h.g.clear();
  if (jb.kind != BIRES_KIND_RESULTANT) {
    h.rows_g = 0, h.ld_g = sf.ld, h.L_g = sf.L;
    if ((e = derive_operand_stats(jb.kind, h.stf, h.stg))) return e;
  } else {
    const Shape sg = shape_of(jb.g, jb.var);
    h.rows_g = sg.rows, h.ld_g = sg.ld, h.L_g = sg.L;
    h.g.assign((size_t)sg.rows * sg.ld * sg.L, 0u);
    if (sg.rows) pack_rect(jb.g, jb.var, h.g.data());
    h.stg = scan_host(h.g.data(), sg.rows, sg.ld, sg.L);
  }
  return make_plan(h.stf, h.stg, h.pl);
}

int plan_host_job(const JobIn& jb, Plan& pl) {
  HostJob h;
  const int e = host_job(jb, h);
  pl = h.pl;
  return e;
}

int bounds_job(const JobIn& jb, int32_t* max_degree, int32_t* max_limbs) {
  int e = validate(jb, false);
  if (e) return e;
  const Shape sf = shape_of(jb.f, jb.var);
  RowStats stf = worst_stats(sf.rows, sf.ld, sf.L), stg;
  if (jb.kind != BIRES_KIND_RESULTANT) {
    if ((e = derive_operand_stats(jb.kind, stf, stg))) return e;
  } else {
    const Shape sg = shape_of(jb.g, jb.var);
    stg = worst_stats(sg.rows, sg.ld, sg.L);
  }
  Plan pl;
  if ((e = make_plan(stf, stg, pl))) return e;
  if (max_degree) *max_degree = pl.D - 1;
  if (max_limbs) *max_limbs = pl.kind_special ? 1 : limbs_for_log2(pl.log2B);
  return BIRES_OK;
}

}  // namespace bires

namespace bires {

int job_footprint(const JobIn& jb, int32_t* cap_degree, int32_t* cap_limbs, size_t* bytes) {
  int e = bounds_job(jb, cap_degree, cap_limbs);
  if (e) return e;
  Plan pl;
  if ((e = plan_host_job(jb, pl))) return e;
  const Shape sf = shape_of(jb.f, jb.var);
  const Shape sg = jb.kind == BIRES_KIND_RESULTANT ? shape_of(jb.g, jb.var) : sf;
  size_t b = (size_t)sf.rows * sf.ld * sf.L * 4 + (size_t)sg.rows * sg.ld * sg.L * 4;
  if (pl.kind_special == 0) {
    const size_t P = pl.P, D = pl.D, Lacc = std::min(*cap_limbs, pl.P + 1);
    b += P * ((size_t)(pl.m + 1) * sf.ld + (size_t)(pl.n + 1) * sg.ld) * 4;  // residues
    b += 3 * P * D * 4 + D * 4 + D * Lacc * 12;                              // values, coefs, digits, limbs
  }
  b += (size_t)(*cap_degree + 1) * (*cap_limbs) * 4;
  *bytes = b;
  return BIRES_OK;
}

}  // namespace bires
