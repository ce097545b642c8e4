// The C ABI of include/bires.h.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/bires.h"
#include "async.hpp"
#include "engine.hpp"
#include "gcd.hpp"
#include "kernels.hpp"
#include "tables.hpp"

using namespace bires;

namespace {

// Runs f with the caller's stream, or with the library stream held exclusively.
template <class F>
int with_stream(void* stream, F&& f) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  if (stream) return f(cx, (hipStream_t)stream);
  std::lock_guard<std::mutex> lk(cx->stream_mu);
  return f(cx, cx->stream);
}

// Job list of a batched call (validation of the array arguments only).
int batch_jobs(int n, const bires_bipoly* f, const bires_bipoly* g, const int32_t* kind, const int32_t* var,
               bires_upoly* out, std::vector<JobIn>* jobs) {
  if (n < 0 || (n > 0 && (!f || !kind || !var || !out))) return BIRES_EINVAL;
  jobs->assign(n, JobIn{});
  for (int i = 0; i < n; ++i) {
    JobIn& jb = (*jobs)[i];
    jb.f = f[i];
    jb.kind = kind[i];
    if (kind[i] == BIRES_KIND_RESULTANT) {
      if (!g) return BIRES_EINVAL;
      jb.g = g[i];
    } else {
      jb.g = f[i];
    }
    jb.var = var[i];
    jb.out = &out[i];
  }
  return BIRES_OK;
}

}  // namespace

extern "C" {

int bires_init(void) {
  int err = BIRES_OK;
  context(&err);
  return err;
}

int bires_resultant_bounds(const bires_bipoly* f, const bires_bipoly* g, int var, int32_t* max_degree,
                           int32_t* max_limbs) {
  if (!f || !g) return BIRES_EINVAL;
  JobIn jb;
  jb.f = *f;
  jb.g = *g;
  jb.var = var;
  jb.kind = BIRES_KIND_RESULTANT;
  return bounds_job(jb, max_degree, max_limbs);
}

int bires_discriminant_bounds(const bires_bipoly* f, int var, int32_t* max_degree, int32_t* max_limbs) {
  if (!f) return BIRES_EINVAL;
  JobIn jb;
  jb.f = *f;
  jb.g = *f;
  jb.var = var;
  jb.kind = BIRES_KIND_DISCRIMINANT;
  return bounds_job(jb, max_degree, max_limbs);
}

int bires_polar_bounds(const bires_bipoly* f, int var, int32_t* max_degree, int32_t* max_limbs) {
  if (!f) return BIRES_EINVAL;
  JobIn jb;
  jb.f = *f;
  jb.g = *f;
  jb.var = var;
  jb.kind = BIRES_KIND_POLAR;
  return bounds_job(jb, max_degree, max_limbs);
}

int bires_resultant(const bires_bipoly* f, const bires_bipoly* g, int var, bires_upoly* out, int mem,
                    void* stream) {
  if (!f || !g || !out) return BIRES_EINVAL;
  std::vector<JobIn> jobs(1);
  jobs[0].f = *f;
  jobs[0].g = *g;
  jobs[0].var = var;
  jobs[0].kind = BIRES_KIND_RESULTANT;
  jobs[0].out = out;
  return with_stream(stream, [&](Context* cx, hipStream_t st) { return run_batch(cx, jobs, mem, st, nullptr); });
}

int bires_discriminant(const bires_bipoly* f, int var, bires_upoly* out, int mem, void* stream) {
  if (!f || !out) return BIRES_EINVAL;
  std::vector<JobIn> jobs(1);
  jobs[0].f = *f;
  jobs[0].g = *f;
  jobs[0].var = var;
  jobs[0].kind = BIRES_KIND_DISCRIMINANT;
  jobs[0].out = out;
  return with_stream(stream, [&](Context* cx, hipStream_t st) { return run_batch(cx, jobs, mem, st, nullptr); });
}

int bires_polar_resultant(const bires_bipoly* f, int var, bires_upoly* out, int mem, void* stream) {
  if (!f || !out) return BIRES_EINVAL;
  std::vector<JobIn> jobs(1);
  jobs[0].f = *f;
  jobs[0].g = *f;
  jobs[0].var = var;
  jobs[0].kind = BIRES_KIND_POLAR;
  jobs[0].out = out;
  return with_stream(stream, [&](Context* cx, hipStream_t st) { return run_batch(cx, jobs, mem, st, nullptr); });
}

int bires_resultant_noalloc(const bires_bipoly* f, const bires_bipoly* g, int kind, int var, bires_upoly* out,
                            int mem, void* stream) {
  if (!f || !out || (kind == BIRES_KIND_RESULTANT && !g)) return BIRES_EINVAL;
  if (kind != BIRES_KIND_RESULTANT && kind != BIRES_KIND_DISCRIMINANT && kind != BIRES_KIND_POLAR)
    return BIRES_EINVAL;
  Context* cx = context_if_ready();  // never sets the library up (that allocates)
  if (!cx) return BIRES_EINVAL;
  std::vector<JobIn> jobs(1);
  jobs[0].f = *f;
  jobs[0].g = kind == BIRES_KIND_RESULTANT ? *g : *f;
  jobs[0].var = var;
  jobs[0].kind = kind;
  jobs[0].out = out;
  if (stream) return run_batch_noalloc(cx, jobs, mem, (hipStream_t)stream, nullptr);
  std::lock_guard<std::mutex> lk(cx->stream_mu);
  return run_batch_noalloc(cx, jobs, mem, cx->stream, nullptr);
}

int bires_resultant_batch(int n, const bires_bipoly* f, const bires_bipoly* g, const int32_t* kind,
                          const int32_t* var, bires_upoly* out, int32_t* status, int mem, void* stream) {
  std::vector<JobIn> jobs;
  const int e = batch_jobs(n, f, g, kind, var, out, &jobs);
  if (e || n == 0) return e;
  return with_stream(stream, [&](Context* cx, hipStream_t st) { return run_batch(cx, jobs, mem, st, status); });
}

int bires_resultant_batch_async(int n, const bires_bipoly* f, const bires_bipoly* g, const int32_t* kind,
                                const int32_t* var, bires_upoly* out, int32_t* status, int mem, void* stream,
                                uint64_t* ticket) {
  if (!ticket) return BIRES_EINVAL;
  std::vector<JobIn> jobs;
  const int e = batch_jobs(n, f, g, kind, var, out, &jobs);
  if (e) return e;
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  return async_submit(cx, std::move(jobs), mem, status, (hipStream_t)stream, ticket);
}

int bires_batch_wait(uint64_t ticket) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  return async_wait(cx, ticket);
}

int bires_psc(const bires_bipoly* f, const bires_bipoly* g, int kind, int var, uint32_t p, uint32_t* out,
              int64_t capacity, int32_t* count, int32_t* points, void* stream) {
  if (!f || (kind == BIRES_KIND_RESULTANT && !g) || (capacity > 0 && !out)) return BIRES_EINVAL;
  JobIn jb;
  jb.f = *f;
  jb.g = kind == BIRES_KIND_RESULTANT ? *g : *f;
  jb.kind = kind;
  jb.var = var;
  return with_stream(stream, [&](Context* cx, hipStream_t st) {
    return run_psc(cx, jb, p, out, capacity, count, points, st);
  });
}

int bires_fiber_bounds(const bires_bipoly* f, int var, const bires_upoly* rstar, int32_t deg_r, uint32_t p,
                       int64_t* n_minus, int64_t* n_plus, int32_t* flags, void* stream) {
  if (!f || !rstar) return BIRES_EINVAL;
  return with_stream(stream, [&](Context* cx, hipStream_t st) {
    return run_fiber_bounds(cx, *f, var, *rstar, deg_r, p, n_minus, n_plus, flags, st);
  });
}

int bires_gcd_bounds(const bires_upoly* a, const bires_upoly* b, int32_t* max_degree, int32_t* max_limbs) {
  return gcd_bounds(a, b, max_degree, max_limbs);
}

int bires_gcd(const bires_upoly* a, const bires_upoly* b, bires_upoly* out, int mem, void* stream) {
  if (!a || !b || !out) return BIRES_EINVAL;
  return with_stream(stream, [&](Context* cx, hipStream_t st) { return run_gcd(cx, *a, *b, out, mem, st); });
}

int bires_squarefree(const bires_upoly* r, bires_upoly* unit, bires_upoly* factors, int32_t max_factors,
                     int32_t* count, int mem, void* stream) {
  if (!r) return BIRES_EINVAL;
  return with_stream(stream, [&](Context* cx, hipStream_t st) {
    return run_squarefree(cx, *r, unit, factors, max_factors, count, mem, st);
  });
}

int bires_plan(const bires_bipoly* f, const bires_bipoly* g, int kind, int var, int32_t* points, int32_t* primes,
               double* log2_bound) {
  if (!f || (kind == BIRES_KIND_RESULTANT && !g)) return BIRES_EINVAL;
  JobIn jb;
  jb.f = *f;
  jb.g = kind == BIRES_KIND_RESULTANT ? *g : *f;
  jb.kind = kind;
  jb.var = var;
  Plan pl;
  int e = plan_host_job(jb, pl);
  if (e) return e;
  if (points) *points = pl.D;
  if (primes) *primes = pl.P;
  if (log2_bound) *log2_bound = pl.log2B;
  return BIRES_OK;
}

int bires_primes(int n, uint32_t* out) {
  if (n < 0 || n > MAX_PRIMES || (n && !out)) return BIRES_EINVAL;
  const HostTables& t = host_tables();
  for (int i = 0; i < n; ++i) out[i] = t.primes[i].p;
  return BIRES_OK;
}

int bires_debug_values(const bires_bipoly* f, const bires_bipoly* g, int kind, int var, uint32_t* values,
                       int64_t capacity, int32_t* points, int32_t* primes) {
  if (!f || !values || (kind == BIRES_KIND_RESULTANT && !g)) return BIRES_EINVAL;
  std::vector<JobIn> jobs(1);
  jobs[0].f = *f;
  jobs[0].g = kind == BIRES_KIND_RESULTANT ? *g : *f;
  jobs[0].kind = kind;
  jobs[0].var = var;
  std::vector<uint32_t> vals;
  std::vector<int> shape;
  int e = with_stream(nullptr, [&](Context* cx, hipStream_t st) {
    return run_batch(cx, jobs, BIRES_MEM_HOST, st, nullptr, &vals, &shape);
  });
  if (e) return e;
  if (points) *points = shape[1];
  if (primes) *primes = shape[0];
  if ((int64_t)vals.size() > capacity) return BIRES_EBUFSIZE;
  std::memcpy(values, vals.data(), vals.size() * 4);
  return BIRES_OK;
}

int bires_set_timing(int enable) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  std::lock_guard<std::mutex> lk(cx->timing_mu);
  cx->timing = enable != 0;
  cx->kernel_ms = 0.0;
  cx->kernel_launches = 0;
  for (double& u : cx->host_us) u = 0.0;
  cx->host_calls = 0;
  return BIRES_OK;
}

int bires_set_graphs(int enable) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  std::lock_guard<std::mutex> lk(cx->graph_mu);
  cx->graphs = enable != 0;
  if (!cx->graphs && !cx->graph_cache.empty()) {
    if (hipDeviceSynchronize() != hipSuccess) return BIRES_EDEVICE;
    for (auto& kv : cx->graph_cache) (void)hipGraphExecDestroy(kv.second);
    cx->graph_cache.clear();
    cx->graph_order.clear();
  }
  return BIRES_OK;
}

int bires_set_eval_kernel(int kernel) {
  if (kernel != BIRES_EVAL_AUTO && kernel != BIRES_EVAL_LDS && kernel != BIRES_EVAL_SCHUR) return BIRES_EINVAL;
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  cx->eval_mode = kernel;
  return BIRES_OK;
}

int bires_issue_rates(double* cycles, int n) {
  if (!cycles || n < 1) return BIRES_EINVAL;
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cx->device) != hipSuccess) return BIRES_EDEVICE;
  const int blocks = prop.multiProcessorCount * 16, iters = 2048;
  uint32_t* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * 256 * 4) != hipSuccess) return BIRES_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BIRES_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = BIRES_EDEVICE;
  const double simds = 4.0 * prop.multiProcessorCount, hz = prop.clockRate * 1e3;
  const double waves = (double)blocks * 256 / 64, instr = waves * iters * 16;
  std::lock_guard<std::mutex> lk(cx->stream_mu);
  for (int k = 0; k < n && k < 6 && rc == BIRES_OK; ++k) {
    float best = 1e30f;
    for (int rep = 0; rep < 3 && rc == BIRES_OK; ++rep) {
      float ms = 0.f;
      if (hipEventRecord(e0, cx->stream) != hipSuccess) rc = BIRES_EDEVICE;
      launch_issue_rate(k, out, blocks, iters, cx->stream);
      if (hipEventRecord(e1, cx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
        rc = BIRES_EDEVICE;
      best = std::min(best, ms);
    }
    cycles[k] = simds * hz * best * 1e-3 / instr;  // SIMD-cycles per wave instruction
  }
  for (int k = 6; k < n; ++k) cycles[k] = 0.0;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return rc;
}

int bires_set_plan_cache(int enable) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  cx->plan_cache = enable != 0;
  std::lock_guard<std::mutex> lk(cx->spec.mu);
  cx->spec.valid = false;
  cx->spec.conf = 0;
  return BIRES_OK;
}

int bires_plan_cache_stats(int64_t* hits, int64_t* misses) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  std::lock_guard<std::mutex> lk(cx->spec.mu);
  if (hits) *hits = cx->spec.hits;
  if (misses) *misses = cx->spec.misses;
  return BIRES_OK;
}

int bires_schur_stats(int64_t* instances, int64_t* fallbacks) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  if (instances) *instances = cx->schur_instances;
  if (fallbacks) *fallbacks = cx->schur_fallbacks;
  return BIRES_OK;
}

int bires_graph_stats(int64_t* captures, int64_t* replays) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  std::lock_guard<std::mutex> lk(cx->graph_mu);
  if (captures) *captures = cx->graph_captures;
  if (replays) *replays = cx->graph_replays;
  return BIRES_OK;
}

int bires_set_schedule(int schedule) {
  if (schedule < BIRES_SCHEDULE_STAGED || schedule > BIRES_SCHEDULE_SCHUR) return BIRES_EINVAL;
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  cx->schedule = schedule;
  return BIRES_OK;
}

int bires_autotune(int n, const bires_bipoly* f, const bires_bipoly* g, const int32_t* kind, const int32_t* var,
                   bires_upoly* out, int32_t* status, int mem, void* stream, int reps, int32_t* chosen) {
  if (reps < 1) return BIRES_EINVAL;
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  // each schedule once to warm up, then the timed rounds in turn (staged,
  // fused, Schur, staged, ...), so that a drift of the device's clocks or a
  // stray slow call does not favour one schedule; the best time of each
  const int scheds[3] = {BIRES_SCHEDULE_STAGED, BIRES_SCHEDULE_FUSED, BIRES_SCHEDULE_SCHUR};
  double t[3] = {1e300, 1e300, 1e300};
  std::string key;
  for (int r = -1; r < reps; ++r) {
    for (int i = 0; i < 3; ++i) {
      cx->forced_schedule = scheds[i];
      const auto t0 = std::chrono::steady_clock::now();
      const int e = bires_resultant_batch(n, f, g, kind, var, out, status, mem, stream);
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      cx->forced_schedule = -1;
      if (e != BIRES_OK) return e;
      if (r >= 0) t[i] = std::min(t[i], dt);
      std::lock_guard<std::mutex> lk(cx->tune_mu);
      key = cx->last_key;
    }
  }
  int best_s = BIRES_SCHEDULE_STAGED;
  double best = 1e300;
  for (int i = 0; i < 3; ++i)
    if (t[i] < best) {
      best = t[i];
      best_s = scheds[i];
    }
  tune_store(cx, key, best_s);
  if (chosen) *chosen = best_s;
  return BIRES_OK;
}

int bires_kernel_time(double* ms, int64_t* launches) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  std::lock_guard<std::mutex> lk(cx->timing_mu);
  if (ms) *ms = cx->kernel_ms;
  if (launches) *launches = cx->kernel_launches;
  return BIRES_OK;
}

int bires_host_time(double* us, int64_t* calls) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  std::lock_guard<std::mutex> lk(cx->timing_mu);
  if (us)
    for (int k = 0; k < BIRES_HOST_PHASES; ++k) us[k] = cx->host_us[k];
  if (calls) *calls = cx->host_calls;
  return BIRES_OK;
}

int bires_device_info(int32_t* compute_units, int32_t* clock_khz, int64_t* lds_per_block, int64_t* hbm_bytes) {
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cx->device) != hipSuccess) return BIRES_EDEVICE;
  if (compute_units) *compute_units = prop.multiProcessorCount;
  if (clock_khz) *clock_khz = prop.clockRate;
  if (lds_per_block) *lds_per_block = (int64_t)prop.sharedMemPerBlock;
  if (hbm_bytes) *hbm_bytes = (int64_t)prop.totalGlobalMem;
  return BIRES_OK;
}

const char* bires_strerror(int code) {
  switch (code) {
    case BIRES_OK: return "success";
    case BIRES_EINVAL: return "invalid argument";
    case BIRES_EBUFSIZE: return "output buffer too small";
    case BIRES_ENOMEM: return "out of device or pinned memory, or over the HBM budget";
    case BIRES_ETOOBIG: return "input beyond the compiled limits";
    case BIRES_EDEVICE: return "HIP runtime error or no gfx950 device";
    case BIRES_ECHECK: return "internal consistency check failed";
    case BIRES_ENOTFOUND: return "unknown ticket";
    case BIRES_ETIMEOUT: return "timed out";
    default: return "unknown error";
  }
}

}  // extern "C"
