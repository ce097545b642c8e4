// Host orchestration of the batched multi-modular pipeline (see engine.hpp).
#include "engine.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>

#include "kernels.hpp"
#include "tables.hpp"

namespace bires {

#define HIP_OK(x)                       \
  do {                                  \
    if ((x) != hipSuccess) return BIRES_EDEVICE; \
  } while (0)

// ---------------------------------------------------------------------------
// pools

static size_t size_class(size_t b) {
  if (b < 4096) b = 4096;
  if (b <= ((size_t)64 << 20)) {
    size_t c = 4096;
    while (c < b) c <<= 1;
    return c;
  }
  const size_t g = (size_t)16 << 20;
  return (b + g - 1) / g * g;
}

void* Pool::alloc(size_t bytes) {
  const size_t c = size_class(bytes);
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].bytes == c) {
        Block b = free_[i];
        free_.erase(free_.begin() + i);
        used_.push_back(b);
        return b.p;
      }
    }
  }
  void* p = nullptr;
  hipError_t e = pinned_ ? hipHostMalloc(&p, c, hipHostMallocDefault) : hipMalloc(&p, c);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim();
    e = pinned_ ? hipHostMalloc(&p, c, hipHostMallocDefault) : hipMalloc(&p, c);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(mu_);
  used_.push_back({p, c});
  return p;
}

void Pool::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  for (size_t i = 0; i < used_.size(); ++i) {
    if (used_[i].p == p) {
      free_.push_back(used_[i]);
      used_.erase(used_.begin() + i);
      return;
    }
  }
}

size_t Pool::cached_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  size_t s = 0;
  for (auto& b : free_) s += b.bytes;
  return s;
}

void Pool::trim() {
  std::lock_guard<std::mutex> lk(mu_);
  for (auto& b : free_) {
    if (pinned_) (void)hipHostFree(b.p);
    else (void)hipFree(b.p);
  }
  free_.clear();
}

// ---------------------------------------------------------------------------
// context

static int init_context(Context& cx) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_OK(hipGetDeviceProperties(&prop, dev));
  if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos) return BIRES_EDEVICE;
  cx.device = dev;
  cx.lds_per_block = prop.sharedMemPerBlock;
  cx.lds_per_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor : prop.sharedMemPerBlock;
  cx.compute_units = prop.multiProcessorCount;
  HIP_OK(hipStreamCreateWithFlags(&cx.stream, hipStreamNonBlocking));
  const HostTables& t = host_tables();
  ModP* primes = nullptr;
  uint32_t *gm = nullptr, *cm = nullptr, *pi = nullptr, *pm = nullptr;
  HIP_OK(hipMalloc(&primes, t.primes.size() * sizeof(ModP)));
  HIP_OK(hipMalloc(&gm, t.gm.size() * sizeof(uint32_t)));
  HIP_OK(hipMalloc(&cm, t.cm.size() * sizeof(uint32_t)));
  HIP_OK(hipMalloc(&pi, t.pi.size() * sizeof(uint32_t)));
  HIP_OK(hipMalloc(&pm, t.pm.size() * sizeof(uint32_t)));
  HIP_OK(hipMemcpy(pm, t.pm.data(), t.pm.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(primes, t.primes.data(), t.primes.size() * sizeof(ModP), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(gm, t.gm.data(), t.gm.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(cm, t.cm.data(), t.cm.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(pi, t.pi.data(), t.pi.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  cx.tab.primes = primes;
  cx.tab.gm = gm;
  cx.tab.cm = cm;
  cx.tab.pi = pi;
  cx.tab.pm = pm;
  cx.tab.K = t.K;
  uint32_t* invfact = nullptr;
  HIP_OK(hipMalloc(&invfact, (size_t)t.K * MAX_POINTS * sizeof(uint32_t)));
  launch_invfact(primes, t.K, invfact, MAX_POINTS, cx.stream);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(cx.stream));
  cx.tab.invfact = invfact;
  cx.tab.dmax = MAX_POINTS;
  std::vector<double> invp(t.K);
  for (int k = 0; k < t.K; ++k) invp[k] = 1.0 / (double)t.primes[k].p;
  double* d_invp = nullptr;
  HIP_OK(hipMalloc(&d_invp, invp.size() * sizeof(double)));
  HIP_OK(hipMemcpy(d_invp, invp.data(), invp.size() * sizeof(double), hipMemcpyHostToDevice));
  cx.tab.inv_p = d_invp;
  {
    const int e = scratch_address(&cx.scratch, &cx.scratch_bytes);
    if (e) return e;
  }
  tune_load(&cx);
  return BIRES_OK;
}

const uint32_t* crt_device(Context* cx, int P, int* LM) {
  std::lock_guard<std::mutex> lk(cx->crt_mu);
  auto it = cx->crt.find(P);
  if (it == cx->crt.end()) {
    const CrtHost h = crt_tables(P);
    uint32_t* d = nullptr;
    if (hipMalloc(&d, h.buf.size() * sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (hipMemcpy(d, h.buf.data(), h.buf.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(d);
      return nullptr;
    }
    it = cx->crt.emplace(P, std::make_pair((const uint32_t*)d, h.LM)).first;
  }
  *LM = it->second.second;
  return it->second.first;
}

const uint32_t* crt_device_cached(Context* cx, int P, int* LM) {
  std::lock_guard<std::mutex> lk(cx->crt_mu);
  auto it = cx->crt.find(P);
  if (it == cx->crt.end()) return nullptr;
  *LM = it->second.second;
  return it->second.first;
}

bool graph_launch(Context* cx, uint64_t key, hipStream_t st) {
  std::lock_guard<std::mutex> lk(cx->graph_mu);
  auto it = cx->graph_cache.find(key);
  if (it == cx->graph_cache.end()) return false;
  if (hipGraphLaunch(it->second, st) != hipSuccess) return false;
  cx->graph_replays++;
  return true;
}

bool graph_store_launch(Context* cx, uint64_t key, hipGraphExec_t exec, hipStream_t st) {
  std::lock_guard<std::mutex> lk(cx->graph_mu);
  auto it = cx->graph_cache.find(key);
  if (it != cx->graph_cache.end()) {  // another thread stored the same sequence
    (void)hipGraphExecDestroy(exec);
    exec = it->second;
  } else {
    if (cx->graph_order.size() >= 32) {
      // rare: wait for every launch before destroying the oldest executable
      (void)hipDeviceSynchronize();
      const uint64_t old = cx->graph_order.front();
      cx->graph_order.erase(cx->graph_order.begin());
      (void)hipGraphExecDestroy(cx->graph_cache[old]);
      cx->graph_cache.erase(old);
    }
    cx->graph_cache[key] = exec;
    cx->graph_order.push_back(key);
    cx->graph_captures++;
  }
  return hipGraphLaunch(exec, st) == hipSuccess;
}

bool interp_tables_device(Context* cx, int blocks, int primes, hipStream_t st, const uint32_t** W,
                          const uint32_t** Q, int* nb) {
  std::lock_guard<std::mutex> lk(cx->itab_mu);
  if (!cx->itab || cx->itab_nb < blocks || cx->itab_P < primes) {
    const int nbn = std::max(blocks, cx->itab_nb), Pn = std::max(primes, cx->itab_P);
    size_t qoff = 0;
    const size_t words = interp_table_words(nbn, Pn, &qoff);
    if (words * sizeof(uint32_t) > ((size_t)512 << 20)) return false;
    uint32_t* d = nullptr;
    if (hipMalloc((void**)&d, words * sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    launch_interp_tables(nbn, Pn, cx->tab, d, d + qoff, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      (void)hipFree(d);
      return false;
    }
    if (cx->itab) cx->itab_retired.push_back(cx->itab);
    cx->itab = d;
    cx->itab_nb = nbn;
    cx->itab_P = Pn;
    cx->itab_qoff = qoff;
  }
  *W = cx->itab;
  *Q = cx->itab + cx->itab_qoff;
  *nb = cx->itab_nb;
  return true;
}

const int8_t* vinv_device(Context* cx, int D, int P, hipStream_t st) {
  constexpr size_t kLimit = (size_t)2 << 30;  // bytes of cached tables
  std::lock_guard<std::mutex> lk(cx->vinv_mu);
  auto it = cx->vinv.find({D, P});
  if (it != cx->vinv.end()) return it->second;
  const int Dp = (D + 31) & ~31;
  const size_t bytes = vinv_bytes(Dp, P);
  if (cx->vinv_total + bytes > kLimit) return nullptr;
  int8_t* d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  launch_vinv(D, Dp, P, cx->tab, d, st);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  cx->vinv_total += bytes;
  cx->vinv.emplace(std::make_pair(D, P), d);
  return d;
}

// The context lives until the process ends and is never destroyed: its device
// buffers (pools, tables, cached graphs, the plan cache's statistics copy) are
// not freed from a static destructor, which may run after the HIP runtime has
// shut down.
static std::atomic<Context*> g_ready{nullptr};

Context* context(int* err) {
  static Context* cx = new Context;
  static std::once_flag once;
  static int status = BIRES_OK;
  std::call_once(once, [] {
    status = init_context(*cx);
    if (status == BIRES_OK) g_ready.store(cx, std::memory_order_release);
  });
  *err = status;
  return status == BIRES_OK ? cx : nullptr;
}

Context* context_if_ready() { return g_ready.load(std::memory_order_acquire); }

static int log2_bucket(long long v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

std::string tune_key(long long instances, int max_r, int max_p) {
  return "gfx950/i" + std::to_string(log2_bucket(instances)) + "/r" + std::to_string(log2_bucket(max_r)) + "/p" +
         std::to_string(log2_bucket(max_p));
}

int schedule_for(Context* cx, const std::string& key) {
  if (cx->forced_schedule >= 0) return cx->forced_schedule;
  if (cx->schedule != BIRES_SCHEDULE_AUTO) return cx->schedule;
  {
    std::lock_guard<std::mutex> lk(cx->tune_mu);
    auto it = cx->tuned.find(key);
    if (it != cx->tuned.end()) return it->second;
  }
  return BIRES_SCHEDULE_STAGED;  // faster in every measured untuned case
}

void tune_load(Context* cx) {
  const char* path = std::getenv("BIRES_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  cx->tune_path = path;
  std::ifstream in(path);
  std::string key;
  int sched;
  while (in >> key >> sched)
    if (sched == BIRES_SCHEDULE_STAGED || sched == BIRES_SCHEDULE_FUSED || sched == BIRES_SCHEDULE_SCHUR)
      cx->tuned[key] = sched;
}

void tune_store(Context* cx, const std::string& key, int schedule) {
  std::lock_guard<std::mutex> lk(cx->tune_mu);
  cx->tuned[key] = schedule;
  if (cx->tune_path.empty()) return;
  std::ofstream out(cx->tune_path, std::ios::trunc);
  for (auto& kv : cx->tuned) out << kv.first << " " << kv.second << "\n";
}

// ---------------------------------------------------------------------------
// validation and planning

int check_bipoly(const bires_bipoly* p, int allow_null_c) {
  if (!p) return BIRES_EINVAL;
  if (p->deg_y < -1 || p->deg_x < -1 || p->limbs < 1) return BIRES_EINVAL;
  if (p->deg_y >= 0 && p->deg_x < 0) return BIRES_EINVAL;
  if (p->deg_y >= 0 && !p->c && !allow_null_c) return BIRES_EINVAL;
  if ((int64_t)(p->deg_y + 1) * (p->deg_x + 1) * p->limbs > ((int64_t)1 << 31)) return BIRES_ETOOBIG;
  return BIRES_OK;
}


}  // namespace bires
