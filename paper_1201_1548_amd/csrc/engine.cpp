// Host orchestration of the batched multi-modular pipeline (see engine.hpp).
#include "engine.hpp"

#include <algorithm>
#include <cstring>
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
  return BIRES_OK;
}

Context* context(int* err) {
  static Context cx;
  static std::once_flag once;
  static int status = BIRES_OK;
  std::call_once(once, [] { status = init_context(cx); });
  *err = status;
  return status == BIRES_OK ? &cx : nullptr;
}

int schedule_for(Context* cx, size_t njobs) {
  if (cx->schedule != BIRES_SCHEDULE_AUTO) return cx->schedule;
  return njobs >= 2 ? BIRES_SCHEDULE_FUSED : BIRES_SCHEDULE_STAGED;
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
