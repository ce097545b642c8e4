// Serving: continuous batching of resultant / discriminant requests.
//
// submit() copies the inputs, plans the job on the host (its device
// footprint) and queues it.  A scheduler thread admits queued requests in
// arrival order while the number in flight stays within max_slots and their
// footprints fit in the HBM budget, and hands each admitted set to one of two
// worker threads as one batch (one batched launch sequence on the worker's own
// stream).  Requests that arrive while a batch runs are admitted into the next
// batch as soon as slots and memory free up, and the two workers' batches run
// concurrently on the device.  All intermediate data of a job (residues,
// values, coefficients, digits) stays in device memory until its result is
// copied back; wait() returns the result and the submit-to-completion latency.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bires.h"
#include "engine.hpp"

using namespace bires;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  int kind = 0, var = 0;
  std::vector<uint32_t> fbuf, gbuf;
  bires_bipoly f{}, g{};
  size_t footprint = 0;
  std::vector<uint32_t> out;
  int out_degree = -1, out_limbs = 1, cap_degree = 0;
  int status = BIRES_OK;
  bool done = false;
  Clock::time_point t_submit, t_done;
};

}  // namespace

struct bires_server {
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv_sched, cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> table;
  size_t in_use = 0;
  int in_flight = 0;
  std::deque<std::vector<Request*>> batches;  // admitted, waiting for a worker
  std::thread sched;
  std::thread workers[2];
  hipStream_t streams[2] = {nullptr, nullptr};
  Context* cx = nullptr;
};

namespace {

void copy_bipoly(const bires_bipoly& src, std::vector<uint32_t>& buf, bires_bipoly& dst) {
  dst = src;
  if (src.deg_y < 0) {
    dst.c = nullptr;
    return;
  }
  const size_t n = (size_t)(src.deg_y + 1) * (src.deg_x + 1) * src.limbs;
  buf.assign(src.c, src.c + n);
  dst.c = buf.data();
}

void scheduler(bires_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_sched.wait(lk, [&] { return s->stop || !s->pending.empty(); });
    if (s->stop && s->pending.empty()) break;
    std::vector<Request*> batch;
    while (!s->pending.empty()) {
      Request* r = s->pending.front();
      if (r->footprint > s->budget) {  // can never fit
        s->pending.pop_front();
        r->status = BIRES_ENOMEM;
        r->done = true;
        r->t_done = Clock::now();
        s->cv_done.notify_all();
        continue;
      }
      if (s->in_flight + 1 > s->max_slots || s->in_use + r->footprint > s->budget) break;
      s->pending.pop_front();
      s->in_flight += 1;
      s->in_use += r->footprint;
      batch.push_back(r);
    }
    if (!batch.empty()) {
      s->batches.push_back(std::move(batch));
      s->cv_work.notify_one();
    } else {
      // everything admitted is still running: wait for a completion
      s->cv_sched.wait(lk, [&] {
        return s->stop || (!s->pending.empty() && s->in_flight + 1 <= s->max_slots &&
                           s->in_use + s->pending.front()->footprint <= s->budget) ||
               (!s->pending.empty() && s->pending.front()->footprint > s->budget);
      });
    }
  }
  s->cv_work.notify_all();
}

void worker(bires_server* s, int w) {
  for (;;) {
    std::vector<Request*> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return !s->batches.empty() || (s->stop && s->pending.empty()); });
      if (s->batches.empty()) return;
      batch = std::move(s->batches.front());
      s->batches.pop_front();
    }
    std::vector<JobIn> jobs(batch.size());
    std::vector<bires_upoly> outs(batch.size());
    std::vector<int32_t> status(batch.size(), 0);
    for (size_t i = 0; i < batch.size(); ++i) {
      Request* r = batch[i];
      jobs[i].f = r->f;
      jobs[i].g = r->kind == BIRES_KIND_RESULTANT ? r->g : r->f;
      jobs[i].kind = r->kind;
      jobs[i].var = r->var;
      outs[i].degree = r->cap_degree;
      outs[i].limbs = r->out_limbs;
      outs[i].c = r->out.data();
      jobs[i].out = &outs[i];
    }
    int e = run_batch(s->cx, jobs, BIRES_MEM_HOST, s->streams[w], status.data());
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < batch.size(); ++i) {
      Request* r = batch[i];
      r->status = e == BIRES_EDEVICE || e == BIRES_ENOMEM ? (status[i] ? status[i] : e) : status[i];
      r->out_degree = outs[i].degree;
      r->done = true;
      r->t_done = now;
      s->in_flight -= 1;
      s->in_use -= r->footprint;
    }
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
  }
}

}  // namespace

extern "C" {

int bires_server_create(size_t hbm_budget_bytes, int max_slots, bires_server** out) {
  if (!out || max_slots < 1 || hbm_budget_bytes == 0) return BIRES_EINVAL;
  int err = BIRES_OK;
  Context* cx = context(&err);
  if (!cx) return err;
  bires_server* s = new bires_server();
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->cx = cx;
  for (auto& st : s->streams) {
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return BIRES_EDEVICE;
    }
  }
  s->sched = std::thread(scheduler, s);
  s->workers[0] = std::thread(worker, s, 0);
  s->workers[1] = std::thread(worker, s, 1);
  *out = s;
  return BIRES_OK;
}

int bires_server_submit(bires_server* s, int kind, int var, const bires_bipoly* f, const bires_bipoly* g,
                        uint64_t* ticket) {
  if (!s || !f || !ticket || (kind == BIRES_KIND_RESULTANT && !g)) return BIRES_EINVAL;
  Request* r = new Request();
  r->kind = kind;
  r->var = var;
  r->t_submit = Clock::now();
  copy_bipoly(*f, r->fbuf, r->f);
  if (kind == BIRES_KIND_RESULTANT) copy_bipoly(*g, r->gbuf, r->g);
  JobIn jb;
  jb.f = r->f;
  jb.g = kind == BIRES_KIND_RESULTANT ? r->g : r->f;
  jb.kind = kind;
  jb.var = var;
  int32_t deg = 0, limbs = 1;
  size_t bytes = 0;
  int e = job_footprint(jb, &deg, &limbs, &bytes);
  if (e) {
    delete r;
    return e;
  }
  r->cap_degree = deg;
  r->out_limbs = limbs;
  r->out.assign((size_t)(deg + 1) * limbs, 0u);
  r->footprint = bytes;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete r;
    return BIRES_EINVAL;
  }
  r->ticket = s->next_ticket++;
  s->table[r->ticket] = r;
  s->pending.push_back(r);
  *ticket = r->ticket;
  s->cv_sched.notify_one();
  return BIRES_OK;
}

// Smallest limb count that holds every coefficient of a finished request's
// result in two's complement.
static int needed_limbs(const Request* r) {
  const int Lr = r->out_limbs;
  int need = 1;
  for (int i = 0; i <= r->out_degree; ++i) {
    const uint32_t* c = &r->out[(size_t)i * Lr];
    const uint32_t ext = (c[Lr - 1] >> 31) ? 0xFFFFFFFFu : 0u;
    int l = Lr;
    while (l > 1 && c[l - 1] == ext && (c[l - 2] >> 31) == (ext >> 31)) --l;
    need = std::max(need, l);
  }
  return need;
}

int bires_server_wait(bires_server* s, uint64_t ticket, bires_upoly* out, double timeout_s, double* latency_s) {
  if (!s || !out) return BIRES_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->table.find(ticket);
  if (it == s->table.end()) return BIRES_ENOTFOUND;
  Request* r = it->second;
  if (timeout_s < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->done; })) {
    return BIRES_ETIMEOUT;
  }
  int e = r->status;
  if (!e) {
    // a buffer that is too small keeps the ticket: the needed sizes are
    // written back and the caller can wait again with a larger one
    const int deg = r->out_degree;
    const int need = needed_limbs(r);
    if (!out->c || out->limbs < 1) return BIRES_EINVAL;
    if (out->degree < std::max(deg, 0) || out->limbs < need) {
      out->degree = std::max(deg, out->degree);
      out->limbs = std::max(need, out->limbs);
      return BIRES_EBUFSIZE;
    }
    // re-encode at the caller's limb count (sign-extend or truncate the
    // sign-extension words, which need_limbs checked)
    const int Lr = r->out_limbs, Lc = out->limbs;
    for (int i = 0; i <= out->degree; ++i) {
      const uint32_t* src = i <= deg ? &r->out[(size_t)i * Lr] : nullptr;
      const uint32_t ext = src && (src[Lr - 1] >> 31) ? 0xFFFFFFFFu : 0u;
      for (int l = 0; l < Lc; ++l) out->c[(size_t)i * Lc + l] = src ? (l < Lr ? src[l] : ext) : 0u;
    }
    out->degree = deg;
  }
  s->table.erase(it);
  lk.unlock();
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  delete r;
  return e;
}

int bires_server_destroy(bires_server* s) {
  if (!s) return BIRES_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  s->cv_work.notify_all();
  s->sched.join();
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& st : s->streams) (void)hipStreamDestroy(st);
  for (auto& kv : s->table) delete kv.second;
  delete s;
  return BIRES_OK;
}

}  // extern "C"
