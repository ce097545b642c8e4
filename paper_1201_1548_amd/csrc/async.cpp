// Asynchronous batched calls: the submitting thread plans the batch and
// queues its device work (run_batch_launch) on the caller's stream, or on the
// library stream when the caller names none, and returns; bires_batch_wait
// waits for that batch's completion event and finishes the call
// (run_batch_finish).  While one batch runs on the device, the caller plans
// and queues the next one, so the device does not idle between them.
#include "async.hpp"

#include <unordered_map>
#include <utility>

namespace bires {

namespace {

struct Tickets {
  std::mutex mu;
  std::unordered_map<uint64_t, PendingPtr> pending;
  uint64_t next = 1;
};

Tickets& tickets() {
  static Tickets* t = new Tickets;  // kept for the life of the process
  return *t;
}

}  // namespace

int async_submit(Context* cx, std::vector<JobIn>&& jobs, int mem, int32_t* status, hipStream_t caller,
                 uint64_t* ticket) {
  if (mem != BIRES_MEM_HOST && mem != BIRES_MEM_DEVICE) return BIRES_EINVAL;
  PendingPtr p;
  int e;
  if (caller) {
    e = run_batch_launch(cx, jobs, mem, caller, status, &p);
  } else {
    std::lock_guard<std::mutex> lk(cx->stream_mu);
    e = run_batch_launch(cx, jobs, mem, cx->stream, status, &p);
  }
  if (e) return e;
  if (!caller) set_pending_stream_lock(p.get());
  Tickets& t = tickets();
  std::lock_guard<std::mutex> lk(t.mu);
  *ticket = t.next++;
  t.pending.emplace(*ticket, std::move(p));
  return BIRES_OK;
}

int async_wait(Context* cx, uint64_t ticket) {
  (void)cx;
  PendingPtr p;
  {
    Tickets& t = tickets();
    std::lock_guard<std::mutex> lk(t.mu);
    auto it = t.pending.find(ticket);
    if (it == t.pending.end()) return BIRES_EINVAL;
    p = std::move(it->second);
    t.pending.erase(it);
  }
  return run_batch_finish(std::move(p));
}

}  // namespace bires
