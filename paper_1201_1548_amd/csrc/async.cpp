// Asynchronous batched calls: two library worker threads, each with its own
// stream, run queued batches with run_batch.  A batch waits on its worker's
// stream for an event recorded on the caller's stream at submission (if the
// caller names one), so inputs produced there are complete, but never for
// other batches: while one worker's batch runs on the device, the other
// worker scans and plans the next one.
#include "async.hpp"

#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <utility>

namespace bires {

namespace {

struct Task {
  uint64_t ticket = 0;
  std::vector<JobIn> jobs;
  int mem = BIRES_MEM_DEVICE;
  int32_t* status = nullptr;
  hipEvent_t ready = nullptr;
};

constexpr int kWorkers = 2;

struct AsyncExec {
  Context* cx = nullptr;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_task, cv_done;
  std::deque<Task> queue;
  std::unordered_map<uint64_t, int> state;  // ticket -> -1 while queued or running, else its return code
  uint64_t next = 1;
  hipStream_t streams[kWorkers] = {};
};

void worker(AsyncExec* ax, int w) {
  (void)hipSetDevice(ax->device);
  for (;;) {
    Task t;
    {
      std::unique_lock<std::mutex> lk(ax->mu);
      ax->cv_task.wait(lk, [&] { return !ax->queue.empty(); });
      t = std::move(ax->queue.front());
      ax->queue.pop_front();
    }
    int e = BIRES_OK;
    if (t.ready && hipStreamWaitEvent(ax->streams[w], t.ready, 0) != hipSuccess) e = BIRES_EDEVICE;
    if (e == BIRES_OK) e = run_batch(ax->cx, t.jobs, t.mem, ax->streams[w], t.status);
    // run_batch has synchronised the worker's stream, so the wait is done
    if (t.ready) (void)hipEventDestroy(t.ready);
    {
      std::lock_guard<std::mutex> lk(ax->mu);
      ax->state[t.ticket] = e;
    }
    ax->cv_done.notify_all();
  }
}

// Started on first use and kept for the life of the process (the workers
// block on the queue when idle).
AsyncExec* exec_of(Context* cx, int* err) {
  static AsyncExec* ax = nullptr;
  static std::once_flag once;
  static int status = BIRES_OK;
  std::call_once(once, [&] {
    AsyncExec* a = new AsyncExec;
    a->cx = cx;
    a->device = cx->device;
    for (int w = 0; w < kWorkers; ++w)
      if (hipStreamCreateWithFlags(&a->streams[w], hipStreamNonBlocking) != hipSuccess) {
        status = BIRES_EDEVICE;
        return;
      }
    for (int w = 0; w < kWorkers; ++w) std::thread(worker, a, w).detach();
    ax = a;
  });
  *err = status;
  return ax;
}

}  // namespace

int async_submit(Context* cx, std::vector<JobIn>&& jobs, int mem, int32_t* status, hipStream_t caller,
                 uint64_t* ticket) {
  if (mem != BIRES_MEM_HOST && mem != BIRES_MEM_DEVICE) return BIRES_EINVAL;
  int err = BIRES_OK;
  AsyncExec* ax = exec_of(cx, &err);
  if (!ax) return err;
  Task t;
  // no caller stream: the inputs are complete already.  (An event on the
  // legacy default stream would also wait for the batches in flight.)
  if (caller) {
    if (hipEventCreateWithFlags(&t.ready, hipEventDisableTiming) != hipSuccess) return BIRES_EDEVICE;
    if (hipEventRecord(t.ready, caller) != hipSuccess) {
      (void)hipEventDestroy(t.ready);
      return BIRES_EDEVICE;
    }
  }
  t.jobs = std::move(jobs);
  t.mem = mem;
  t.status = status;
  {
    std::lock_guard<std::mutex> lk(ax->mu);
    t.ticket = ax->next++;
    ax->state[t.ticket] = -1;
    *ticket = t.ticket;
    ax->queue.push_back(std::move(t));
  }
  ax->cv_task.notify_one();
  return BIRES_OK;
}

int async_wait(Context* cx, uint64_t ticket) {
  int err = BIRES_OK;
  AsyncExec* ax = exec_of(cx, &err);
  if (!ax) return err;
  std::unique_lock<std::mutex> lk(ax->mu);
  auto it = ax->state.find(ticket);
  if (it == ax->state.end()) return BIRES_EINVAL;
  ax->cv_done.wait(lk, [&] { return ax->state[ticket] != -1; });
  const int e = ax->state[ticket];
  ax->state.erase(ticket);
  return e;
}

}  // namespace bires
