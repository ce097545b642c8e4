// Host orchestration: device context, memory pools and the batched pipeline.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bires.h"
#include "job.hpp"
#include "plan.hpp"

namespace bires {

// Caching allocator over hipMalloc / hipHostMalloc: blocks are rounded up to a
// size class and returned to a free list instead of being freed.
class Pool {
 public:
  explicit Pool(bool pinned) : pinned_(pinned) {}
  void* alloc(size_t bytes);
  void release(void* p);
  size_t cached_bytes();
  void trim();

 private:
  struct Block {
    void* p;
    size_t bytes;
  };
  bool pinned_;
  std::mutex mu_;
  std::vector<Block> free_;
  std::vector<Block> used_;
};

// Plans of the last batched call with device-memory inputs, reused by the
// next call with the same extents and capacities while the row statistics
// repeat; the reusing call checks the fresh statistics against `image` on the
// device and is rerun with fresh plans when they differ.
struct SpecJob {
  int status = 0;
  bool active = false;
  Plan pl;
  int Lout = 1, degcap = 0, Tf = 0, Tg = 0, ldg = 0, Lacc = 1;
  int rd_off = 0;  // into rowdeg: m + 1 + n + 1 row degrees when active
};
struct SpecKey {  // the fields of a JobIn that planning reads (not its buffer addresses)
  int32_t f[3], g[3], kind, var, odeg, olimbs;
};
// A device copy of a statistics image; calls in flight hold a reference, so
// a newer image never overwrites one a pending check still reads.
struct DevImage {
  int32_t* d = nullptr;
  ~DevImage() {
    if (d) (void)hipFree(d);
  }
};
struct SpecCache {
  std::mutex mu;
  bool valid = false;
  int conf = 0;  // consecutive planned calls whose statistics equalled the previous ones
  std::vector<SpecKey> keys;
  std::vector<int32_t> image;  // the scan's output words
  std::shared_ptr<DevImage> dimg;  // device copy of image
  std::vector<SpecJob> plans;
  std::vector<int32_t> rowdeg;
  int64_t hits = 0, misses = 0;
};

struct Context {
  int device = -1;
  hipStream_t stream = nullptr;     // library stream (default priority)
  std::mutex stream_mu;             // serialises use of the library stream
  TablesDev tab{};                  // device copies of the host tables
  Pool dev{false};
  Pool host{true};
  size_t lds_per_block = 65536;
  size_t lds_per_cu = 65536;
  int compute_units = 1;
  bool timing = false;
  int schedule = BIRES_SCHEDULE_AUTO;    // BIRES_SCHEDULE_*
  int forced_schedule = -1;              // set by the autotuner while it measures
  std::mutex tune_mu;
  std::map<std::string, int> tuned;      // batch key -> schedule
  std::string tune_path;                 // BIRES_AUTOTUNE_CACHE
  std::string last_key;                  // key of the last batch planned
  std::mutex timing_mu;
  double kernel_ms = 0.0;
  int64_t kernel_launches = 0;
  double host_us[BIRES_HOST_PHASES] = {0};
  int64_t host_calls = 0;
  std::mutex crt_mu;
  std::map<int, std::pair<const uint32_t*, int>> crt;  // P -> (device CrtHost buffer, LM)
  std::atomic<int> eval_mode{BIRES_EVAL_AUTO};           // evaluation + elimination kernel (BIRES_EVAL_*)
  std::atomic<long long> schur_instances{0}, schur_fallbacks{0};  // Schur kernel statistics
  std::atomic<bool> graphs{false};                       // replay device sequences as captured graphs
  std::atomic<bool> plan_cache{true};                    // speculative reuse of the last call's plans
  SpecCache spec;
  std::mutex graph_mu;
  std::map<uint64_t, hipGraphExec_t> graph_cache;       // sequence hash -> instantiated graph
  std::vector<uint64_t> graph_order;                    // insertion order (oldest first)
  int64_t graph_captures = 0, graph_replays = 0;        // under graph_mu
  std::mutex itab_mu;                                   // interpolation block tables (interp_tables_device)
  uint32_t* itab = nullptr;
  int itab_nb = 0, itab_P = 0;
  size_t itab_qoff = 0;
  std::vector<uint32_t*> itab_retired;                  // outgrown tables (kernels in flight may still read them)
  std::mutex ev_mu;
  std::vector<hipEvent_t> ev_free;                      // completion events of batched calls, reused
  std::mutex vinv_mu;
  std::map<std::pair<int, int>, const int8_t*> vinv;   // (D, P) -> inverse Vandermonde digit planes
  size_t vinv_total = 0;
  // the fixed device array of allocation-free calls (its device address on
  // this context's device, from the symbol lookup at set-up) and the lock
  // that gives it to one call at a time
  uint8_t* scratch = nullptr;
  size_t scratch_bytes = 0;
  std::mutex scratch_mu;
};

// Device address of the allocation-free calls' scratch array on the current
// device (symbol lookup; csrc/scratch.hip) and its size in bytes.
int scratch_address(uint8_t** ptr, size_t* bytes);

// Captured device sequences keyed by the hash of their call arguments:
// graph_launch launches a cached one (false if absent or the launch failed);
// graph_store_launch caches a new executable (at most 32, the oldest is
// destroyed after a device synchronisation) and launches it.
bool graph_launch(Context* cx, uint64_t key, hipStream_t st);
bool graph_store_launch(Context* cx, uint64_t key, hipGraphExec_t exec, hipStream_t st);

// Inverse Vandermonde digit planes for nodes 0..D-1 and the first P primes,
// built on first use (on stream st, which is then synchronised) and kept;
// nullptr when it would exceed the cache limit or allocation fails.
const int8_t* vinv_device(Context* cx, int D, int P, hipStream_t st);
// Newton-to-monomial block tables for at least `blocks` blocks and `primes`
// primes, built on `st` and cached (grown when a call needs more); false when
// they would exceed 512 MiB or the build failed (the kernel then computes the
// blocks itself).  *nb receives the table's block count (its stride).
bool interp_tables_device(Context* cx, int blocks, int primes, hipStream_t st, const uint32_t** W,
                          const uint32_t** Q, int* nb);

// Device copy of crt_tables(P), built on first use and kept (nullptr on failure).
const uint32_t* crt_device(Context* cx, int P, int* LM);
// The same when it already exists, else nullptr (never allocates).
const uint32_t* crt_device_cached(Context* cx, int P, int* LM);

// Autotuning key of a planned batch: log2-buckets of the total (prime, point)
// instances, of the largest m + n and of the largest prime count.
std::string tune_key(long long instances, int max_r, int max_p);
// The schedule a batch with this key runs with (resolves BIRES_SCHEDULE_AUTO:
// the autotuner's choice for the key, else staged below 64k instances).
int schedule_for(Context* cx, const std::string& key);
void tune_load(Context* cx);
void tune_store(Context* cx, const std::string& key, int schedule);

// Returns the initialised context or nullptr (err set).
Context* context(int* err);
// The context if set-up has already run and succeeded, else nullptr (never
// initialises).
Context* context_if_ready();

// One job of a batch as the caller described it.
struct JobIn {
  bires_bipoly f, g;
  int kind = BIRES_KIND_RESULTANT;
  int var = BIRES_VAR_Y;
  bires_upoly* out = nullptr;
};

// Runs the jobs on `stream` (all buffers in memory space `mem`) and waits.
// status[i] receives each job's code; the return value is the first error.
int run_batch(Context* cx, const std::vector<JobIn>& jobs, int mem, hipStream_t stream, int32_t* status,
              std::vector<uint32_t>* debug_values = nullptr, std::vector<int>* debug_shape = nullptr);
// The same without allocating device or pinned memory: the call's device
// buffers lie in the scratch array (BIRES_ETOOBIG when they do not fit), its
// host staging in ordinary memory; staged schedule, per-job interpolation,
// the explicit CRT only where its tables already exist.  Calls are serialised.
int run_batch_noalloc(Context* cx, const std::vector<JobIn>& jobs, int mem, hipStream_t stream, int32_t* status);

// The same in two halves: run_batch_launch issues the device work and returns
// (its state in *pending, or an error before anything was queued);
// run_batch_finish waits for that work only (an event, not the stream) and
// completes the call.  Between the two, the caller's buffers belong to the call.
struct PendingBatch;
struct PendingDeleter {
  void operator()(PendingBatch* p) const;
};
using PendingPtr = std::unique_ptr<PendingBatch, PendingDeleter>;
int run_batch_launch(Context* cx, const std::vector<JobIn>& jobs, int mem, hipStream_t stream, int32_t* status,
                     PendingPtr* pending);
int run_batch_finish(PendingPtr pending);
// Marks a launched call as running on the library stream: a rerun inside
// run_batch_finish then holds cx->stream_mu.
void set_pending_stream_lock(PendingBatch* pending);

// One host-memory job as the kernels read it: the limb rectangles packed with
// rows = powers of the eliminated variable (g empty for the kinds derived
// from f), the row statistics of the two Sylvester operands and the plan.
struct HostJob {
  std::vector<uint32_t> f, g;
  int rows_f = 0, ld_f = 0, L_f = 1, rows_g = 0, ld_g = 0, L_g = 1;
  RowStats stf, stg;
  Plan pl;
};
int host_job(const JobIn& job, HostJob& h);

// Plan of one host-memory job, and output sizes from the extents only (host-only).
int bounds_job(const JobIn& job, int32_t* max_degree, int32_t* max_limbs);
int plan_host_job(const JobIn& job, Plan& pl);
// Output capacity (from the extents) and the device bytes one job holds while it runs.
int job_footprint(const JobIn& job, int32_t* cap_degree, int32_t* cap_limbs, size_t* bytes);

// Principal subresultant coefficients of a host-memory job modulo the table
// prime p (psc.cpp): out[i * D + c] for i < *count, c < *points.
int psc_count(int m, int n);
int run_psc(Context* cx, const JobIn& job, uint32_t p, uint32_t* out, int64_t capacity, int32_t* count,
            int32_t* points, hipStream_t st);
// N^- and N^+ of Section 3.2.2 for a host-memory curve f, R* and deg R.
int run_fiber_bounds(Context* cx, const bires_bipoly& f, int var, const bires_upoly& rstar, int32_t deg_r,
                     uint32_t p, int64_t* n_minus, int64_t* n_plus, int32_t* flags, hipStream_t st);

// Validates the descriptor of a bivariate input.
int check_bipoly(const bires_bipoly* p, int allow_null_c);

}  // namespace bires
