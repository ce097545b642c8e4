// Asynchronous batched calls (bires_resultant_batch_async / bires_batch_wait).
#pragma once
#include <stdint.h>

#include <vector>

#include "engine.hpp"

namespace bires {

// Plans the batch and queues its device work on `caller` (the library stream
// when null), after the work queued there before, and returns; an error found
// before anything was queued is returned here.  *ticket names the call for
// async_wait, which blocks until it has finished and returns its run_batch
// code (BIRES_EINVAL for an unknown or already collected ticket).
int async_submit(Context* cx, std::vector<JobIn>&& jobs, int mem, int32_t* status, hipStream_t caller,
                 uint64_t* ticket);
int async_wait(Context* cx, uint64_t ticket);

}  // namespace bires
