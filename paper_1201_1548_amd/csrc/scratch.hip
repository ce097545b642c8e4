// The fixed device array behind the allocation-free entry point
// (bires_resultant_noalloc): its definition and the one lookup of its device
// address live in this file.  Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in); it uses the
// address scratch_address() returns, which the context keeps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bires.h"

namespace bires {

static __device__ __align__(256) uint8_t scratch[BIRES_NOALLOC_SCRATCH_BYTES];

// Called once per device at library set-up, with that device current.
int scratch_address(uint8_t** ptr, size_t* bytes) {
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return BIRES_EDEVICE;
  }
  *ptr = (uint8_t*)p;
  *bytes = (size_t)BIRES_NOALLOC_SCRATCH_BYTES;
  return BIRES_OK;
}

}  // namespace bires
