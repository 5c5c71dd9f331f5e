// Fixed device-resident scratch for the entry point that allocates nothing
// (bb_synth_collect_eig_noalloc): the staging area and metadata of one
// instance live in this file-scope array instead of a caller's workspace.
//
// In host code the name `scratch` is a host-side stand-in, not a device
// address.  The only host use of it is the symbol lookup below, made once per
// device with that device current; every kernel argument and copy uses the
// address the lookup returned.  Each device holds its own copy of the array
// until the process ends.

#include <hip/hip_runtime.h>

#include "bb_internal.h"

static __device__ __align__(256) unsigned char scratch[bb::kNoallocScratchBytes];

namespace bb {

hipError_t noalloc_scratch_address(void** out) {
  if (!out) return hipErrorInvalidValue;
  *out = nullptr;
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

}  // namespace bb
