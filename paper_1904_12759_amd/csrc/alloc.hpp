// Device and pinned-host allocations of the library, with a fault-injection
// hook for tests of the out-of-memory paths: with MC_EXPMV_FAULT=alloc:K in the
// environment, the K-th allocation made during one entry-point call fails with
// hipErrorOutOfMemory (nothing is allocated), so that call's cleanup and its
// MC_ERR_NO_MEMORY can be checked.  Entry points that allocate call
// fault_scope_begin() first, which re-reads the variable and restarts the count
// (per host thread).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mc {

void fault_scope_begin();
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t host_malloc(void **p, size_t bytes);

}  // namespace mc
