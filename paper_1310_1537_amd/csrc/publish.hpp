// Cross-block publication within one launch (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace glmk {

// Data that one block of a launch writes and another block of the same
// launch reads after a ticket (the merge's partials).  The L2 caches of the
// XCDs are not coherent with each other; an agent-scope release fence would
// make plain stores visible by writing back the writer's whole L2, and the
// matching acquire invalidates the reader's, several microseconds per launch.
// Instead such data is written with agent-scope atomic stores, which write
// through to memory, and read with agent-scope atomic loads (cache policy
// sc1), which do not hit stale lines.  Before the block barrier that precedes
// its ticket every thread waits for its own stores to complete, so the block
// whose ticket completes a count reads completed stores only.  In the AMDGPU
// memory model of gfx942-class targets the release fence is that same wait
// plus the L2 write-back, and the write-back serves non-atomic stores only.
__device__ __forceinline__ void publish(double* a, double v) {
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double fetch_published(const double* a) {
    return __hip_atomic_load(const_cast<double*>(a), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Buffer-load cache policy of an agent-scope atomic load (sc1).
constexpr int kLoadPublished = 16;

}  // namespace glmk
