// Optional per-kernel event timing around the library's launches.
#pragma once
#include <hip/hip_runtime.h>

namespace sfoc {
// Record the start / end event of one launch of kernel `kid` on `st` (no-op
// unless tracing is enabled).
void trace_begin(hipStream_t st, int kid);
void trace_end(hipStream_t st, int kid);
}  // namespace sfoc
