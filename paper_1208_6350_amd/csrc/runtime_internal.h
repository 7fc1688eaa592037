// runtime_internal.h -- host-side hooks shared by the runtime and the server
// (C++ linkage: not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/swx.h"

namespace swx {
// records msg as the calling thread's last error and returns code
int internal_fail(int code, const char *msg);
// the context's stream (work queued on it runs before the context's next call)
hipStream_t internal_stream(swx_ctx *ctx);
// the context's HIP device ordinal
int internal_device(const swx_ctx *ctx);
}  // namespace swx
