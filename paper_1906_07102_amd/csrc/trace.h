// Scoped per-kernel timing (enabled by lmg_trace_enable or LMG_TRACE=1).
#pragma once

#include <hip/hip_runtime.h>

#include "lmg_internal.h"

namespace lmg {
class TraceScope {
  public:
    TraceScope(const char* name, hipStream_t s);
    ~TraceScope();
    TraceScope(const TraceScope&) = delete;
    TraceScope& operator=(const TraceScope&) = delete;

  private:
    const char* name_;
    hipStream_t s_;
    hipEvent_t a_{}, b_{};
    bool active_ = false;
};
}  // namespace lmg
