// Scoped HIP-event timer around one kernel launch (no-op unless enabled by
// bmpc_profile_enable).
#pragma once

#include <hip/hip_runtime.h>

namespace bmpc {

bool profiling_enabled();

class ProfScope {
public:
    ProfScope(const char* name, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

private:
    const char* name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

}  // namespace bmpc
