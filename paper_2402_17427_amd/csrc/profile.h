// RAII bracket of one enqueued stage with HIP events (active only while
// gs_profile_enable(1) is in effect).
#pragma once

#include <hip/hip_runtime.h>

namespace gs {

class ProfScope {
   public:
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

   private:
    const char* name_;
    hipStream_t st_;
    void* a_;
};

}  // namespace gs
