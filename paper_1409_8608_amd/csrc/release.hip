// Release of a plan's device workspace.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace tc {

void release_plan_device(tc_plan_s* p) {
    void** bufs[] = {&p->d_ktab, &p->d_var_ktab, &p->d_temp[0], &p->d_temp[1], &p->d_temp[2], &p->d_split, &p->d_splitk,
                     &p->d_zexp};
    for (void** b : bufs) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
}

}  // namespace tc

