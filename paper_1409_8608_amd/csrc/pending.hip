// Entry points whose implementation lands in later files.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace tc {

void release_plan_device(tc_plan_s* p) {
    void** bufs[] = {&p->d_ktab, &p->d_var_ktab, &p->d_temp[0], &p->d_temp[1], &p->d_split};
    for (void** b : bufs) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
}

}  // namespace tc

extern "C" {
tc_status tc_batch_create(tc_batch_t* out, const tc_plan_t*, int) {
    if (out) *out = nullptr;
    return tc::fail(TC_E_UNSUPPORTED, "batches not built yet");
}
tc_status tc_batch_tune(tc_batch_t, int) { return tc::fail(TC_E_UNSUPPORTED, "batches not built yet"); }
tc_status tc_batch_contract(tc_batch_t, const void* const*, const void* const*, void* const*, const double*,
                            const double*, void*) {
    return tc::fail(TC_E_UNSUPPORTED, "batches not built yet");
}
tc_status tc_batch_destroy(tc_batch_t) { return TC_OK; }
}
