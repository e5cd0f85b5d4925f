// Batched persistent AFMM (placeholder until the persistent kernel lands).
#include "afmm.h"

extern "C" {
afmm_status afmm_plan_create(const afmm_problem*, int32_t, afmm_mode, afmm_plan**) {
    return AFMM_ERR_UNSUPPORTED;
}
afmm_status afmm_plan_launch(afmm_plan*, hipStream_t) { return AFMM_ERR_UNSUPPORTED; }
afmm_status afmm_plan_problem_adds(const afmm_plan*, uint64_t*, hipStream_t) {
    return AFMM_ERR_UNSUPPORTED;
}
afmm_status afmm_plan_destroy(afmm_plan*) { return AFMM_ERR_UNSUPPORTED; }
afmm_status afmm_multiply_batched(const afmm_problem*, int32_t, afmm_mode, hipStream_t) {
    return AFMM_ERR_UNSUPPORTED;
}
}
