#include "common.h"

extern "C" {
mmm_status mmm_batch_create(const mmm_problem*, int32_t, const mmm_config*, void*, mmm_batch** out)
{
    if (out) *out = nullptr;
    return MMM_EUNSUPPORTED;
}
mmm_status mmm_batch_launch(mmm_batch*, void*) { return MMM_EUNSUPPORTED; }
mmm_status mmm_batch_destroy(mmm_batch*) { return MMM_OK; }
}
