// batch.cpp -- batched entry points (work-list build, persistent launch, plans).
#include "kr_api_internal.h"

using namespace kr;

extern "C" {

size_t kr_resize_batch_workspace_size(int n) { return n > 0 ? (size_t)n * 256 : 0; }

kr_status kr_resize_batch(const kr_batch_item *, int, int, kr_dtype, kr_dtype, kr_border, float,
                          const kr_normalize *, void *, size_t, void *)
{
    clear_error();
    return fail(KR_ERR_UNSUPPORTED, "batched launch not available in this build");
}

kr_status kr_batch_plan_create(const kr_batch_item *, int, int, kr_dtype, kr_dtype, kr_border, float,
                               const kr_normalize *, kr_batch_plan **plan)
{
    clear_error();
    if (plan)
        *plan = nullptr;
    return fail(KR_ERR_UNSUPPORTED, "batched launch not available in this build");
}

kr_status kr_batch_plan_launch(kr_batch_plan *, void *)
{
    clear_error();
    return fail(KR_ERR_UNSUPPORTED, "batched launch not available in this build");
}

void kr_batch_plan_destroy(kr_batch_plan *) {}

}  // extern "C"
