// Batched plans and the autotuner (placeholder until the kernels land).
#include "host_common.hpp"

struct lip_plan {
    int dummy;
};

extern "C" lip_status lip_plan_create(lip_plan **plan, const lip_batch_desc *, int32_t, uint32_t,
                                      lip_stream)
{
    if (plan) *plan = nullptr;
    return LIP_E_UNSUPPORTED;
}
extern "C" lip_status lip_plan_execute(lip_plan *, lip_stream) { return LIP_E_UNSUPPORTED; }
extern "C" lip_status lip_plan_destroy(lip_plan *) { return LIP_OK; }
extern "C" lip_status lip_autotune(int32_t, int32_t, int32_t, int64_t, int64_t, lip_stream,
                                   lip_tile_cfg *)
{
    return LIP_E_UNSUPPORTED;
}
