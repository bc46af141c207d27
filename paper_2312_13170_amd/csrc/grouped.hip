// Grouped execution of many uneven problems (placeholder until the
// persistent grouped kernels land).
#include <hip/hip_runtime.h>

#include "li_internal.h"

struct li_group_plan {
    int count;
};

extern "C" {

li_status li_group_plan_create(const li_problem *problems, int32_t count, li_group_plan **plan)
{
    (void)problems;
    (void)count;
    (void)plan;
    return li::fail(LI_ERR_NOT_FOUND, "grouped plans are not available in this build");
}

li_status li_group_plan_launch(li_group_plan *plan, li_stream stream)
{
    (void)plan;
    (void)stream;
    return li::fail(LI_ERR_NOT_FOUND, "grouped plans are not available in this build");
}

li_status li_group_plan_launch_loop(li_group_plan *plan, li_stream stream)
{
    (void)plan;
    (void)stream;
    return li::fail(LI_ERR_NOT_FOUND, "grouped plans are not available in this build");
}

double li_group_plan_flops(const li_group_plan *plan)
{
    (void)plan;
    return 0.0;
}

void li_group_plan_destroy(li_group_plan *plan) { (void)plan; }

}  // extern "C"
