// Form (2): persistent box-per-workgroup stepping of many small boxes.
#include <hip/hip_runtime.h>

#include "md_internal.h"

namespace mdk {

int batched_prepare(Ctx &c)
{
    (void)c;
    return MD_OK;
}

void launch_batched_steps(Ctx &c, int nsteps, hipStream_t s)
{
    (void)c;
    (void)nsteps;
    (void)s;
}

}  // namespace mdk
