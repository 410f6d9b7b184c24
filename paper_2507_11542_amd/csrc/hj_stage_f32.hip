// FP32 instantiations of the fused stage kernel (FP32 storage and arithmetic;
// alpha, dt and t are double on the host and rounded once per launch).
#include "hj_launch_impl.h"

namespace hj {
hipError_t launch_stage_f32(int ndim, int space, int dyn, const StageArgs<float> &a,
                            hipStream_t s)
{
    return launch_stage_t<float, kAllSpaces>(ndim, space, dyn, a, s);
}
}  // namespace hj
