// FP32 instantiations of the grid-wide costate box reduction.
#include "hj_box_impl.h"

namespace hj {
hipError_t launch_box_f32(int ndim, int space, const StageArgs<float> &a, float *partial,
                          float *box, hipStream_t s)
{
    return box_launch_t<float>(ndim, space, a, partial, box, s);
}
}  // namespace hj
