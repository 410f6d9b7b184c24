// FP32 instantiations of the batched round kernel (FP32 bulk, FP64 t).
#include "hj_batch_impl.h"

namespace hj {
hipError_t batch_launch_f32(int ndim, int space, int dyn, const BatchPtrs<float> &p,
                            uint32_t rounds, const BatchShape &shape, hipStream_t s)
{
    return batch_launch_t<float>(ndim, space, dyn, p, rounds, shape, s);
}
}  // namespace hj
