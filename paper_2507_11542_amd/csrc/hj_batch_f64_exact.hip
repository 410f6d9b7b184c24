// FP64 instantiations of the batched round kernel, built without
// contraction like the FP64 single-solve kernels (same per-node arithmetic,
// so a batched instance equals its plain solve bit for bit).
#include "hj_batch_impl.h"

namespace hj {
hipError_t batch_launch_f64(int ndim, int space, int dyn, const BatchPtrs<double> &p,
                            uint32_t rounds, const BatchShape &shape, hipStream_t s)
{
    return batch_launch_t<double>(ndim, space, dyn, p, rounds, shape, s);
}
}  // namespace hj
