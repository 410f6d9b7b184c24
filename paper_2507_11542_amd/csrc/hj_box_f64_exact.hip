// FP64 instantiations of the grid-wide costate box reduction, built without
// contraction like the FP64 stage kernels (the same derivative values).
#include "hj_box_impl.h"

namespace hj {
uint32_t box_partial_values(uint32_t total, int ndim) { return box_blocks(total) * 2u * ndim; }

hipError_t launch_box_f64(int ndim, int space, const StageArgs<double> &a, double *partial,
                          double *box, hipStream_t s)
{
    return box_launch_t<double>(ndim, space, a, partial, box, s);
}
}  // namespace hj
