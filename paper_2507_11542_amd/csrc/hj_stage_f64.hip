// FP64 WENO5 instantiations of the fused stage kernel, built with fused
// multiply-add contraction.  WENO5 takes no discrete decision, so rounding
// differences from a plain FP64 evaluation stay at rounding level.  The
// first-order and ENO2 schemes go to the contraction-free translation unit.
#include "hj_stage_impl.h"

namespace hj {
hipError_t launch_stage_f64_exact(int ndim, int space, int dyn, const StageArgs<double> &a,
                                  hipStream_t s);

hipError_t launch_stage_f64(int ndim, int space, int dyn, const StageArgs<double> &a,
                            hipStream_t s)
{
    if (space != kWeno5) return launch_stage_f64_exact(ndim, space, dyn, a, s);
    return launch_stage_t<double, (1u << kWeno5)>(ndim, space, dyn, a, s);
}
}  // namespace hj
