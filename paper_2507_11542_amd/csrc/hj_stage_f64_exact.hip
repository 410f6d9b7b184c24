// FP64 instantiations of the fused stage kernel, built with -ffp-contract=off
// (see build_lib.py): every product and sum is rounded on its own, in the
// order the formulas are written, and divisions are correctly rounded.  The
// result is the rounding of a plain FP64 evaluation of the same formulas, so
// ENO2's choice between two second differences and WENO5's weights see the
// same values as such an evaluation, step after step.
#include "hj_launch_impl.h"

namespace hj {
hipError_t launch_stage_f64(int ndim, int space, int dyn, const StageArgs<double> &a,
                            hipStream_t s)
{
    return launch_stage_t<double, kAllSpaces>(ndim, space, dyn, a, s);
}
}  // namespace hj
