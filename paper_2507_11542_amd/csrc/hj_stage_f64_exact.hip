// FP64 first-order and ENO2 instantiations of the fused stage kernel, built
// with -ffp-contract=off (see build_lib.py): every product and sum is rounded
// on its own, in the order the formulas are written, so ENO2's choice between
// two second differences (a comparison of |D2| values) is taken on the same
// values as a plain FP64 evaluation of the paper's divided-difference table.
#include "hj_stage_impl.h"

namespace hj {
hipError_t launch_stage_f64_exact(int ndim, int space, int dyn, const StageArgs<double> &a,
                                  hipStream_t s)
{
    return launch_stage_t<double, (1u << kUpwind1) | (1u << kEno2)>(ndim, space, dyn, a, s);
}
}  // namespace hj
