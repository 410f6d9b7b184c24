// Stage launchers: the fused per-node kernel for every dimension, scheme and
// dynamics (template instantiation by dispatch on the runtime enums).
#pragma once

#include "hj_stage_impl.h"

namespace hj {

template <typename T, int D, int SCH, int DYN>
hipError_t launch_one(const StageArgs<T> &a, hipStream_t s)
{
    const uint32_t blocks = (a.total + 255u) / 256u;
    if (!a.addr64 && fits_off32<T>(a.total))
        hipLaunchKernelGGL((stage_kernel<T, D, SCH, DYN, true>), dim3(blocks), dim3(256), 0, s,
                           a);
    else
        hipLaunchKernelGGL((stage_kernel<T, D, SCH, DYN, false>), dim3(blocks), dim3(256), 0, s,
                           a);
    return hipGetLastError();
}

// SPACES: bit mask of the derivative schemes this translation unit builds
// (1 << scheme); the others return hipErrorInvalidValue.
template <typename T, int D, int DYN, unsigned SPACES>
hipError_t launch_space(int space, const StageArgs<T> &a, hipStream_t s)
{
    if constexpr ((SPACES >> kUpwind1) & 1u)
        if (space == kUpwind1) return launch_one<T, D, kUpwind1, DYN>(a, s);
    if constexpr ((SPACES >> kEno2) & 1u)
        if (space == kEno2) return launch_one<T, D, kEno2, DYN>(a, s);
    if constexpr ((SPACES >> kEno3) & 1u)
        if (space == kEno3) return launch_one<T, D, kEno3, DYN>(a, s);
    if constexpr ((SPACES >> kWeno5) & 1u)
        if (space == kWeno5) return launch_one<T, D, kWeno5, DYN>(a, s);
    return hipErrorInvalidValue;
}

template <typename T, unsigned SPACES>
hipError_t launch_stage_t(int ndim, int space, int dyn, const StageArgs<T> &a, hipStream_t s)
{
    switch (dyn) {
    case kTranslation:
        switch (ndim) {
        case 1: return launch_space<T, 1, kTranslation, SPACES>(space, a, s);
        case 2: return launch_space<T, 2, kTranslation, SPACES>(space, a, s);
        case 3: return launch_space<T, 3, kTranslation, SPACES>(space, a, s);
        case 4: return launch_space<T, 4, kTranslation, SPACES>(space, a, s);
        }
        break;
    case kBall:
        switch (ndim) {
        case 1: return launch_space<T, 1, kBall, SPACES>(space, a, s);
        case 2: return launch_space<T, 2, kBall, SPACES>(space, a, s);
        case 3: return launch_space<T, 3, kBall, SPACES>(space, a, s);
        case 4: return launch_space<T, 4, kBall, SPACES>(space, a, s);
        }
        break;
    case kDoubleIntegrator:
        if (ndim == 2) return launch_space<T, 2, kDoubleIntegrator, SPACES>(space, a, s);
        break;
    case kRelDubins:
        if (ndim == 3) return launch_space<T, 3, kRelDubins, SPACES>(space, a, s);
        break;
    case kDubins4D:
        if (ndim == 4) return launch_space<T, 4, kDubins4D, SPACES>(space, a, s);
        break;
    case kRockets:
        if (ndim == 3) return launch_space<T, 3, kRockets, SPACES>(space, a, s);
        break;
    }
    return hipErrorInvalidValue;
}

constexpr unsigned kAllSpaces =
    (1u << kUpwind1) | (1u << kEno2) | (1u << kEno3) | (1u << kWeno5);


}  // namespace hj
