// FP32-bulk / FP64-boundary helpers of hj_solve_mixed: rounding the FP64
// initial values to the FP32 working arrays, and the FP64 tube finalisation
// near the zero level set (Sec. 6.1 tube, V <- min(V, V0), taken in FP64 on
// the band |V| <= band where the zero level set lies).  Also the scan for
// non-finite values behind the optional result check.
#include "hj_internal.h"

namespace hj {

namespace {

__global__ __launch_bounds__(256) void round_to_f32(const double *__restrict__ src,
                                                     float *__restrict__ dst, uint32_t n)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        dst[i] = float(src[i]);
}

__global__ __launch_bounds__(256) void finalize_f64(const float *__restrict__ v32,
                                                     const double *__restrict__ v0,
                                                     double *__restrict__ out, uint32_t n,
                                                     double band, int tube)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double v = double(v32[i]);
        out[i] = (tube && fabs(v) <= band) ? fmin(v, v0[i]) : v;
    }
}

// flag <- 0 (a kernel, not a memset node, so the call may be captured)
__global__ void clear_flag(int *flag) { *flag = 0; }

// flag <- 1 if any of v[0..n) is NaN or infinite (every writer writes the
// same value, so no atomics are needed)
template <typename T>
__global__ __launch_bounds__(256) void scan_nonfinite(const T *__restrict__ v, uint32_t n,
                                                       int *flag)
{
    bool bad = false;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        bad |= !isfinite(v[i]);
    if (bad) *flag = 1;
}

uint32_t grid_for(uint32_t n)
{
    const uint32_t b = (n + 255) / 256;
    return b < 4096 ? (b ? b : 1) : 4096;
}

}  // namespace

hipError_t launch_round_to_f32(const double *src, float *dst, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(round_to_f32, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_finalize_f64(const float *v32, const double *v0, double *out, uint32_t n,
                               double band, int tube, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_f64, dim3(grid_for(n)), dim3(256), 0, s, v32, v0, out, n, band,
                       tube);
    return hipGetLastError();
}

hipError_t launch_scan_nonfinite(const void *v, int fp64, uint32_t n, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, s, flag);
    if (fp64)
        hipLaunchKernelGGL(scan_nonfinite<double>, dim3(grid_for(n)), dim3(256), 0, s,
                           (const double *)v, n, flag);
    else
        hipLaunchKernelGGL(scan_nonfinite<float>, dim3(grid_for(n)), dim3(256), 0, s,
                           (const float *)v, n, flag);
    return hipGetLastError();
}

}  // namespace hj
