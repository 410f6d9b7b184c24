// Lax-Friedrichs dissipation coefficients on the GPU (Sec. 4): alpha_d is the
// maximum over all grid nodes of the bound max_{u,d} |f_d(x,u,d)| = |dH/dp_d|
// of the compiled dynamics.  FP64 in both precisions.
//
// Pass 1: every workgroup folds a grid-stride slice of nodes, reduces across
// its 64-lane wavefronts with cross-lane shuffles, then across its four
// wavefronts through LDS, and writes one partial maximum per axis.
// Pass 2: one workgroup folds the partials.  No atomics, no memset: the
// result is deterministic and the sequence is safe to capture in a graph.
#include "hj_internal.h"

namespace hj {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kMaxBlocks = 1024;

// Per-node speed bound along axis d.  Contraction is off so every node's
// bound is the plain product/sum of its terms.
template <int DYN>
__device__ inline double speed_bound(const AlphaArgs &a, const int *ii, int d)
{
#pragma clang fp contract(off)
    if constexpr (DYN == kTranslation) {
        return fabs(a.prm[d]);
    } else if constexpr (DYN == kBall) {
        return fabs(a.prm[0]);
    } else if constexpr (DYN == kDoubleIntegrator) {
        if (d == 0) return fabs(a.tab[a.tab_off[1] + ii[1]]);
        return a.prm[0];
    } else if constexpr (DYN == kRelDubins) {
        const double ve = a.prm[0], vp = a.prm[1], we = a.prm[2], wp = a.prm[3];
        const double x = a.tab[a.tab_off[0] + ii[0]];
        const double y = a.tab[a.tab_off[1] + ii[1]];
        const double c = a.tab[a.tab_off[2] + a.n[2] + ii[2]];
        const double s = a.tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        if (d == 0) return fabs(-ve + vp * c) + we * fabs(y);
        if (d == 1) return fabs(vp * s) + we * fabs(x);
        return we + wp;
    } else if constexpr (DYN == kRockets) {
        const double am = a.prm[0], grav = a.prm[1], um = a.prm[2];
        const double x = a.tab[a.tab_off[0] + ii[0]];
        const double c = a.tab[a.tab_off[2] + a.n[2] + ii[2]];
        const double s = a.tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        if (d == 0) return fabs(am * c) + um * fabs(x);
        if (d == 1) return fabs(am * s + am - grav) + um * fabs(x);
        return 2.0 * um;
    } else {
        const double c = a.tab[a.tab_off[2] + a.n[2] + ii[2]];
        const double s = a.tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        const double v = a.tab[a.tab_off[3] + ii[3]];
        if (d == 0) return fabs(v * c);
        if (d == 1) return fabs(v * s);
        if (d == 2) return a.prm[0];
        return a.prm[1];
    }
}

__device__ inline double wave_max(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

template <int D, int DYN>
__global__ __launch_bounds__(kThreads) void alpha_partial(const AlphaArgs a, double *partial)
{
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = 0.0;
    for (uint32_t node = blockIdx.x * kThreads + threadIdx.x; node < a.total;
         node += gridDim.x * kThreads) {
        int ii[D];
        uint32_t r = node;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            ii[d] = int(r % a.n[d]);
            r /= a.n[d];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) m[d] = fmax(m[d], speed_bound<DYN>(a, ii, d));
    }
    __shared__ double lds[kWaves][D];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double w = wave_max(m[d]);
        if (lane == 0) lds[wave][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < D) {
        double r = lds[0][threadIdx.x];
        for (int w = 1; w < kWaves; ++w) r = fmax(r, lds[w][threadIdx.x]);
        partial[blockIdx.x * D + threadIdx.x] = r;
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void alpha_final(const double *partial, uint32_t blocks,
                                                         double *alpha)
{
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = 0.0;
    for (uint32_t b = threadIdx.x; b < blocks; b += kThreads)
#pragma unroll
        for (int d = 0; d < D; ++d) m[d] = fmax(m[d], partial[b * D + d]);
    __shared__ double lds[kWaves][D];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double w = wave_max(m[d]);
        if (lane == 0) lds[wave][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < D) {
        double r = lds[0][threadIdx.x];
        for (int w = 1; w < kWaves; ++w) r = fmax(r, lds[w][threadIdx.x]);
        alpha[threadIdx.x] = r;
    }
}

template <int D, int DYN>
hipError_t run(const AlphaArgs &a, double *partial, double *alpha, hipStream_t s)
{
    const uint32_t blocks = alpha_blocks(a.total);
    hipLaunchKernelGGL((alpha_partial<D, DYN>), dim3(blocks), dim3(kThreads), 0, s, a, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((alpha_final<D>), dim3(1), dim3(kThreads), 0, s, partial, blocks, alpha);
    return hipGetLastError();
}

}  // namespace

uint32_t alpha_blocks(uint32_t total)
{
    uint32_t b = (total + kThreads - 1) / kThreads;
    return b < kMaxBlocks ? (b ? b : 1) : kMaxBlocks;
}

hipError_t launch_alpha(int ndim, int dyn, const AlphaArgs &a, double *partial, double *alpha,
                        hipStream_t s)
{
    switch (dyn) {
    case kTranslation:
        switch (ndim) {
        case 1: return run<1, kTranslation>(a, partial, alpha, s);
        case 2: return run<2, kTranslation>(a, partial, alpha, s);
        case 3: return run<3, kTranslation>(a, partial, alpha, s);
        case 4: return run<4, kTranslation>(a, partial, alpha, s);
        }
        break;
    case kBall:
        switch (ndim) {
        case 1: return run<1, kBall>(a, partial, alpha, s);
        case 2: return run<2, kBall>(a, partial, alpha, s);
        case 3: return run<3, kBall>(a, partial, alpha, s);
        case 4: return run<4, kBall>(a, partial, alpha, s);
        }
        break;
    case kDoubleIntegrator:
        if (ndim == 2) return run<2, kDoubleIntegrator>(a, partial, alpha, s);
        break;
    case kRelDubins:
        if (ndim == 3) return run<3, kRelDubins>(a, partial, alpha, s);
        break;
    case kRockets:
        if (ndim == 3) return run<3, kRockets>(a, partial, alpha, s);
        break;
    case kDubins4D:
        if (ndim == 4) return run<4, kDubins4D>(a, partial, alpha, s);
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace hj
