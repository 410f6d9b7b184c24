// Grid-wide costate box of one stage input (the global Lax-Friedrichs
// coefficients of Sec. 4 take the one-sided derivatives of the whole grid):
// per axis the minimum and maximum over all nodes of both p- and p+.
// Pass 1: every workgroup folds a grid-stride slice of nodes (the same
// derivative code as the stage kernel), reduces across its wavefronts with
// cross-lane shuffles and across its four wavefronts through LDS, and writes
// one partial [lo, hi] per axis.  Pass 2: one workgroup folds the partials.
// Minimum and maximum are exact, so the result does not depend on the order;
// no atomics, no memset.
#pragma once

#include "hj_stage_impl.h"

namespace hj {

constexpr uint32_t kBoxMaxBlocks = 1024;

inline uint32_t box_blocks(uint32_t total)
{
    const uint32_t b = (total + 255u) / 256u;
    return b < kBoxMaxBlocks ? (b ? b : 1u) : kBoxMaxBlocks;
}

template <typename T>
__device__ inline T wave_min(T x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const T y = __shfl_xor(x, off, 64);
        x = y < x ? y : x;
    }
    return x;
}

template <typename T>
__device__ inline T wave_maxv(T x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const T y = __shfl_xor(x, off, 64);
        x = y > x ? y : x;
    }
    return x;
}

// Folds lo[D], hi[D] of the workgroup into out[2d], out[2d + 1].
template <typename T, int D>
__device__ inline void box_block_reduce(const T *lo, const T *hi, T *out)
{
    __shared__ T lds[4][2 * D];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const T l = wave_min(lo[d]);
        const T h = wave_maxv(hi[d]);
        if (lane == 0) {
            lds[wave][2 * d] = l;
            lds[wave][2 * d + 1] = h;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        const int k = threadIdx.x;
        T r = lds[0][k];
        for (int w = 1; w < 4; ++w) {
            const T v = lds[w][k];
            if (k & 1)
                r = v > r ? v : r;
            else
                r = v < r ? v : r;
        }
        out[k] = r;
    }
}

template <typename T, int D, int SCH>
__global__ __launch_bounds__(256) void box_partial(const StageArgs<T> a, T *partial)
{
    T lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = T(INFINITY);
        hi[d] = T(-INFINITY);
    }
    for (uint32_t node = blockIdx.x * 256u + threadIdx.x; node < a.total;
         node += gridDim.x * 256u) {
        int ii[D];
        node_indices<T, D>(a, node, ii);
        T center;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T pm, pp;
            axis_derivs<T, SCH>(Arr<T, false>{global_ptr(a.vs)}, node, ii[d], int(a.n[d]), a.stride[d],
                                (a.periodic >> d) & 1u, a.dx[d], a.inv_dx[d], a.inv_2dx[d],
                                a.inv_3dx[d], pm, pp, center, d == D - 1);
            const T l = pm < pp ? pm : pp, h = pm < pp ? pp : pm;
            lo[d] = l < lo[d] ? l : lo[d];
            hi[d] = h > hi[d] ? h : hi[d];
        }
    }
    box_block_reduce<T, D>(lo, hi, partial + size_t(blockIdx.x) * 2 * D);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void box_final(const T *partial, uint32_t blocks, T *box)
{
    T lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = T(INFINITY);
        hi[d] = T(-INFINITY);
    }
    for (uint32_t b = threadIdx.x; b < blocks; b += 256u) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const T l = partial[size_t(b) * 2 * D + 2 * d];
            const T h = partial[size_t(b) * 2 * D + 2 * d + 1];
            lo[d] = l < lo[d] ? l : lo[d];
            hi[d] = h > hi[d] ? h : hi[d];
        }
    }
    box_block_reduce<T, D>(lo, hi, box);
}

template <typename T, int D, int SCH>
hipError_t box_run(const StageArgs<T> &a, T *partial, T *box, hipStream_t s)
{
    const uint32_t blocks = box_blocks(a.total);
    hipLaunchKernelGGL((box_partial<T, D, SCH>), dim3(blocks), dim3(256), 0, s, a, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((box_final<T, D>), dim3(1), dim3(256), 0, s, partial, blocks, box);
    return hipGetLastError();
}

template <typename T, int D>
hipError_t box_space(int space, const StageArgs<T> &a, T *partial, T *box, hipStream_t s)
{
    switch (space) {
    case kUpwind1: return box_run<T, D, kUpwind1>(a, partial, box, s);
    case kEno2: return box_run<T, D, kEno2>(a, partial, box, s);
    case kEno3: return box_run<T, D, kEno3>(a, partial, box, s);
    case kWeno5: return box_run<T, D, kWeno5>(a, partial, box, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t box_launch_t(int ndim, int space, const StageArgs<T> &a, T *partial, T *box,
                        hipStream_t s)
{
    switch (ndim) {
    case 1: return box_space<T, 1>(space, a, partial, box, s);
    case 2: return box_space<T, 2>(space, a, partial, box, s);
    case 3: return box_space<T, 3>(space, a, partial, box, s);
    case 4: return box_space<T, 4>(space, a, partial, box, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hj
