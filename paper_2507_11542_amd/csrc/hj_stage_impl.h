// Fused TVD-RK stage kernel for gfx950: one launch evaluates, at every grid
// node, the one-sided derivatives along every axis (Sec. 3), the
// Lax-Friedrichs numerical Hamiltonian (Sec. 4) and the RK stage combination
// (Sec. 5), and applies the tube minimum on the last stage (Sec. 6.1).
//
// Stencil values come straight from global memory: the per-node stencil is a
// cross of 2w+1 points per axis, neighbours along the fastest axis are
// coalesced across a wavefront and the other axes hit L2 (the whole
// working set of one stage is a few MB).  Ghost values are formed on the fly:
// wrap-around on periodic axes, linear extrapolation v_{-k} = v_0 + k(v_0 - v_1)
// on bounded axes, so no padded copy of the grid exists.
#pragma once

#include "hj_internal.h"

namespace hj {

template <int SCH>
struct Halo;
template <>
struct Halo<kUpwind1> { static constexpr int w = 1; };
template <>
struct Halo<kEno2> { static constexpr int w = 2; };
template <>
struct Halo<kWeno5> { static constexpr int w = 3; };

// Jiang-Peng WENO5 approximation from five consecutive one-sided differences
// (Sec. 3.3; Osher-Fedkiw eqs. 3.28-3.39), eps = 1e-6 max v_k^2 + floor.
//
// FP64: candidates, smoothness indicators and weights in the written order
// with correctly rounded divisions, built without contraction, so every
// rounding equals that of a plain FP64 evaluation of the same formulas.  The
// discrete scheme amplifies rounding differences by up to ~1e11 over a long
// horizon near the ridges of a game's value function, so FP64 results are only
// comparable at 1e-12 when the rounding is reproduced.
// FP32: fused multiply-adds and hardware reciprocals (v_rcp_f32); the floor
// is 1e-18 because 1e-99 underflows in float.
template <typename T>
__device__ inline T weno5(T v1, T v2, T v3, T v4, T v5)
{
    constexpr T c13_12 = T(13.0 / 12.0);
    constexpr T c1_3 = T(1.0 / 3.0);
    constexpr T c1_6 = T(1.0 / 6.0);
    constexpr T c5_6 = T(5.0 / 6.0);
    constexpr T c7_6 = T(7.0 / 6.0);
    constexpr T c11_6 = T(11.0 / 6.0);

    const T phi1 = v1 * c1_3 - v2 * c7_6 + v3 * c11_6;
    const T phi2 = -v2 * c1_6 + v3 * c5_6 + v4 * c1_3;
    const T phi3 = v3 * c1_3 + v4 * c5_6 - v5 * c1_6;

    const T e1 = v1 - T(2) * v2 + v3, f1 = v1 - T(4) * v2 + T(3) * v3;
    const T e2 = v2 - T(2) * v3 + v4, f2 = v2 - v4;
    const T e3 = v3 - T(2) * v4 + v5, f3 = T(3) * v3 - T(4) * v4 + v5;
    const T s1 = c13_12 * e1 * e1 + T(0.25) * f1 * f1;
    const T s2 = c13_12 * e2 * e2 + T(0.25) * f2 * f2;
    const T s3 = c13_12 * e3 * e3 + T(0.25) * f3 * f3;

    T mx = v1 * v1;
    mx = fmax(mx, v2 * v2);
    mx = fmax(mx, v3 * v3);
    mx = fmax(mx, v4 * v4);
    mx = fmax(mx, v5 * v5);
    if constexpr (sizeof(T) == 8) {
        const T eps = T(1e-6) * mx + T(1e-99);
        const T a1 = T(0.1) / ((s1 + eps) * (s1 + eps));
        const T a2 = T(0.6) / ((s2 + eps) * (s2 + eps));
        const T a3 = T(0.3) / ((s3 + eps) * (s3 + eps));
        return (a1 * phi1 + a2 * phi2 + a3 * phi3) / (a1 + a2 + a3);
    } else {
        const T eps = T(1e-6) * mx + T(1e-18);
        const T a1 = T(0.1) * __builtin_amdgcn_rcpf((s1 + eps) * (s1 + eps));
        const T a2 = T(0.6) * __builtin_amdgcn_rcpf((s2 + eps) * (s2 + eps));
        const T a3 = T(0.3) * __builtin_amdgcn_rcpf((s3 + eps) * (s3 + eps));
        return (a1 * phi1 + a2 * phi2 + a3 * phi3) * __builtin_amdgcn_rcpf(a1 + a2 + a3);
    }
}

// ENO2 choice of the smaller second difference; ties go to the first (<=).
template <typename T>
__device__ inline T eno_pick(T a, T b)
{
    return fabs(a) <= fabs(b) ? a : b;
}

// Value at axis index j (possibly a ghost) of the grid line through `node`,
// whose own axis index is i.  Interior values are loaded; ghost values wrap
// (periodic) or extrapolate linearly from the two end nodes (bounded).
template <typename T>
__device__ inline T line_value(const T *__restrict__ v, uint32_t node, int i, int j, int n,
                               uint32_t stride, bool periodic)
{
    const uint32_t base = node - uint32_t(i) * stride;
    if (j >= 0 && j < n) return v[base + uint32_t(j) * stride];
    if (periodic) {
        const int jj = j < 0 ? j + n : j - n;
        return v[base + uint32_t(jj) * stride];
    }
    if (j < 0) {
        const T e0 = v[base], e1 = v[base + stride];
        return e0 + T(-j) * (e0 - e1);
    }
    const T e0 = v[base + uint32_t(n - 1) * stride], e1 = v[base + uint32_t(n - 2) * stride];
    return e0 + T(j - (n - 1)) * (e0 - e1);
}

// p- and p+ along one axis at one node (Sec. 3.1-3.3).
// First divided differences use the reciprocal cell size 1/dx, second ones
// 1/(2 dx) (both computed once on the host in FP64).
template <typename T, int SCH>
__device__ inline void axis_derivs(const T *__restrict__ v, uint32_t node, int i, int n,
                                   uint32_t stride, bool periodic, T dx, T inv_dx, T inv_2dx,
                                   T &pm, T &pp, T &center)
{
    constexpr int W = Halo<SCH>::w;
    T s[2 * W + 1];
    const bool interior = i >= W && i < n - W;
    if (interior) {
#pragma unroll
        for (int k = 0; k <= 2 * W; ++k) s[k] = v[node + (k - W) * int(stride)];
    } else {
#pragma unroll
        for (int k = 0; k <= 2 * W; ++k)
            s[k] = line_value(v, node, i, i - W + k, n, stride, periodic);
    }
    center = s[W];
    if constexpr (SCH == kUpwind1) {
        pm = (s[1] - s[0]) * inv_dx;
        pp = (s[2] - s[1]) * inv_dx;
    } else if constexpr (SCH == kEno2) {
        // divided-difference table of Sec. 3.2
        T d1[4], d2[3];
#pragma unroll
        for (int k = 0; k < 4; ++k) d1[k] = (s[k + 1] - s[k]) * inv_dx;
#pragma unroll
        for (int k = 0; k < 3; ++k) d2[k] = (d1[k + 1] - d1[k]) * inv_2dx;
        pm = d1[1] + dx * eno_pick(d2[0], d2[1]);
        pp = d1[2] - dx * eno_pick(d2[1], d2[2]);
    } else {
        T d1[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) d1[k] = (s[k + 1] - s[k]) * inv_dx;
        pm = weno5(d1[0], d1[1], d1[2], d1[3], d1[4]);
        pp = weno5(d1[5], d1[4], d1[3], d1[2], d1[1]);
    }
}

// H(x, p) of the compiled dynamics (sign convention V_t + H = 0).
template <typename T, int D, int DYN>
__device__ inline T hamiltonian(const StageArgs<T> &a, const int *ii, const T *p)
{
    if constexpr (DYN == kTranslation) {
        T h = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) h -= a.prm[d] * p[d];
        return h;
    } else if constexpr (DYN == kBall) {
        T s = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) s += p[d] * p[d];
        return a.prm[0] * sqrt(s);
    } else if constexpr (DYN == kDoubleIntegrator) {
        const T x2 = a.tab[a.tab_off[1] + ii[1]];
        return -p[0] * x2 + a.prm[0] * fabs(p[1]);
    } else if constexpr (DYN == kRelDubins) {
        const T ve = a.prm[0], vp = a.prm[1], we = a.prm[2], wp = a.prm[3];
        const T x = a.tab[a.tab_off[0] + ii[0]];
        const T y = a.tab[a.tab_off[1] + ii[1]];
        const T c = a.tab[a.tab_off[2] + a.n[2] + ii[2]];
        const T s = a.tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        return -p[0] * (-ve + vp * c) - p[1] * (vp * s) - we * fabs(p[0] * y - p[1] * x - p[2]) +
               wp * fabs(p[2]);
    } else {
        const T wm = a.prm[0], am = a.prm[1];
        const T c = a.tab[a.tab_off[2] + a.n[2] + ii[2]];
        const T s = a.tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        const T v = a.tab[a.tab_off[3] + ii[3]];
        return -p[0] * (v * c) - p[1] * (v * s) + wm * fabs(p[2]) + am * fabs(p[3]);
    }
}

// One node of one stage: derivatives along every axis, Lax-Friedrichs
// right-hand side, RK combination and tube minimum; writes a.out[node].
template <typename T, int D, int SCH, int DYN>
__device__ inline void stage_node(const StageArgs<T> &a, uint32_t node)
{
    int ii[D];
    {
        uint32_t r = node;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            ii[d] = int(r % a.n[d]);
            r /= a.n[d];
        }
    }
    T pm[D], pp[D], center = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d)
        axis_derivs<T, SCH>(a.vs, node, ii[d], int(a.n[d]), a.stride[d], (a.periodic >> d) & 1u,
                            a.dx[d], a.inv_dx[d], a.inv_2dx[d], pm[d], pp[d], center);
    T pbar[D];
#pragma unroll
    for (int d = 0; d < D; ++d) pbar[d] = (pp[d] + pm[d]) * T(0.5);
    T h = hamiltonian<T, D, DYN>(a, ii, pbar);
#pragma unroll
    for (int d = 0; d < D; ++d) h -= a.alpha[d] * ((pp[d] - pm[d]) * T(0.5));
    const T l = -h;

    T val;
    if (a.combine == kRhs) {
        val = l;
    } else {
        const T v2 = center + a.dt * l;
        if (a.combine == kEuler)
            val = v2;
        else
            val = (a.wb * a.vb[node] + a.w2 * v2) / a.den;
    }
    if (a.tube) val = fmin(val, a.v0[node]);
    a.out[node] = val;
}

template <typename T, int D, int SCH, int DYN>
__global__ __launch_bounds__(256) void stage_kernel(const StageArgs<T> a)
{
    const uint32_t node = blockIdx.x * 256u + threadIdx.x;
    if (node >= a.total) return;
    stage_node<T, D, SCH, DYN>(a, node);
}

template <typename T, int D, int SCH, int DYN>
hipError_t launch_one(const StageArgs<T> &a, hipStream_t s)
{
    const uint32_t blocks = (a.total + 255u) / 256u;
    hipLaunchKernelGGL((stage_kernel<T, D, SCH, DYN>), dim3(blocks), dim3(256), 0, s, a);
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
    }
    return hipErrorInvalidValue;
}

constexpr unsigned kAllSpaces = (1u << kUpwind1) | (1u << kEno2) | (1u << kWeno5);

}  // namespace hj
