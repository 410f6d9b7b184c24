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

#include "hj_divseq.h"
#include "hj_internal.h"

namespace hj {

// Device pointers taken into the global address space, so that loads and
// stores through them are global (vector-memory) instructions whatever the
// pointer's origin: a kernel argument, or a table in device memory (batched
// launches), where the compiler would otherwise emit flat instructions, which
// also wait on the LDS counter.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ inline const gmem<T> *global_ptr(const T *p)
{
    return (const gmem<T> *)p;
}

template <typename T>
__device__ inline gmem<T> *global_ptr(T *p)
{
    return (gmem<T> *)p;
}

// An array of the grid read by node index.  OFF32: the element's byte offset
// is formed in 32 bits (for arrays under 4 GiB), so the compiler can load from
// the array's base in scalar registers plus a 32-bit offset per lane instead
// of forming a 64-bit address per load (measured 3-6 % faster FP32 stages).
template <typename T, bool OFF32>
struct Arr {
    const gmem<T> *p;
    __device__ T operator[](uint32_t i) const { return *elem(i); }
    __device__ const gmem<T> *elem(uint32_t i) const
    {
        if constexpr (OFF32) {
            using gbyte = __attribute__((address_space(1))) const char;
            return (const gmem<T> *)((gbyte *)p + i * uint32_t(sizeof(T)));
        } else {
            return p + i;
        }
    }
};

template <bool OFF32, typename T>
__device__ inline gmem<T> *elem_at(gmem<T> *p, uint32_t i)
{
    if constexpr (OFF32) {
        using gbyte = __attribute__((address_space(1))) char;
        return (gmem<T> *)((gbyte *)p + i * uint32_t(sizeof(T)));
    } else {
        return p + i;
    }
}

// node index -> axis indices (C order) with the host's division magic; the
// quotient left after the last D-1 axes is the first axis's index, since
// node < n[0] n[1] ... n[D-1]
template <typename T, int D>
__device__ inline void node_indices(const StageArgs<T> &a, uint32_t node, int *ii)
{
    uint32_t r = node;
#pragma unroll
    for (int d = D - 1; d >= 1; --d) {
        const uint32_t q = uint32_t((uint64_t(r) * a.nmul[d]) >> a.nshift[d]);
        ii[d] = int(r - q * a.n[d]);
        r = q;
    }
    ii[0] = int(r);
}

template <int SCH>
struct Halo;
template <>
struct Halo<kUpwind1> { static constexpr int w = 1; };
template <>
struct Halo<kEno2> { static constexpr int w = 2; };
template <>
struct Halo<kEno3> { static constexpr int w = 3; };
template <>
struct Halo<kWeno5> { static constexpr int w = 3; };

// Jiang-Peng WENO5 (Sec. 3.3; Osher-Fedkiw eqs. 3.28-3.39) on a window of
// five consecutive one-sided differences w0..w4 (increasing grid order).  The
// left-biased approximation of the node right of the window centre and the
// right-biased one of the node left of it share the window's smoothness
// indicators, eps and reciprocal weights:
//   SA = 13/12 e^2 + 1/4 ((a + 3c) - 4b)^2 on (w0,w1,w2), e = (a + c) - 2b
//   SB = 13/12 e^2 + 1/4 (a - c)^2          on (w1,w2,w3)
//   SC = 13/12 e^2 + 1/4 ((3a + c) - 4b)^2  on (w2,w3,w4)
//   eps = 1e-6 max w_k^2 + floor, r_X = 1/(S_X + eps)^2
// left-biased: gamma (0.1, 0.6, 0.3) on (rA, rB, rC); right-biased: on
// (rC, rB, rA) with the window reversed.
//
// FP64: every operation in the written order with correctly rounded
// divisions (div_rn_inrange below), built without contraction, so each rounding equals that of a
// plain FP64 evaluation of the same formulas (the scheme amplifies rounding
// differences by up to ~1e11 over a long horizon near the ridges of a game's
// value function, so FP64 results are only comparable at 1e-12 when the
// rounding is reproduced).  FP32: fused multiply-adds and hardware
// reciprocals (v_rcp_f32); the eps floor is 1e-18 because 1e-99 underflows.
template <typename T>
struct WenoR {
    T ra, rb, rc;
};

// FP64 division for the WENO weights: Newton-Raphson refinement of the
// hardware reciprocal with Markstein's final correction (hj_divseq.h), the
// correctly rounded quotient for every operand the weights can produce.
struct HwRcp {
    __device__ double operator()(double b) const { return __builtin_amdgcn_rcp(b); }
};

__device__ inline double div_rn_inrange(double a, double b) { return div_rn_seq(a, b, HwRcp()); }

__device__ inline double rcp_rn_inrange(double b) { return rcp_rn_seq(b, HwRcp()); }

template <typename T>
__device__ inline T wrecip(T x)
{
    if constexpr (sizeof(T) == 8)
        return rcp_rn_inrange(x);
    else
        return __builtin_amdgcn_rcpf(x);
}

// m: max_k |w_k|, the caller's (the two windows of a node share four of
// their five differences, so they share most of the maximum)
template <typename T>
__device__ inline WenoR<T> weno_window(T w0, T w1, T w2, T w3, T w4, T m)
{
    constexpr T c13_12 = T(13.0 / 12.0);
    T sa, sb, sc;
    if constexpr (sizeof(T) == 8) {
        // The products by 2, 4 and 1/4 are exact, so a fused multiply-add
        // that takes one of them rounds once, where the written product and
        // sum round once (the sum) too: the same value, one instruction
        // fewer.  For the 1/4 the product fa fa is rounded first, which
        // differs from rounding (fa/4) fa only below the normal range, and
        // there by less than the eps floor resolves in S + eps.
        const double ea = __builtin_fma(-2.0, w1, w0 + w2);
        const double eb = __builtin_fma(-2.0, w2, w1 + w3);
        const double ec = __builtin_fma(-2.0, w3, w2 + w4);
        const double fa = __builtin_fma(-4.0, w1, w0 + 3.0 * w2);
        const double fb = w1 - w3;
        const double fc = __builtin_fma(-4.0, w3, 3.0 * w2 + w4);
        sa = __builtin_fma(0.25, fa * fa, c13_12 * ea * ea);
        sb = __builtin_fma(0.25, fb * fb, c13_12 * eb * eb);
        sc = __builtin_fma(0.25, fc * fc, c13_12 * ec * ec);
    } else {
        // FP32: the weights depend on S + eps only through their ratios, so
        // S and eps are both taken 12/13 times their values (S as
        // e^2 + 3/13 f^2), one product fewer per indicator
        constexpr T c3_13 = T(3.0 / 13.0);
        const T ea = (w0 + w2) - T(2) * w1;
        const T eb = (w1 + w3) - T(2) * w2;
        const T ec = (w2 + w4) - T(2) * w3;
        const T fa = (w0 + T(3) * w2) - T(4) * w1;
        const T fb = w1 - w3;
        const T fc = (T(3) * w2 + w4) - T(4) * w3;
        sa = ea * ea + c3_13 * fa * fa;
        sb = eb * eb + c3_13 * fb * fb;
        sc = ec * ec + c3_13 * fc * fc;
    }
    // max_k w_k^2 as (max_k |w_k|)^2: rounding is monotone in |w|, so the
    // rounded square of the largest magnitude is the largest rounded square
    const T eps = sizeof(T) == 8 ? T(1e-6) * (m * m) + T(1e-99)
                                 : T(1e-6 * 12.0 / 13.0) * (m * m) + T(1e-18 * 12.0 / 13.0);
    WenoR<T> r;
    r.ra = wrecip((sa + eps) * (sa + eps));
    r.rb = wrecip((sb + eps) * (sb + eps));
    r.rc = wrecip((sc + eps) * (sc + eps));
    return r;
}

// weighted blend of the third-order candidates on v1..v5 with the reciprocal
// weights r1, r2, r3 of their substencils
template <typename T>
__device__ inline T weno_blend(T v1, T v2, T v3, T v4, T v5, T r1, T r2, T r3)
{
    if constexpr (sizeof(T) == 8) {
        constexpr T c1_3 = T(1.0 / 3.0);
        constexpr T c1_6 = T(1.0 / 6.0);
        constexpr T c5_6 = T(5.0 / 6.0);
        constexpr T c7_6 = T(7.0 / 6.0);
        constexpr T c11_6 = T(11.0 / 6.0);
        const T phi1 = v1 * c1_3 - v2 * c7_6 + v3 * c11_6;
        const T phi2 = -v2 * c1_6 + v3 * c5_6 + v4 * c1_3;
        const T phi3 = v3 * c1_3 + v4 * c5_6 - v5 * c1_6;
        const T a1 = T(0.1) * r1, a2 = T(0.6) * r2, a3 = T(0.3) * r3;
        return div_rn_inrange(a1 * phi1 + a2 * phi2 + a3 * phi3, a1 + a2 + a3);
    } else {
        // FP32: the candidates times 6 (integer coefficients, two fused
        // steps each; the caller's 1/dx takes the 1/6) and the ideal weights
        // 1/10, 6/10, 3/10 times 10 (the normalisation removes the factor)
        const T q1 = T(11) * v3 + (T(2) * v1 - T(7) * v2);
        const T q2 = T(5) * v3 + (T(2) * v4 - v2);
        const T q3 = T(5) * v4 + (T(2) * v3 - v5);
        const T a1 = r1, a2 = T(6) * r2, a3 = T(3) * r3;
        return (a1 * q1 + a2 * q2 + a3 * q3) * wrecip(a1 + a2 + a3);
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
template <typename T, bool O>
__device__ inline T line_value(const Arr<T, O> &v, uint32_t node, int i, int j, int n,
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

// The 2W+1 stencil values of the grid line through `node` around its axis
// index i, ghosts included, without branches: every load uses a wrapped
// (periodic) or clamped index, and the values beyond a bounded end are then
// replaced by their linear extrapolations (the same formula as line_value).
// Every lane of a wavefront runs the same instructions whether or not its node
// is near an end; this suits the fastest axis, along which most wavefronts
// hold some node near a line's end.
template <typename T, int W, bool O>
__device__ inline void line_stencil_select(const Arr<T, O> &v, uint32_t node, int i, int n,
                                           uint32_t stride, bool periodic, T *s)
{
    // 0 <= i < n, so an index left of the node can leave the line only at
    // its first end and one right of it only at its last: one test each
    const uint32_t base = node - uint32_t(i) * stride;
    if (periodic) {
#pragma unroll
        for (int k = 0; k <= 2 * W; ++k) {
            const int j = i - W + k;
            const int jw = k < W ? (j < 0 ? j + n : j) : (k > W ? (j >= n ? j - n : j) : i);
            s[k] = v[base + uint32_t(jw) * stride];
        }
        return;
    }
#pragma unroll
    for (int k = 0; k <= 2 * W; ++k) {
        const int j = i - W + k;
        const int jc = k < W ? (j < 0 ? 0 : j) : (k > W ? (j >= n ? n - 1 : j) : i);
        s[k] = v[base + uint32_t(jc) * stride];
    }
    const T e0 = v[base], e1 = v[base + stride];
    const T f0 = v[base + uint32_t(n - 1) * stride], f1 = v[base + uint32_t(n - 2) * stride];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int j = i - W + k;
        const T g = e0 + T(-j) * (e0 - e1);
        s[k] = j < 0 ? g : s[k];
    }
#pragma unroll
    for (int k = W + 1; k <= 2 * W; ++k) {
        const int j = i - W + k;
        const T g = f0 + T(j - (n - 1)) * (f0 - f1);
        s[k] = j >= n ? g : s[k];
    }
}

// The same 2W+1 values along the fastest axis (stride 1) from one load per
// node: the lanes of a wavefront hold consecutive nodes, so the neighbours at
// offsets -W..W come from the lanes beside it (cross-lane shuffles through
// the LDS crossbar, which spare the vector-memory address and data units
// that the stencil loads otherwise keep busy).  A lane loads a neighbour
// itself where the lane holding it is outside the wavefront or inactive, and
// on a periodic axis where the neighbour wraps round the line; on a bounded
// axis the ghosts are the linear extrapolations of line_value, from the
// line's two end values, which lie in the node's own stencil whenever a
// ghost is needed (every axis has at least 2W+1 nodes).
template <typename T, int W, bool O>
__device__ inline void line_stencil_shuffle(const Arr<T, O> &v, uint32_t node, int i, int n,
                                            bool periodic, T *s)
{
    const uint64_t act = __ballot(1);
    const int lane = int(__lane_id());
    const uint32_t base = node - uint32_t(i);
    const T c = v[node];
#pragma unroll
    for (int k = 0; k <= 2 * W; ++k) {
        const int o = k - W;
        if (o == 0) {
            s[k] = c;
            continue;
        }
        T x = o < 0 ? T(__shfl_up(c, unsigned(-o))) : T(__shfl_down(c, unsigned(o)));
        const int src = lane + o;
        const bool have = src >= 0 && src < 64 && ((act >> src) & 1u);
        const int j = i + o;
        const bool inside = j >= 0 && j < n;
        if ((inside && !have) || (periodic && !inside)) {
            const int jw = j < 0 ? j + n : (j >= n ? j - n : j);
            x = v[base + uint32_t(jw)];
        }
        s[k] = x;
    }
    if (!periodic) {
        // line positions 0, 1 and n-1, n-2: stencil entries W - i (+1) near
        // the first end, W + n-1-i (-1) near the last
        T e0 = s[W], e1 = s[W], f0 = s[W], f1 = s[W];
#pragma unroll
        for (int m = 0; m < W; ++m) {
            e0 = i == m ? s[W - m] : e0;
            e1 = i == m ? s[W - m + 1] : e1;
            f0 = i == n - 1 - m ? s[W + m] : f0;
            f1 = i == n - 1 - m ? s[W + m - 1] : f1;
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int j = i - W + k;
            const T g = e0 + T(-j) * (e0 - e1);
            s[k] = j < 0 ? g : s[k];
        }
#pragma unroll
        for (int k = W + 1; k <= 2 * W; ++k) {
            const int j = i - W + k;
            const T g = f0 + T(j - (n - 1)) * (f0 - f1);
            s[k] = j >= n ? g : s[k];
        }
    }
}

// Whether the fastest axis is gathered by cross-lane shuffles: the FP64 ENO2
// kernels, whose time is set by the vector-memory units (counters: address
// and data units busy about 80 % of a rockets 100^3 stage, 18 cycles per
// 64-lane FP64 load) and which have VALU issue to spare (47 %); measured
// 13.5 -> 11.9 us per rockets stage.  FP32 loads cost those units half as
// much, and the shuffles, selects and edge loads made the FP32 kernel 10 %
// slower; the WENO5 kernels are bound by VALU issue.
template <typename T, int SCH>
struct ShuffleFastest {
    static constexpr bool value = SCH == kEno2 && sizeof(T) == 8;
};

// p- and p+ along one axis at one node (Sec. 3.1-3.3).
// First divided differences use the reciprocal cell size 1/dx, second ones
// 1/(2 dx), third ones 1/(3 dx) (all computed once on the host in FP64).
// fastest: the axis is the last one (the stencil is gathered without
// branches); on the other axes only the few wavefronts near an end take the
// ghost path.
template <typename T, int SCH, bool O>
__device__ inline void axis_derivs(const Arr<T, O> &v, uint32_t node, int i, int n,
                                   uint32_t stride, bool periodic, T dx, T inv_dx, T inv_2dx,
                                   T inv_3dx, T &pm, T &pp, T &center, bool fastest = false)
{
    constexpr int W = Halo<SCH>::w;
    T s[2 * W + 1];
    const bool interior = i >= W && i < n - W;
    if (fastest) {
        // the last axis is the contiguous one (C order): stride 1, which
        // spares the index arithmetic its integer multiplies
        if constexpr (ShuffleFastest<T, SCH>::value)
            line_stencil_shuffle<T, W>(v, node, i, n, periodic, s);
        else
            line_stencil_select<T, W>(v, node, i, n, 1u, periodic, s);
    } else if (interior) {
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
    } else if constexpr (SCH == kEno3) {
        // HJ ENO3 (Osher-Fedkiw Sec. 3.3): d1[j] = D1 at i-5/2+j, d2[j] = D2
        // at i-2+j, d3[j] = D3 at i-3/2+j; p = (Q1' + Q2') + Q3' with
        // Q2' = +-c dx and Q3' = c* (2 or -1) dx^2 by where the stencil grew.
        T d1[6], d2[5], d3[4];
#pragma unroll
        for (int k = 0; k < 6; ++k) d1[k] = (s[k + 1] - s[k]) * inv_dx;
#pragma unroll
        for (int k = 0; k < 5; ++k) d2[k] = (d1[k + 1] - d1[k]) * inv_2dx;
#pragma unroll
        for (int k = 0; k < 4; ++k) d3[k] = (d2[k + 1] - d2[k]) * inv_3dx;
        const T dxx = dx * dx;
        T c, cs, f;
        if (fabs(d2[1]) <= fabs(d2[2])) {
            c = d2[1];
            cs = eno_pick(d3[0], d3[1]);
            f = T(2);
        } else {
            c = d2[2];
            cs = eno_pick(d3[1], d3[2]);
            f = T(-1);
        }
        pm = (d1[2] + c * dx) + cs * (f * dxx);
        if (fabs(d2[2]) <= fabs(d2[3])) {
            c = d2[2];
            cs = eno_pick(d3[1], d3[2]);
            f = T(-1);
        } else {
            c = d2[3];
            cs = eno_pick(d3[2], d3[3]);
            f = T(2);
        }
        pp = (d1[3] - c * dx) + cs * (f * dxx);
    } else {
        // FP64: divided differences, as the formulas are written.  FP32: the
        // undivided ones, scaled by 1/dx at the end (WENO5 is homogeneous of
        // degree one in the differences; eps scales with them, its floor
        // aside), which saves four multiplies per axis.
        constexpr bool undivided = sizeof(T) == 4;
        T d1[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            d1[k] = undivided ? s[k + 1] - s[k] : (s[k + 1] - s[k]) * inv_dx;
        // p-: left-biased on the window d1[0..4]; p+: right-biased on d1[1..5]
        // the largest |difference| of each window (max is exact in any order)
        const T mc = fmax(fmax(fabs(d1[1]), fabs(d1[2])), fmax(fabs(d1[3]), fabs(d1[4])));
        const WenoR<T> rl = weno_window(d1[0], d1[1], d1[2], d1[3], d1[4], fmax(fabs(d1[0]), mc));
        pm = weno_blend(d1[0], d1[1], d1[2], d1[3], d1[4], rl.ra, rl.rb, rl.rc);
        const WenoR<T> rr = weno_window(d1[1], d1[2], d1[3], d1[4], d1[5], fmax(mc, fabs(d1[5])));
        pp = weno_blend(d1[5], d1[4], d1[3], d1[2], d1[1], rr.rc, rr.rb, rr.ra);
        if (undivided) {  // 1/dx, and the 1/6 of the FP32 candidates
            const T k = inv_dx * T(1.0 / 6.0);
            pm *= k;
            pp *= k;
        }
    }
}

// H(x, p) of the compiled dynamics (sign convention V_t + H = 0).  The
// coordinate tables (x, cos x, sin x per node of each axis) are read with
// 32-bit byte offsets: they hold 3 entries per grid line position.
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
        const T x2 = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[1] + ii[1]];
        return -p[0] * x2 + a.prm[0] * fabs(p[1]);
    } else if constexpr (DYN == kRelDubins) {
        const T ve = a.prm[0], vp = a.prm[1], we = a.prm[2], wp = a.prm[3];
        const T x = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[0] + ii[0]];
        const T y = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[1] + ii[1]];
        const T c = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[2] + a.n[2] + ii[2]];
        const T s = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        return -p[0] * (-ve + vp * c) - p[1] * (vp * s) - we * fabs(p[0] * y - p[1] * x - p[2]) +
               wp * fabs(p[2]);
    } else if constexpr (DYN == kRockets) {
        // (x, z, th): p.f = p1 a cos th + p2 (a sin th + a - g) + ue (p1 x - p3)
        // + up (p2 x + p3), evader ue maximising, pursuer up minimising
        const T am = a.prm[0], grav = a.prm[1], um = a.prm[2];
        const T x = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[0] + ii[0]];
        const T c = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[2] + a.n[2] + ii[2]];
        const T s = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        const T drift1 = am * c;
        const T drift2 = am * s + am - grav;
        return -p[0] * drift1 - p[1] * drift2 - um * fabs(p[0] * x - p[2]) +
               um * fabs(p[1] * x + p[2]);
    } else {
        const T wm = a.prm[0], am = a.prm[1];
        const T c = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[2] + a.n[2] + ii[2]];
        const T s = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[2] + 2 * a.n[2] + ii[2]];
        const T v = Arr<T, true>{global_ptr(a.tab)}[a.tab_off[3] + ii[3]];
        return -p[0] * (v * c) - p[1] * (v * s) + wm * fabs(p[2]) + am * fabs(p[3]);
    }
}

// Costate-box Lax-Friedrichs coefficients (the dissipation routine of Sec. 4
// takes the one-sided derivatives): max over p in the box lo..hi and over
// the controls of |dH/dp_d| at a node.  A switching function s = a.p has the
// interval sum_j [min(a_j lo_j, a_j hi_j), max(..)] (axes in order) and may
// take the sign +1 where its upper end is >= 0, -1 where its lower end is
// <= 0.  Dynamics whose |dH/dp_d| does not depend on p give their control
// bound.
template <typename T>
__device__ inline void lin_interval(const T *a, const T *lo, const T *hi, T *smin, T *smax)
{
    T l = T(0), h = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T u = a[j] * lo[j], w = a[j] * hi[j];
        l = l + (u < w ? u : w);
        h = h + (u < w ? w : u);
    }
    *smin = l;
    *smax = h;
}

// max over the signs the interval allows of |base + k sigma|
template <typename T>
__device__ inline T sign_max(T base, T k, T smin, T smax)
{
    T m = T(0);
    if (smax >= T(0)) {
        const T v = fabs(base + k);
        if (v > m) m = v;
    }
    if (smin <= T(0)) {
        const T v = fabs(base - k);
        if (v > m) m = v;
    }
    return m;
}

template <typename T, int D, int DYN>
__device__ inline T box_bound(const StageArgs<T> &a, const int *ii, int d, const T *lo,
                              const T *hi)
{
    const Arr<T, true> tab{global_ptr(a.tab)};
    if constexpr (DYN == kBall) {
        const T big = fabs(lo[d]) > fabs(hi[d]) ? fabs(lo[d]) : fabs(hi[d]);
        T rest = T(0);
        bool all_zero = big == T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j == d) continue;
            const T m = (lo[j] <= T(0) && hi[j] >= T(0))
                            ? T(0)
                            : (fabs(lo[j]) < fabs(hi[j]) ? fabs(lo[j]) : fabs(hi[j]));
            if (m != T(0)) all_zero = false;
            rest = rest + m * m;
        }
        if (big == T(0)) return all_zero ? fabs(a.prm[0]) : T(0);
        return fabs(a.prm[0]) * (big / sqrt(big * big + rest));
    } else if constexpr (DYN == kRelDubins) {
        const T ve = a.prm[0], vp = a.prm[1], we = a.prm[2], wp = a.prm[3];
        const T x = tab[a.tab_off[0] + ii[0]];
        const T y = tab[a.tab_off[1] + ii[1]];
        const T coef[3] = {y, -x, T(-1)};
        T smin, smax;
        lin_interval(coef, lo, hi, &smin, &smax);
        if (d == 0) {
            const T c = tab[a.tab_off[2] + a.n[2] + ii[2]];
            return sign_max(ve - vp * c, -we * y, smin, smax);
        }
        if (d == 1) {
            const T s = tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
            return sign_max(-(vp * s), we * x, smin, smax);
        }
        T m = T(0);
        if (smax >= T(0)) {
            const T v = sign_max(we, wp, lo[2], hi[2]);
            if (v > m) m = v;
        }
        if (smin <= T(0)) {
            const T v = sign_max(-we, wp, lo[2], hi[2]);
            if (v > m) m = v;
        }
        return m;
    } else if constexpr (DYN == kRockets) {
        const T am = a.prm[0], grav = a.prm[1], um = a.prm[2];
        const T x = tab[a.tab_off[0] + ii[0]];
        const T c1[3] = {x, T(0), T(-1)}, c2[3] = {T(0), x, T(1)};
        T l1, h1, l2, h2;
        lin_interval(c1, lo, hi, &l1, &h1);
        lin_interval(c2, lo, hi, &l2, &h2);
        if (d == 0) {
            const T c = tab[a.tab_off[2] + a.n[2] + ii[2]];
            return sign_max(-(am * c), -um * x, l1, h1);
        }
        if (d == 1) {
            const T s = tab[a.tab_off[2] + 2 * a.n[2] + ii[2]];
            return sign_max(-(am * s + am - grav), um * x, l2, h2);
        }
        T m = T(0);
        if (h1 >= T(0)) {
            const T v = sign_max(um, um, l2, h2);
            if (v > m) m = v;
        }
        if (l1 <= T(0)) {
            const T v = sign_max(-um, um, l2, h2);
            if (v > m) m = v;
        }
        return m;
    } else if constexpr (DYN == kTranslation) {
        return fabs(a.prm[d]);
    } else if constexpr (DYN == kDoubleIntegrator) {
        if (d == 0) return fabs(tab[a.tab_off[1] + ii[1]]);
        return a.prm[0];
    } else {
        const T v = tab[a.tab_off[3] + ii[3]];
        if (d == 0) return fabs(v * tab[a.tab_off[2] + a.n[2] + ii[2]]);
        if (d == 1) return fabs(v * tab[a.tab_off[2] + 2 * a.n[2] + ii[2]]);
        if (d == 2) return a.prm[0];
        return a.prm[1];
    }
}

// One node of one stage: derivatives along every axis, Lax-Friedrichs
// right-hand side, RK combination and tube minimum; writes a.out[node].
template <typename T, int D, int SCH, int DYN, bool OFF32>
__device__ inline void stage_node(const StageArgs<T> &a, uint32_t node)
{
    int ii[D];
    node_indices<T, D>(a, node, ii);
    T pm[D], pp[D], center = T(0);
    // the fastest axis first where it is gathered by shuffles, so that its
    // one load is the first in flight (measured 7 % faster than last)
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const int d = ShuffleFastest<T, SCH>::value ? (q + D - 1) % D : q;
        axis_derivs<T, SCH>(Arr<T, OFF32>{global_ptr(a.vs)}, node, ii[d], int(a.n[d]), a.stride[d],
                            (a.periodic >> d) & 1u, a.dx[d], a.inv_dx[d], a.inv_2dx[d],
                            a.inv_3dx[d], pm[d], pp[d], center, d == D - 1);
    }
    // Twice p-bar and twice the dissipation: H is positively homogeneous of
    // degree one in p (sums, products by coefficients, absolute values, the
    // square root of a sum of squares), and a factor 2 commutes with every
    // rounding, so H(pp + pm) - sum alpha (pp - pm) is exactly twice the
    // Lax-Friedrichs Hhat and one product by -1/2 below replaces the 2 D
    // halvings (outside the normal range aside).
    T pbar[D];
    T diss = T(0);
    if (a.diss == kLF) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            pbar[d] = pp[d] + pm[d];
            diss += a.alpha[d] * (pp[d] - pm[d]);
        }
    } else {
        T lo[D], hi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (a.diss == kGLF) {
                lo[d] = global_ptr(a.box)[2 * d];
                hi[d] = global_ptr(a.box)[2 * d + 1];
            } else {
                lo[d] = pm[d] < pp[d] ? pm[d] : pp[d];
                hi[d] = pm[d] < pp[d] ? pp[d] : pm[d];
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            pbar[d] = pp[d] + pm[d];
            diss += box_bound<T, D, DYN>(a, ii, d, lo, hi) * (pp[d] - pm[d]);
        }
    }
    T l = (hamiltonian<T, D, DYN>(a, ii, pbar) - diss) * T(-0.5);
    if (a.vi && l > T(0)) l = T(0);

    T val;
    if (a.combine == kRhs) {
        val = l;
    } else {
        const T v2 = center + a.dt * l;
        if (a.combine == kEuler) {
            val = v2;
        } else {
            // the blends divide by 2, 4 (RK2, RK3 stage 2: the same as
            // multiplying by 1/2, 1/4, exactly) or 3
            const T x = a.wb * Arr<T, OFF32>{global_ptr(a.vb)}[node] + a.w2 * v2;
            val = a.den == T(3) ? x / T(3) : x * (a.den == T(4) ? T(0.25) : T(0.5));
        }
    }
    if (a.tube) val = fmin(val, Arr<T, OFF32>{global_ptr(a.v0)}[node]);
    // a streaming store: nothing in this launch reads the output again (the
    // next stage is another launch, on any XCD); measured 1-3 % faster
    __builtin_nontemporal_store(val, elem_at<OFF32>(global_ptr(a.out), node));
}

// Occupancy floor of the per-node kernel: the 3-D FP64 WENO5 kernels fit 72
// VGPRs without spilling, which gives 7 waves per SIMD (left to itself the
// compiler takes 74 and 6 waves); elsewhere no floor (a floor of 6 makes the
// 3-D ENO3 and 4-D FP64 kernels spill, and 8 waves spill the 3-D FP64 WENO5
// kernels, slower).
template <typename T, int D, int SCH>
struct StageWaves {
    static constexpr int value = 1;
};
template <>
struct StageWaves<double, 3, kWeno5> {
    static constexpr int value = 7;
};

// Tile of workgroup b out of nb.  Workgroups are dispatched to the chip's 8
// XCDs round-robin (b on XCD b % 8), and each XCD has its own L2: XCD x takes
// the x-th contiguous eighth of the tiles (the first nb % 8 eighths one tile
// longer), so the stencil neighbours along the slow axes of the nodes an XCD
// updates are mostly in tiles that the same XCD updates.  A bijection of
// [0, nb) whatever the dispatch order, so correctness does not depend on it.
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u, i = b >> 3;
    return (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + i;
}

template <typename T, int D, int SCH, int DYN, bool OFF32>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(StageWaves<T, D, SCH>::value))) void stage_kernel(
    const StageArgs<T> a)
{
    const uint32_t node = xcd_tile(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
    if (node >= a.total) return;
    stage_node<T, D, SCH, DYN, OFF32>(a, node);
}

// Whether every array of `total` elements of T is under 4 GiB (32-bit byte
// offsets).
template <typename T>
inline bool fits_off32(uint64_t total)
{
    return total * sizeof(T) <= 0xffffffffull;
}

}  // namespace hj
