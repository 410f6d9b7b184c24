// Implicit-surface initial value functions (Sec. 2.2, Fig. 4) built on the
// device: one thread per node evaluates every shape at the node's
// coordinates and combines them left to right (union min, intersection max,
// difference max(v, -s)).  FP64 arithmetic in source order, built without
// contraction; the value is stored as double or rounded once to float.
//   sphere, cylinder  sqrt(sum over the shape's axes of (x_d - c_d)^2) - r
//   box               |max(q, 0)|_2 + min(max_d q_d, 0), q_d = |x_d - c_d| - h_d
//   ellipsoid         sum over the shape's axes of w_d (x_d - c_d)^2 - r
#include "hj_internal.h"

#include "../../include/hj.h"

namespace hj {

namespace {

__device__ inline double shape_value(const ShapeDesc &s, int nd, const double *x)
{
    if (s.kind == HJ_SHAPE_BOX) {
        double outside = 0.0, inside = -INFINITY;
        for (int d = 0; d < nd; ++d) {
            if (!((s.mask >> d) & 1u)) continue;
            const double q = fabs(x[d] - s.center[d]) - s.size[d];
            if (q > 0.0) outside = outside + q * q;
            if (q > inside) inside = q;
        }
        return sqrt(outside) + (inside < 0.0 ? inside : 0.0);
    }
    double acc = 0.0;
    for (int d = 0; d < nd; ++d) {
        if (!((s.mask >> d) & 1u)) continue;
        const double t = x[d] - s.center[d];
        if (s.kind == HJ_SHAPE_ELLIPSOID)
            acc = acc + s.size[d] * (t * t);
        else
            acc = acc + t * t;
    }
    if (s.kind == HJ_SHAPE_ELLIPSOID) return acc - s.radius;
    return sqrt(acc) - s.radius;
}

__global__ __launch_bounds__(256) void shapes_kernel(const ShapeArgs a)
{
    const uint32_t node = blockIdx.x * 256u + threadIdx.x;
    if (node >= a.total) return;
    double x[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
    uint32_t r = node;
    for (int d = a.nd - 1; d >= 0; --d) {
        x[d] = a.tab[a.tab_off[d] + r % a.n[d]];
        r /= a.n[d];
    }
    double v = 0.0;
    for (int k = 0; k < a.nshapes; ++k) {
        const double sv = shape_value(a.s[k], a.nd, x);
        if (k == 0)
            v = sv;
        else if (a.s[k].op == HJ_OP_UNION)
            v = sv < v ? sv : v;
        else if (a.s[k].op == HJ_OP_INTERSECT)
            v = sv > v ? sv : v;
        else
            v = -sv > v ? -sv : v;
    }
    if (a.fp32)
        ((float *)a.out)[node] = float(v);
    else
        ((double *)a.out)[node] = v;
}

}  // namespace

hipError_t launch_shapes(const ShapeArgs &a, hipStream_t s)
{
    const uint32_t blocks = (a.total + 255u) / 256u;
    hipLaunchKernelGGL(shapes_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hj
