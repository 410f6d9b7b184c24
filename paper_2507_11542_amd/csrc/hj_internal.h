// Internal interface between the libhj host runtime (hj_api.cpp) and the
// gfx950 kernels (hj_stage.hip, hj_alpha.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hj_divmagic.h"

namespace hj {

constexpr int kMaxDim = 4;

enum Space { kUpwind1 = 1, kEno2 = 2, kEno3 = 3, kWeno5 = 5 };
enum Dyn {
    kTranslation = 0,
    kBall = 1,
    kDoubleIntegrator = 2,
    kRelDubins = 3,
    kDubins4D = 4,
    kRockets = 5
};

// Lax-Friedrichs coefficients: the per-solve control-set bound alpha (kLF), or
// per node the max of |dH/dp_d| over a costate box: the node's own
// [min(p-, p+), max(p-, p+)] (kLLF) or the grid-wide box of the stage input
// (kGLF, reduced on the device before the stage).
enum Diss { kLF = 0, kLLF = 1, kGLF = 2 };

// How a stage kernel combines the right-hand side L(Vs) with its inputs:
//   kRhs      out = L(Vs)
//   kEuler    out = Vs + dt L(Vs)
//   kBlend    out = (wb Vb + w2 (Vs + dt L(Vs))) / den, den in {2, 3, 4}
enum Combine { kRhs = 0, kEuler = 1, kBlend = 2 };

// Everything one stage launch needs, by value (kernel argument).
template <typename T>
struct StageArgs {
    const T *vs;      // stage input, read with the stencil
    const T *vb;      // RK base, read at the node only (kBlend)
    const T *v0;      // tube target, read at the node only (tube != 0)
    T *out;           // may alias vb (each node reads vb then writes out)
    const T *tab;     // per-axis [x(n) | cos x(n) | sin x(n)] blocks
    uint32_t n[kMaxDim];
    uint32_t stride[kMaxDim];
    uint32_t tab_off[kMaxDim];
    uint32_t nmul[kMaxDim];    // floor(x / n[d]) = (x * nmul[d]) >> nshift[d]
    uint32_t nshift[kMaxDim];
    uint32_t total;
    uint32_t periodic;  // bit d: axis d periodic
    uint32_t addr64;    // host side: launch the 64-bit-addressing form whatever the size
    T dx[kMaxDim];
    T inv_dx[kMaxDim];   // 1/dx (FP64 on the host, then rounded to T)
    T inv_2dx[kMaxDim];  // 1/(2 dx)
    T inv_3dx[kMaxDim];  // 1/(3 dx)
    T alpha[kMaxDim];
    T prm[8];
    T dt, wb, w2, den;
    int combine;
    int tube;         // out = min(out, v0[node])
    int vi;           // restricted update: L = min(L, 0) (variational-inequality tube)
    int diss;         // Diss
    const T *box;     // kGLF: [lo_0, hi_0, lo_1, hi_1, ...] on the device
};

struct AlphaArgs {
    const double *tab;
    uint32_t n[kMaxDim];
    uint32_t tab_off[kMaxDim];
    uint32_t total;
    double prm[8];
};

// Launchers (defined in the .hip files).  Return hipSuccess or the launch error.
hipError_t launch_stage_f64(int ndim, int space, int dyn, const StageArgs<double> &a,
                            hipStream_t s);
hipError_t launch_stage_f32(int ndim, int space, int dyn, const StageArgs<float> &a,
                            hipStream_t s);
// Two-pass max reduction of the per-node bounds |dH/dp_d| into alpha[0..ndim).
// partial must hold alpha_blocks(total) * ndim doubles.
uint32_t alpha_blocks(uint32_t total);
hipError_t launch_alpha(int ndim, int dyn, const AlphaArgs &a, double *partial, double *alpha,
                        hipStream_t s);

hipError_t launch_round_to_f32(const double *src, float *dst, uint32_t n, hipStream_t s);

// Grid-wide costate box of a.vs (kGLF): box[2d], box[2d+1] = min, max over all
// nodes of p- and p+ along axis d.  partial holds box_blocks(total) * 2 * ndim
// values.
uint32_t box_partial_values(uint32_t total, int ndim);
hipError_t launch_box_f64(int ndim, int space, const StageArgs<double> &a, double *partial,
                          double *box, hipStream_t s);
hipError_t launch_box_f32(int ndim, int space, const StageArgs<float> &a, float *partial,
                          float *box, hipStream_t s);

// Implicit-surface initial values (the shapes of include/hj.h, evaluated in
// FP64 and stored as double or float).
constexpr int kMaxShapes = 16;

struct ShapeDesc {
    int kind;
    int op;
    uint32_t mask;  // axes taking part (already resolved: never 0)
    uint32_t pad;
    double center[kMaxDim];
    double size[kMaxDim];
    double radius;
};

struct ShapeArgs {
    const double *tab;  // per-axis [x | cos x | sin x] blocks
    void *out;
    uint32_t n[kMaxDim];
    uint32_t tab_off[kMaxDim];
    uint32_t total;
    int nd;
    int nshapes;
    int fp32;  // store as float
    ShapeDesc s[kMaxShapes];
};

hipError_t launch_shapes(const ShapeArgs &a, hipStream_t s);
// flag <- 1 if any of the n values (double if fp64, else float) is NaN or
// infinite, else 0 (flag is one device int)
hipError_t launch_scan_nonfinite(const void *v, int fp64, uint32_t n, int *flag, hipStream_t s);
hipError_t launch_finalize_f64(const float *v32, const double *v0, double *out, uint32_t n,
                               double band, int tube, hipStream_t s);

}  // namespace hj
