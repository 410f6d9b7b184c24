// Batched solve: many independent grids (instances) advanced together, one
// fused launch per RK-stage round covering every instance still running.
//
// Round r is stage r % order of RK step r / order.  The instances are sorted
// by step count (descending), so the instances still running in round r are
// a prefix of that order; the round's work is the concatenation of their
// tiles (each instance's own tile size: the configured maximum, shrunk so a
// small instance still spreads over enough workgroups), and tile k of every
// round is the same (instance, tile) pair, listed once in a tile map.  The round kernel's workgroups stride over
// those tiles; the kernel boundary between rounds is the only barrier, so no
// workgroup ever waits on another.  All rounds are launched back to back (and
// captured once in a hipGraph by the host), each kernel reading the round
// tables from device memory.
//
// Time: each instance keeps t in FP64 on the device, double-buffered by step
// parity; the tiles of a step read t_n and use h = min(dt, tf - t_n); tile 0
// of the step's last stage stores t_n + h into the other slot.
#pragma once

#include "hj_launch_impl.h"

namespace hj {

template <typename T>
struct BatchInst {
    StageArgs<T> geo;  // geometry, tables, alpha, dynamics parameters
    T *v;              // instance state V (caller's V_out), updated in place
    T *a;              // stage buffer A
    T *b;              // stage buffer B
    const T *v0;       // V0 (tube target)
    double dt, t0, tf; // CFL step and horizon (FP64)
    uint32_t tiles;    // tiles per round
    uint32_t steps;    // RK steps
    uint32_t tile_nodes;  // nodes per tile of this instance
    int tube;          // min with v0 after every step
    int vi;            // restricted update in every stage
};

struct TileRef {
    uint32_t inst;     // instance id (original order)
    uint32_t tile;     // tile index within the instance
    uint32_t rounds;   // the instance runs in rounds [0, rounds); 0 past the map's tiles
    uint32_t pad;
};
static_assert(sizeof(TileRef) == 16, "the round kernel reads a map entry as 4 words");

struct BatchCtl {
    double t[2];       // t at the start of even / odd steps
};

struct BatchGlobal {
    uint32_t items;      // total tiles over all rounds
    uint32_t rounds;
    uint32_t ninst;
    uint32_t tile_nodes;
    uint32_t order;      // RK order (2 or 3)
    uint32_t pad[3];
};

template <typename T>
struct BatchPtrs {
    const BatchInst<T> *inst;  // [ninst], original order
    BatchCtl *ctl;             // [ninst]
    const TileRef *tile_map;   // [map_cap] tiles of the instances by step count,
                               // descending (round r runs a prefix of it), then
                               // entries with rounds = 0
    const uint32_t *round_off; // [rounds + 1] first work item of each round
    const BatchGlobal *gl;
    uint32_t map_cap;          // entries allocated for tile_map (>= 1)
};

template <typename T>
__global__ __launch_bounds__(256) void batch_init(BatchPtrs<T> p)
{
    const uint32_t n = p.gl->ninst;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        p.ctl[i].t[0] = p.inst[i].t0;
        p.ctl[i].t[1] = p.inst[i].t0;
    }
}

// Arguments of stage `stage` of step `step` (round step * order + stage) of
// instance `inst`, and the step size h of that step (from the instance's
// device time t_n).
template <typename T>
__device__ inline StageArgs<T> batch_stage_args(const BatchPtrs<T> &p, uint32_t inst,
                                                uint32_t order, uint32_t stage, uint32_t step,
                                                double *h_out, double *tn_out)
{
    const BatchInst<T> &in = p.inst[inst];
    const double t_n = p.ctl[inst].t[step & 1u];
    const double rem = in.tf - t_n;
    const double h = in.dt < rem ? in.dt : rem;
    StageArgs<T> a = in.geo;
    // every field read before the stage picks among them (selects, not
    // branches, so that the instance's fields are one round of loads)
    T *const v = in.v, *const ba = in.a, *const bb = in.b;
    const int tube = in.tube;
    // stage 0: V -> A (Euler); RK3 stage 1: (3 V + (A + h L(A))) / 4 -> B;
    // last stage: (V + 2 (B + h L(B))) / 3 -> V (RK3) or (V + (A + h L(A))) / 2
    // -> V (RK2), with the tube minimum
    const bool first = stage == 0;
    const bool mid = stage == 1 && order == 3;
    const bool last = !first && !mid;
    a.dt = T(h);
    a.v0 = in.v0;
    a.vi = in.vi;
    a.vs = first ? v : (mid || order == 2 ? ba : bb);
    a.vb = first ? nullptr : v;
    a.out = first ? ba : (mid ? bb : v);
    a.combine = first ? kEuler : kBlend;
    a.wb = mid ? T(3) : T(1);
    a.w2 = (last && order == 3) ? T(2) : T(1);
    a.den = mid ? T(4) : (order == 2 ? T(2) : T(3));
    a.tube = last ? tube : 0;
    *h_out = h;
    *tn_out = t_n;
    return a;
}

// tile `local` of a round: its instance and tile (wave-uniform)
template <typename T>
__device__ inline void batch_item(const BatchPtrs<T> &p, uint32_t local, uint32_t *inst,
                                  uint32_t *tile)
{
    const TileRef t = p.tile_map[local];
    *inst = __builtin_amdgcn_readfirstlane(t.inst);
    *tile = __builtin_amdgcn_readfirstlane(t.tile);
}

// Round r of the batch.  Strided form: the launch's workgroups stride over
// the round's tiles, each tile a loop over its nodes.  Flat form (FLAT): one
// workgroup per 256-node tile and one node per thread, no loop at all, so the
// kernel keeps the register footprint of the plain stage kernel (the loops of
// the strided form keep about twice the VGPRs live, halving occupancy);
// workgroups beyond the round's tiles return at once.
// Round r is stage `stage` (r % order) of RK step `step` (r / order), both
// passed in by the host with r, so the kernel forms no quotient.
template <typename T, int D, int SCH, int DYN, bool FLAT, bool OFF32>
__global__ __launch_bounds__(256) void batch_round(BatchPtrs<T> p, uint32_t r, uint32_t order,
                                                   uint32_t stage, uint32_t step)
{
    // r < the batch's round count: rounds are launched for exactly the batch's
    // rounds (a replayed graph was captured for the same round count)
    const uint32_t b = blockIdx.x;
    if (FLAT) {
        // Workgroup b takes map entry b, whose instance runs in this round
        // when r < rounds (the round's tiles are a prefix of the map): one
        // scalar load (constant address space: the map does not change
        // during a launch) before the instance's own tables, instead of the
        // round bounds and then the entry.
        // (the entry is one 16-byte load, made before any branch, so that
        // the kernel arguments and then the entry are each one round of loads)
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const uint32_t cap = p.map_cap;
        const u32x4 e = *(const __attribute__((address_space(4))) u32x4 *)(p.tile_map +
                                                                          (b < cap ? b : cap - 1u));
        const uint32_t inst = e.x, tile = e.y;
        if (b >= cap || r >= e.z) return;
        double h, t_n;
        const StageArgs<T> a = batch_stage_args(p, inst, order, stage, step, &h, &t_n);
        const uint32_t node = tile * 256u + threadIdx.x;
        if (node < a.total) stage_node<T, D, SCH, DYN, OFF32>(a, node);
        // the other slot: read by no tile of this step
        if (stage == order - 1 && tile == 0 && threadIdx.x == 0)
            p.ctl[inst].t[(step + 1) & 1u] = t_n + h;
        return;
    }
    const uint32_t begin = p.round_off[r], end = p.round_off[r + 1];
    for (uint32_t k = begin + blockIdx.x; k < end; k += gridDim.x) {
        uint32_t inst, tile;
        batch_item(p, k - begin, &inst, &tile);
        double h, t_n;
        const StageArgs<T> a = batch_stage_args(p, inst, order, stage, step, &h, &t_n);
        const uint32_t tn = p.inst[inst].tile_nodes;
        const uint32_t first = tile * tn;
        const uint32_t last = first + tn < a.total ? first + tn : a.total;
        for (uint32_t node = first + threadIdx.x; node < last; node += 256)
            stage_node<T, D, SCH, DYN, OFF32>(a, node);
        if (stage == order - 1 && tile == 0 && threadIdx.x == 0)
            p.ctl[inst].t[(step + 1) & 1u] = t_n + h;
    }
}

// How the rounds are launched: workgroups > 0 selects the strided form with
// that many workgroups per round; workgroups == 0 the flat form, with
// round_grid[r] workgroups for round r (at least the round's tiles).
struct BatchShape {
    uint32_t workgroups;
    const uint32_t *round_grid;  // host array [rounds], flat form only
    uint32_t order;              // RK order of the batch (1, 2 or 3)
    bool off32;                  // every instance's arrays under 4 GiB (fits_off32)
};

// The init kernel and rounds [0, rounds) of the round kernel, back to back.
template <typename T, int D, int SCH, int DYN>
hipError_t batch_launch_one(const BatchPtrs<T> &p, uint32_t rounds, const BatchShape &sh,
                            hipStream_t s)
{
    const uint32_t order = sh.order;
    hipLaunchKernelGGL((batch_init<T>), dim3(1), dim3(256), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint32_t st = r % order, sp = r / order;
        if (sh.workgroups) {
            if (sh.off32)
                hipLaunchKernelGGL((batch_round<T, D, SCH, DYN, false, true>),
                                   dim3(sh.workgroups), dim3(256), 0, s, p, r, order, st, sp);
            else
                hipLaunchKernelGGL((batch_round<T, D, SCH, DYN, false, false>),
                                   dim3(sh.workgroups), dim3(256), 0, s, p, r, order, st, sp);
        } else {
            if (sh.off32)
                hipLaunchKernelGGL((batch_round<T, D, SCH, DYN, true, true>),
                                   dim3(sh.round_grid[r]), dim3(256), 0, s, p, r, order, st, sp);
            else
                hipLaunchKernelGGL((batch_round<T, D, SCH, DYN, true, false>),
                                   dim3(sh.round_grid[r]), dim3(256), 0, s, p, r, order, st, sp);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int D, int DYN>
hipError_t batch_launch_space(int space, const BatchPtrs<T> &p, uint32_t rounds,
                              const BatchShape &wg, hipStream_t s)
{
    if (space == kEno2) return batch_launch_one<T, D, kEno2, DYN>(p, rounds, wg, s);
    if (space == kEno3) return batch_launch_one<T, D, kEno3, DYN>(p, rounds, wg, s);
    if (space == kWeno5) return batch_launch_one<T, D, kWeno5, DYN>(p, rounds, wg, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t batch_launch_t(int ndim, int space, int dyn, const BatchPtrs<T> &p, uint32_t rounds,
                          const BatchShape &wg, hipStream_t s)
{
    switch (dyn) {
    case kTranslation:
        switch (ndim) {
        case 1: return batch_launch_space<T, 1, kTranslation>(space, p, rounds, wg, s);
        case 2: return batch_launch_space<T, 2, kTranslation>(space, p, rounds, wg, s);
        case 3: return batch_launch_space<T, 3, kTranslation>(space, p, rounds, wg, s);
        case 4: return batch_launch_space<T, 4, kTranslation>(space, p, rounds, wg, s);
        }
        break;
    case kBall:
        switch (ndim) {
        case 1: return batch_launch_space<T, 1, kBall>(space, p, rounds, wg, s);
        case 2: return batch_launch_space<T, 2, kBall>(space, p, rounds, wg, s);
        case 3: return batch_launch_space<T, 3, kBall>(space, p, rounds, wg, s);
        case 4: return batch_launch_space<T, 4, kBall>(space, p, rounds, wg, s);
        }
        break;
    case kDoubleIntegrator:
        if (ndim == 2) return batch_launch_space<T, 2, kDoubleIntegrator>(space, p, rounds, wg, s);
        break;
    case kRelDubins:
        if (ndim == 3) return batch_launch_space<T, 3, kRelDubins>(space, p, rounds, wg, s);
        break;
    case kDubins4D:
        if (ndim == 4) return batch_launch_space<T, 4, kDubins4D>(space, p, rounds, wg, s);
        break;
    case kRockets:
        if (ndim == 3) return batch_launch_space<T, 3, kRockets>(space, p, rounds, wg, s);
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace hj
