// Batched solves (C ABI part of include/hj.h): many independent grids that
// share ndim, dynamics kind, derivative scheme, RK order and precision are
// advanced together, one fused launch per RK-stage round over every running
// instance (hj_batch_impl.h).  The sequence of round launches is captured once
// in a hipGraph and replayed; every table the kernels read lives in device
// memory, so a new batch composition only needs uploads before the replay.
// The handle keeps a few captured graphs, each for one kernel variant, launch
// shape and round count (flat launches: with per-round workgroup counts that
// a replayed batch must not exceed), and captures a new one when none fits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "hj_batch_impl.h"
#include "hj_host.h"

using namespace hj;

namespace hj {
hipError_t batch_launch_f64(int ndim, int space, int dyn, const BatchPtrs<double> &p,
                            uint32_t rounds, const BatchShape &shape, hipStream_t s);
hipError_t batch_launch_f32(int ndim, int space, int dyn, const BatchPtrs<float> &p,
                            uint32_t rounds, const BatchShape &shape, hipStream_t s);
}  // namespace hj

struct hj_batch_s {
    int device = 0;
    uint32_t tile_nodes = 256;
    uint32_t workgroups = 0;   // 0: flat launches (one workgroup per 256-node tile)
    bool use_graph = true;
    bool off32 = true;         // the current batch's arrays are all under 4 GiB
    bool addr64 = false;       // HJ_ADDR64 set at creation: 64-bit addressing (test switch)

    // device tables and their capacities
    uint32_t cap_inst = 0, cap_rounds = 0, cap_tiles = 0;
    void *inst = nullptr;        // BatchInst<T>[cap_inst]
    BatchCtl *ctl = nullptr;     // [cap_inst]
    TileRef *tile_map = nullptr;    // [cap_tiles]
    uint32_t *round_off = nullptr;  // [cap_rounds + 1]
    BatchGlobal *gl = nullptr;
    // pinned host staging
    void *h_inst = nullptr;
    TileRef *h_tile_map = nullptr;
    uint32_t *h_round_off = nullptr;
    BatchGlobal *h_gl = nullptr;
    BatchCtl *h_ctl_out = nullptr;    // read back after a solve
    uint32_t last_n = 0;
    std::vector<uint32_t> last_steps;
    // recorded after the read-back of a solve: the next solve reuses the
    // tables and staging buffers only after it
    hipEvent_t done_evt = nullptr;
    bool pending = false;

    // captured graphs and the launches they were captured for
    struct Graph {
        hipGraphExec_t exec = nullptr;
        int nd = -1, space = -1, dyn = -1, prec = -1, order = -1;
        uint32_t wg = 0, rounds = 0;
        bool off32 = true;
        std::vector<uint32_t> grid;  // flat: workgroups of each round
        uint64_t used = 0;           // last use (LRU)
    };
    std::vector<Graph> graphs;
    uint64_t clock = 0;
    hipStream_t capture_stream = nullptr;
    std::vector<uint32_t> round_grid;  // scratch: workgroups per round
};

namespace {

size_t inst_size(hj_precision p)
{
    return p == HJ_FP64 ? sizeof(BatchInst<double>) : sizeof(BatchInst<float>);
}

void free_tables(hj_batch_t b)
{
    if (b->inst) (void)hipFree(b->inst);
    if (b->ctl) (void)hipFree(b->ctl);
    if (b->tile_map) (void)hipFree(b->tile_map);
    if (b->round_off) (void)hipFree(b->round_off);
    if (b->h_inst) (void)hipHostFree(b->h_inst);
    if (b->h_tile_map) (void)hipHostFree(b->h_tile_map);
    if (b->h_round_off) (void)hipHostFree(b->h_round_off);
    if (b->h_ctl_out) (void)hipHostFree(b->h_ctl_out);
    b->inst = nullptr;
    b->ctl = nullptr;
    b->tile_map = nullptr;
    b->round_off = nullptr;
    b->h_inst = nullptr;
    b->h_tile_map = nullptr;
    b->h_round_off = nullptr;
    b->h_ctl_out = nullptr;
    b->cap_inst = b->cap_rounds = b->cap_tiles = 0;
}

void drop_graph(hj_batch_t b)
{
    for (auto &g : b->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

constexpr size_t kMaxGraphs = 16;

hj_status host_alloc(void **p, size_t bytes, const char *what)
{
    HJ_HIP(hipHostMalloc(p, bytes, 0), what);
    return HJ_OK;
}

// Grow the tables to hold n instances, `rounds` rounds and `tiles` tiles per
// round (the tile map grows by at least half its size).  Any change of a
// device address invalidates the captured graphs.
hj_status reserve(hj_batch_t b, uint32_t n, uint32_t rounds, uint32_t tiles)
{
    if (n <= b->cap_inst && rounds <= b->cap_rounds && tiles <= b->cap_tiles) return HJ_OK;
    const uint32_t ci = std::max(n, b->cap_inst), cr = std::max(rounds, b->cap_rounds);
    const uint32_t ct = tiles <= b->cap_tiles
                            ? b->cap_tiles
                            : uint32_t(std::min<uint64_t>(
                                  0xffffffffu, std::max<uint64_t>(tiles, b->cap_tiles * 3ull / 2)));
    drop_graph(b);
    free_tables(b);
    hj_status s;
    const size_t isz = std::max(sizeof(BatchInst<double>), sizeof(BatchInst<float>));
    if ((s = dev_alloc(&b->inst, isz * ci, "batch instance table")) != HJ_OK) return s;
    if ((s = dev_alloc((void **)&b->ctl, sizeof(BatchCtl) * ci, "batch control")) != HJ_OK)
        return s;
    if ((s = dev_alloc((void **)&b->tile_map, sizeof(TileRef) * ct, "batch tile map")) != HJ_OK)
        return s;
    if ((s = dev_alloc((void **)&b->round_off, sizeof(uint32_t) * (cr + 1), "batch rounds")) !=
        HJ_OK)
        return s;
    if ((s = host_alloc(&b->h_inst, isz * ci, "pinned instance table")) != HJ_OK) return s;
    if ((s = host_alloc((void **)&b->h_tile_map, sizeof(TileRef) * ct, "pinned tile map")) !=
        HJ_OK)
        return s;
    if ((s = host_alloc((void **)&b->h_round_off, sizeof(uint32_t) * (cr + 1),
                        "pinned rounds")) != HJ_OK)
        return s;
    if ((s = host_alloc((void **)&b->h_ctl_out, sizeof(BatchCtl) * ci, "pinned control")) !=
        HJ_OK)
        return s;
    b->cap_inst = ci;
    b->cap_rounds = cr;
    b->cap_tiles = ct;
    return HJ_OK;
}

template <typename T>
BatchPtrs<T> ptrs(hj_batch_t b)
{
    BatchPtrs<T> p;
    p.inst = (const BatchInst<T> *)b->inst;
    p.ctl = b->ctl;
    p.tile_map = b->tile_map;
    p.round_off = b->round_off;
    p.gl = b->gl;
    p.map_cap = b->cap_tiles;
    return p;
}

hipError_t launch_any(hj_batch_t b, int nd, int space, int dyn, hj_precision prec,
                      uint32_t rounds, const BatchShape &sh, hipStream_t s)
{
    if (prec == HJ_FP64) return batch_launch_f64(nd, space, dyn, ptrs<double>(b), rounds, sh, s);
    return batch_launch_f32(nd, space, dyn, ptrs<float>(b), rounds, sh, s);
}

// Flat launches in a graph: a round's workgroup count rounded up so that
// about 8 sizes per power of two share one capture.
uint32_t grid_capacity(uint32_t tiles)
{
    if (tiles == 0) return 1;
    uint32_t q = 1;
    while (q * 16u <= tiles) q <<= 1;  // tiles / 16 < q <= tiles / 8 (for tiles >= 16)
    const uint64_t c = (uint64_t(tiles) + q - 1) / q * q;
    return c > 0x7fffffffu ? 0x7fffffffu : uint32_t(c);
}

// Launches the init kernel and the batch's rounds: directly, or by replaying
// a captured graph of the same kernel variant, launch shape and round count
// whose per-round workgroups (flat launches) cover the batch's tiles of
// every round, captured on demand (least recently used one dropped beyond
// kMaxGraphs).  The round tables (h_round_off) are the batch's.
hj_status run(hj_batch_t b, int nd, int space, int dyn, hj_precision prec, int order,
              uint32_t rounds, hipStream_t s)
{
    const bool flat = b->workgroups == 0;
    std::vector<uint32_t> &grid = b->round_grid;
    grid.assign(flat ? rounds : 0, 0u);
    for (uint32_t r = 0; flat && r < rounds; ++r)
        grid[r] = b->h_round_off[r + 1] - b->h_round_off[r];
    if (!b->use_graph) {
        const BatchShape sh{b->workgroups, grid.data(), uint32_t(order), b->off32};
        hipError_t e = launch_any(b, nd, space, dyn, prec, rounds, sh, s);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        return HJ_OK;
    }
    hj_batch_s::Graph *hit = nullptr;
    for (auto &g : b->graphs) {
        if (g.nd != nd || g.space != space || g.dyn != dyn || g.prec != prec ||
            g.order != order || g.wg != b->workgroups || g.rounds != rounds ||
            g.off32 != b->off32)
            continue;
        bool fits = true;
        for (uint32_t r = 0; flat && r < rounds && fits; ++r) fits = grid[r] <= g.grid[r];
        if (fits) {
            hit = &g;
            break;
        }
    }
    if (!hit) {
        hj_batch_s::Graph g;
        g.nd = nd;
        g.space = space;
        g.dyn = dyn;
        g.order = order;
        g.prec = prec;
        g.wg = b->workgroups;
        g.rounds = rounds;
        g.off32 = b->off32;
        g.grid.resize(grid.size());
        for (size_t r = 0; r < grid.size(); ++r) g.grid[r] = grid_capacity(grid[r]);
        if (!b->capture_stream)
            HJ_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking),
                   "capture stream");
        hipGraph_t graph = nullptr;
        HJ_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal),
               "begin capture");
        const BatchShape sh{b->workgroups, g.grid.data(), uint32_t(order), b->off32};
        hipError_t e = launch_any(b, nd, space, dyn, prec, rounds, sh, b->capture_stream);
        hipError_t e2 = hipStreamEndCapture(b->capture_stream, &graph);
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e, "batch launch (capture)");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "end capture");
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        if (b->graphs.size() >= kMaxGraphs) {
            auto lru = std::min_element(
                b->graphs.begin(), b->graphs.end(),
                [](const hj_batch_s::Graph &x, const hj_batch_s::Graph &y) {
                    return x.used < y.used;
                });
            (void)hipGraphExecDestroy(lru->exec);
            b->graphs.erase(lru);
        }
        b->graphs.push_back(std::move(g));
        hit = &b->graphs.back();
    }
    hit->used = ++b->clock;
    HJ_HIP(hipGraphLaunch(hit->exec, s), "graph launch");
    return HJ_OK;
}

// Nodes per tile of one instance: the configured maximum, shrunk (in steps
// of 256) so that the instance has at least kMinTiles tiles when it can.
constexpr uint32_t kMinTiles = 512;

uint32_t instance_tile(uint32_t total, uint32_t max_tile)
{
    uint32_t t = (total + kMinTiles - 1) / kMinTiles;
    t = (t + 255u) & ~255u;
    return t < 256u ? 256u : (t > max_tile ? max_tile : t);
}

template <typename T>
void fill_inst(void *dst, hj_grid_t g, void *vout, const void *v0, double dt, double t0,
               double tf, uint32_t tiles, uint32_t tile_nodes, uint32_t steps, hj_mode mode)
{
    BatchInst<T> in;
    std::memset(&in, 0, sizeof(in));
    in.geo = base_args<T>(g);
    in.v = (T *)vout;
    in.a = (T *)g->bufA;
    in.b = (T *)g->bufB;
    in.v0 = (const T *)v0;
    in.dt = dt;
    in.t0 = t0;
    in.tf = tf;
    in.tiles = tiles;
    in.tile_nodes = tile_nodes;
    in.steps = steps;
    in.tube = mode == HJ_TUBE ? 1 : 0;
    in.vi = mode == HJ_TUBE_VI ? 1 : 0;
    std::memcpy(dst, &in, sizeof(in));
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = uintptr_t(a), y = uintptr_t(b);
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

hj_status hj_batch_create(hj_batch_t *out)
{
    if (!out) return fail(HJ_E_ARG, "out is NULL");
    *out = nullptr;
    hj_batch_s *b = new (std::nothrow) hj_batch_s();
    if (!b) return fail(HJ_E_OOM, "host allocation of the batch handle");
    hj_status s = HJ_OK;
    b->addr64 = std::getenv("HJ_ADDR64") != nullptr;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) s = hip_fail(e, "hipGetDevice");
    if (s == HJ_OK) s = dev_alloc((void **)&b->gl, sizeof(BatchGlobal), "batch globals");
    if (s == HJ_OK) s = host_alloc((void **)&b->h_gl, sizeof(BatchGlobal), "pinned globals");
    if (s == HJ_OK) {
        e = hipEventCreateWithFlags(&b->done_evt, hipEventDisableTiming);
        if (e != hipSuccess) s = hip_fail(e, "batch event");
    }
    if (s != HJ_OK) {
        hj_batch_destroy(b);
        return s;
    }
    *out = b;
    return HJ_OK;
}

hj_status hj_batch_config(hj_batch_t b, int tile_nodes, int workgroups, int use_graph)
{
    if (!b) return fail(HJ_E_ARG, "null batch handle");
    if (tile_nodes < 256 || tile_nodes > (1 << 22) || (tile_nodes & 255))
        return fail(HJ_E_ARG, "tile_nodes must be a multiple of 256 in [256, 2^22]");
    if (workgroups < 0 || workgroups > 65536)
        return fail(HJ_E_ARG, "workgroups in [0, 65536] (0: flat launches)");
    if (b->workgroups != uint32_t(workgroups)) drop_graph(b);
    b->tile_nodes = uint32_t(tile_nodes);
    b->workgroups = uint32_t(workgroups);
    b->use_graph = use_graph != 0;
    return HJ_OK;
}

}  // extern "C"

namespace {

// Shared body of hj_solve_batch and hj_step_batch: instance i advances V[i]
// in place by up to max_steps RK steps (all remaining steps if max_steps <= 0)
// from time tcur[i] toward tf[i], with the termination rule taken relative to
// its original start t0[i].  copy_v0: V[i] <- V0[i] first (a fresh solve).
// fresh_alpha: reduce alpha again even where the handle has it cached.
hj_status batch_run(hj_batch_t b, int n, const hj_grid_t *gs, const void *const *V0s,
                    void *const *Vs, const double *t0, const double *tcur, const double *tf,
                    const hj_mode *modes, int64_t max_steps, bool copy_v0, bool fresh_alpha,
                    double *t_reached, hipStream_t st)
{
    if (!b) return fail(HJ_E_ARG, "null batch handle");
    if (n < 1 || !gs || !Vs || !t0 || !tcur || !tf || !modes)
        return fail(HJ_E_ARG, "need n >= 1 and non-NULL arrays");
    hj_status s;
    const hj_grid_t g0 = gs[0];
    for (int i = 0; i < n; ++i) {
        const hj_grid_t g = gs[i];
        if ((s = check_ready(g)) != HJ_OK) return s;
        if (g->nd != g0->nd || g->dyn != g0->dyn || g->space != g0->space ||
            g->order != g0->order || g->prec != g0->prec || g->device != b->device)
            return fail(HJ_E_ARG, "instances must share ndim, dynamics, scheme, RK order, "
                                  "precision and device");
        if (modes[i] != HJ_SET && modes[i] != HJ_TUBE && modes[i] != HJ_TUBE_VI)
            return fail(HJ_E_ARG, "batched modes are HJ_SET, HJ_TUBE and HJ_TUBE_VI");
        const void *v0 = V0s ? V0s[i] : nullptr;
        if (!Vs[i] || ((copy_v0 || modes[i] == HJ_TUBE) && !v0))
            return fail(HJ_E_ARG, "NULL V, or NULL V0 where it is read");
        if (!(std::isfinite(t0[i]) && std::isfinite(tcur[i]) && std::isfinite(tf[i]) &&
              tf[i] >= t0[i] && tcur[i] >= t0[i]))
            return fail(HJ_E_ARG, "need finite t0 <= t and t0 <= tf");
        if (v0 && overlap(v0, g->bytes(), Vs[i], g->bytes()))
            return fail(HJ_E_ARG, "V overlaps V0 for instance " + std::to_string(i));
        for (int j = 0; j < i; ++j) {
            const void *w0 = V0s ? V0s[j] : nullptr;
            if (gs[j] == g)
                return fail(HJ_E_ARG, "instances " + std::to_string(j) + " and " +
                                          std::to_string(i) +
                                          " use the same grid handle (its stage buffers "
                                          "hold one instance)");
            if (overlap(Vs[i], g->bytes(), Vs[j], gs[j]->bytes()) ||
                (w0 && overlap(Vs[i], g->bytes(), w0, gs[j]->bytes())))
                return fail(HJ_E_ARG, "instances " + std::to_string(j) + " and " +
                                          std::to_string(i) + " share memory");
        }
    }
    if (g0->space == HJ_UPWIND1 || g0->order == 1)
        return fail(HJ_E_UNSUPPORTED, "batched solves support ENO2, ENO3 and WENO5 with RK2/RK3");
    for (int i = 0; i < n; ++i)
        if (gs[i]->diss == HJ_DISS_GLF)
            return fail(HJ_E_UNSUPPORTED,
                        "batched solves take HJ_DISS_LF or HJ_DISS_LLF (GLF needs a grid-wide "
                        "reduction per stage)");
    HJ_HIP(hipSetDevice(b->device), "hipSetDevice");
    if (b->pending) {
        HJ_HIP(hipEventSynchronize(b->done_evt), "previous batch");
        b->pending = false;
    }

    // stage buffers: every instance's own, apart from every other instance's
    // buffers and from every V and V0 of the batch (caller workspaces may be
    // placed anywhere)
    const bool need_b = g0->order == 3;
    for (int i = 0; i < n; ++i)
        if ((s = ensure_buffers(gs[i], need_b)) != HJ_OK) return s;
    for (int i = 0; i < n; ++i) {
        const size_t bi = gs[i]->bytes();
        const void *own[2] = {gs[i]->bufA, need_b ? gs[i]->bufB : nullptr};
        for (const void *w : own) {
            if (!w) continue;
            for (int j = 0; j < n; ++j) {
                const size_t bj = gs[j]->bytes();
                const void *v0 = V0s ? V0s[j] : nullptr;
                bool clash = overlap(w, bi, Vs[j], bj) || (v0 && overlap(w, bi, v0, bj));
                if (j != i) {
                    clash = clash || overlap(w, bi, gs[j]->bufA, bj) ||
                            (need_b && overlap(w, bi, gs[j]->bufB, bj));
                }
                if (clash)
                    return fail(HJ_E_ARG, "stage buffers of instance " + std::to_string(i) +
                                              " overlap arrays of instance " +
                                              std::to_string(j));
            }
        }
        if (need_b && overlap(gs[i]->bufA, bi, gs[i]->bufB, bi))
            return fail(HJ_E_ARG, "stage buffers of instance " + std::to_string(i) + " overlap");
    }

    // alpha for every instance that needs it (GPU reductions), one wait
    bool any = false;
    for (int i = 0; i < n; ++i) {
        if (fresh_alpha || !gs[i]->alpha_valid) {
            if ((s = launch_alpha_readback(gs[i], st)) != HJ_OK) return s;
            gs[i]->alpha_valid = false;
            any = true;
        }
    }
    if (any) HJ_HIP(hipStreamSynchronize(st), "alpha synchronise");

    std::vector<double> dts(n);
    std::vector<uint32_t> steps(n), tiles(n), tsize(n);
    uint32_t max_n = 0;
    for (int i = 0; i < n; ++i) {
        if (!gs[i]->alpha_valid) accept_alpha(gs[i]);
        dts[i] = cfl_dt(gs[i]);
        // the Sec. 5 loop from the current time, relative rule as for a solve
        double t = tcur[i];
        uint32_t k = 0;
        if (tf[i] > t0[i])
            while (tf[i] - t >= kEpsT * (tf[i] - t0[i]) && (max_steps <= 0 || k < max_steps)) {
                const double h = dts[i] < tf[i] - t ? dts[i] : tf[i] - t;
                t = t + h;
                ++k;
            }
        steps[i] = k;
        if (t_reached) t_reached[i] = t;
        tsize[i] = b->workgroups ? instance_tile(uint32_t(gs[i]->total), b->tile_nodes) : 256u;
        tiles[i] = uint32_t((gs[i]->total + tsize[i] - 1) / tsize[i]);
        max_n = std::max(max_n, steps[i]);
    }
    const uint32_t order = uint32_t(g0->order);
    b->off32 = !b->addr64;
    for (int i = 0; i < n; ++i)
        b->off32 = b->off32 && (g0->prec == HJ_FP64 ? fits_off32<double>(uint64_t(gs[i]->total))
                                                   : fits_off32<float>(uint64_t(gs[i]->total)));
    const uint64_t rounds64 = uint64_t(order) * max_n;
    if (rounds64 >= (uint64_t(1) << 31)) return fail(HJ_E_ARG, "too many steps");
    const uint32_t rounds = uint32_t(rounds64);
    // instances by step count, descending: the active ones form a prefix
    std::vector<uint32_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0u);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](uint32_t x, uint32_t y) { return steps[x] > steps[y]; });
    std::vector<uint32_t> pre(n + 1, 0u);  // tiles of the first k sorted instances
    for (int k = 0; k < n; ++k) {
        const uint64_t next = uint64_t(pre[k]) + tiles[ord[k]];
        if (next > 0x7fffffffu) return fail(HJ_E_ARG, "too many tiles");
        pre[k + 1] = uint32_t(next);
    }
    if ((s = reserve(b, uint32_t(n), rounds, pre[n])) != HJ_OK) return s;
    for (int k = 0; k < n; ++k) {
        const uint32_t last = order * steps[ord[k]];
        for (uint32_t t = 0; t < tiles[ord[k]]; ++t)
            b->h_tile_map[pre[k] + t] = {ord[k], t, last, 0u};
    }
    // past the batch's tiles: entries that run in no round (a flat launch may
    // have more workgroups than the round has tiles)
    for (uint32_t e = pre[n]; e < b->cap_tiles; ++e) b->h_tile_map[e] = {0u, 0u, 0u, 0u};
    uint64_t total = 0;
    uint32_t active = uint32_t(n);
    for (uint32_t r = 0; r < rounds; ++r) {
        while (active > 0 && uint64_t(order) * steps[ord[active - 1]] <= r) --active;
        b->h_round_off[r] = uint32_t(total);
        total += pre[active];
        if (total >= (uint64_t(1) << 32) - 1) return fail(HJ_E_ARG, "too many work items");
    }
    b->h_round_off[rounds] = uint32_t(total);

    const size_t isz = inst_size(g0->prec);
    for (int i = 0; i < n; ++i) {
        char *dst = (char *)b->h_inst + isz * i;
        const void *v0 = V0s ? V0s[i] : nullptr;
        if (g0->prec == HJ_FP64)
            fill_inst<double>(dst, gs[i], Vs[i], v0, dts[i], tcur[i], tf[i], tiles[i], tsize[i],
                              steps[i], modes[i]);
        else
            fill_inst<float>(dst, gs[i], Vs[i], v0, dts[i], tcur[i], tf[i], tiles[i], tsize[i],
                             steps[i], modes[i]);
    }
    std::memset(b->h_gl, 0, sizeof(BatchGlobal));
    b->h_gl->items = uint32_t(total);
    b->h_gl->rounds = rounds;
    b->h_gl->ninst = uint32_t(n);
    b->h_gl->tile_nodes = b->tile_nodes;
    b->h_gl->order = order;

    HJ_HIP(hipMemcpyAsync(b->inst, b->h_inst, isz * n, hipMemcpyHostToDevice, st), "upload");
    HJ_HIP(hipMemcpyAsync(b->tile_map, b->h_tile_map, sizeof(TileRef) * b->cap_tiles,
                          hipMemcpyHostToDevice, st),
           "upload");
    HJ_HIP(hipMemcpyAsync(b->round_off, b->h_round_off, sizeof(uint32_t) * (rounds + 1),
                          hipMemcpyHostToDevice, st),
           "upload");
    HJ_HIP(hipMemcpyAsync(b->gl, b->h_gl, sizeof(BatchGlobal), hipMemcpyHostToDevice, st),
           "upload");
    if (copy_v0)
        for (int i = 0; i < n; ++i)
            HJ_HIP(hipMemcpyAsync(Vs[i], V0s[i], gs[i]->bytes(), hipMemcpyDeviceToDevice, st),
                   "copy V0");
    if ((s = run(b, g0->nd, g0->space, g0->dyn, g0->prec, g0->order, rounds, st)) != HJ_OK)
        return s;
    HJ_HIP(hipMemcpyAsync(b->h_ctl_out, b->ctl, sizeof(BatchCtl) * n, hipMemcpyDeviceToHost, st),
           "read-back");
    HJ_HIP(hipEventRecord(b->done_evt, st), "batch event");
    b->pending = true;
    b->last_n = uint32_t(n);
    b->last_steps = steps;
    return HJ_OK;
}

}  // namespace

extern "C" {

hj_status hj_solve_batch(hj_batch_t b, int n, const hj_grid_t *gs, const void *const *V0s,
                         void *const *Vouts, const double *t0, const double *tf,
                         const hj_mode *modes, void *hip_stream)
{
    if (!V0s) return fail(HJ_E_ARG, "V0s is NULL");
    return batch_run(b, n, gs, V0s, Vouts, t0, t0, tf, modes, 0, true, true, nullptr,
                     (hipStream_t)hip_stream);
}

hj_status hj_step_batch(hj_batch_t b, int n, const hj_grid_t *gs, const void *const *V0s,
                        void *const *Vs, const double *t0, double *t, const double *tf,
                        const hj_mode *modes, int max_steps, int *steps_taken, int *finished,
                        void *hip_stream)
{
    if (!t) return fail(HJ_E_ARG, "t is NULL");
    std::vector<double> reached(n > 0 ? n : 1);
    hj_status s = batch_run(b, n, gs, V0s, Vs, t0, t, tf, modes, max_steps, false, false,
                            reached.data(), (hipStream_t)hip_stream);
    if (s != HJ_OK) return s;
    for (int i = 0; i < n; ++i) {
        t[i] = reached[i];
        if (steps_taken) steps_taken[i] = int(b->last_steps[i]);
        if (finished) finished[i] = !(tf[i] > t0[i] && tf[i] - t[i] >= kEpsT * (tf[i] - t0[i]));
    }
    return HJ_OK;
}

hj_status hj_batch_wait(hj_batch_t b, void *hip_stream, double *t_final, int64_t *items)
{
    if (!b) return fail(HJ_E_ARG, "null batch handle");
    HJ_HIP(hipStreamSynchronize((hipStream_t)hip_stream), "batch synchronise");
    if (b->last_n == 0) return fail(HJ_E_STATE, "no batch has been solved");
    if (items) *items = int64_t(b->h_gl->items);
    if (t_final)
        for (uint32_t i = 0; i < b->last_n; ++i)
            t_final[i] = b->h_ctl_out[i].t[b->last_steps[i] & 1u];
    return HJ_OK;
}

hj_status hj_batch_destroy(hj_batch_t b)
{
    if (!b) return HJ_OK;
    (void)hipSetDevice(b->device);
    if (b->pending) (void)hipEventSynchronize(b->done_evt);
    drop_graph(b);
    if (b->done_evt) (void)hipEventDestroy(b->done_evt);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    free_tables(b);
    if (b->gl) (void)hipFree(b->gl);
    if (b->h_gl) (void)hipHostFree(b->h_gl);
    delete b;
    return HJ_OK;
}

}  // extern "C"
