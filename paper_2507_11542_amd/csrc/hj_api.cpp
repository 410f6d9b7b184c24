// libhj host runtime: the C ABI of include/hj.h.
//
// A handle holds the grid geometry (Sec. 2.1), the per-axis coordinate and
// trigonometric tables (computed once with the host libm), the compiled
// dynamics and scheme choice, and the device buffers of the TVD-RK stages.
// hj_solve reduces alpha on the GPU, reads it back once, fixes the whole step
// schedule on the host in FP64 (Sec. 5 time loop) and enqueues every stage
// launch on the caller's stream without further synchronisation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hj_host.h"

using namespace hj;

static_assert(sizeof(hj_shape) == 88, "hj_shape layout of include/hj.h");

namespace {

thread_local std::string g_err;

int halo_of(int space) { return space == HJ_UPWIND1 ? 1 : (space == HJ_ENO2 ? 2 : 3); }  // ENO3, WENO5: 3

// Testing hook: HJ_FAULT_OOM=1 makes every device allocation of the library
// report HJ_E_OOM without calling the allocator.
bool fault_oom()
{
    const char *s = std::getenv("HJ_FAULT_OOM");
    return s && s[0] == '1';
}

}  // namespace

namespace hj {

hj_status fail(hj_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

hj_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? HJ_E_OOM : HJ_E_DEVICE;
}

hj_status dev_alloc(void **p, size_t bytes, const char *what)
{
    if (fault_oom()) return fail(HJ_E_OOM, std::string(what) + ": injected allocation failure");
    HJ_HIP(hipMalloc(p, bytes), what);
    return HJ_OK;
}

hj_status use_device(hj_grid_t g)
{
    HJ_HIP(hipSetDevice(g->device), "hipSetDevice");
    return HJ_OK;
}

hj_status ensure_buffers(hj_grid_t g, bool need_b)
{
    hj_status s;
    if (!g->bufA && (s = dev_alloc(&g->bufA, g->bytes(), "stage buffer A")) != HJ_OK) return s;
    if (need_b && !g->bufB && (s = dev_alloc(&g->bufB, g->bytes(), "stage buffer B")) != HJ_OK)
        return s;
    return HJ_OK;
}

hj_status check_ready(hj_grid_t g)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    if (g->dyn < 0) return fail(HJ_E_STATE, "hj_set_dynamics has not been called");
    const int w = halo_of(g->space);
    for (int d = 0; d < g->nd; ++d)
        if (g->n[d] < 2 * w + 1)
            return fail(HJ_E_ARG, "axis " + std::to_string(d) + " has " +
                                      std::to_string(g->n[d]) + " nodes; the scheme needs >= " +
                                      std::to_string(2 * w + 1));
    return HJ_OK;
}

// GPU max-reduction of the speed bounds (Sec. 4), read back through pinned
// memory.
hj_status launch_alpha_readback(hj_grid_t g, hipStream_t s)
{
    AlphaArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tab = g->tab64;
    for (int d = 0; d < kMaxDim; ++d) {
        a.n[d] = uint32_t(g->n[d]);
        a.tab_off[d] = g->tab_off[d];
    }
    a.total = uint32_t(g->total);
    for (int k = 0; k < 8; ++k) a.prm[k] = g->prm[k];
    hipError_t e = launch_alpha(g->nd, g->dyn, a, g->partial, g->alpha_dev, s);
    if (e != hipSuccess) return hip_fail(e, "alpha reduction launch");
    HJ_HIP(hipMemcpyAsync(g->alpha_host, g->alpha_dev, sizeof(double) * g->nd,
                          hipMemcpyDeviceToHost, s),
           "alpha read-back");
    return HJ_OK;
}

void accept_alpha(hj_grid_t g)
{
    for (int d = 0; d < g->nd; ++d) g->alpha[d] = g->alpha_host[d];
    g->alpha_valid = true;
}

// The one synchronisation of a solve.
hj_status compute_alpha(hj_grid_t g, hipStream_t s)
{
    hj_status st = launch_alpha_readback(g, s);
    if (st != HJ_OK) return st;
    HJ_HIP(hipStreamSynchronize(s), "alpha synchronise");
    accept_alpha(g);
    return HJ_OK;
}

// Sec. 4 CFL bound: dt * sum_d alpha_d / dx_d = cfl.
double cfl_dt(hj_grid_t g)
{
    double rate = 0.0;
    for (int d = 0; d < g->nd; ++d) rate += g->alpha[d] / g->dx[d];
    return rate > 0.0 ? g->cfl / rate : INFINITY;
}

const double kEpsT = 100.0 * 2.220446049250313e-16;

// Sec. 5 time loop: step sizes min(dt, tf - t) until tf - t < eps (tf - t0).
void schedule(double dt, double t0, double tf, std::vector<double> *hs)
{
    double t = t0;
    if (!(tf > t0)) return;
    while (tf - t >= kEpsT * (tf - t0)) {
        const double h = dt < tf - t ? dt : tf - t;
        hs->push_back(h);
        t = t + h;
    }
}

template <typename T>
StageArgs<T> base_args(hj_grid_t g)
{
    StageArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.tab = (const T *)(g->prec == HJ_FP64 ? (const void *)g->tab64 : (const void *)g->tab32);
    for (int d = 0; d < kMaxDim; ++d) {
        a.n[d] = uint32_t(g->n[d]);
        a.stride[d] = g->stride[d];
        a.tab_off[d] = g->tab_off[d];
        const DivMagic mg = div_magic(uint32_t(g->n[d]));
        a.nmul[d] = mg.m;
        a.nshift[d] = mg.k;
        a.dx[d] = T(g->dx[d]);
        a.inv_dx[d] = T(1.0 / g->dx[d]);
        a.inv_2dx[d] = T(1.0 / (2.0 * g->dx[d]));
        a.inv_3dx[d] = T(1.0 / (3.0 * g->dx[d]));
        a.alpha[d] = T(g->alpha[d]);
    }
    a.total = uint32_t(g->total);
    a.periodic = g->pmask;
    a.addr64 = g->addr64 ? 1u : 0u;
    for (int k = 0; k < 8; ++k) a.prm[k] = T(g->prm[k]);
    a.diss = g->diss;
    a.box = (const T *)g->box_dev;
    return a;
}
template StageArgs<double> base_args<double>(hj_grid_t g);
template StageArgs<float> base_args<float>(hj_grid_t g);

}  // namespace hj

namespace {

template <typename T>
hj_status launch(hj_grid_t g, const StageArgs<T> &a, hipStream_t s);

// kGLF: the costate box of the stage input a.vs into g->box_dev, on the
// stream before the stage.
hj_status ensure_box(hj_grid_t g)
{
    hj_status s;
    const size_t e = g->elem();
    if (!g->box_dev && (s = dev_alloc(&g->box_dev, e * 2 * kMaxDim, "costate box")) != HJ_OK)
        return s;
    if (!g->box_part &&
        (s = dev_alloc(&g->box_part, e * box_partial_values(uint32_t(g->total), g->nd),
                       "costate box partials")) != HJ_OK)
        return s;
    return HJ_OK;
}

template <>
hj_status launch<double>(hj_grid_t g, const StageArgs<double> &a, hipStream_t s)
{
    if (a.diss == kGLF) {
        hipError_t e = launch_box_f64(g->nd, g->space, a, (double *)g->box_part,
                                      (double *)g->box_dev, s);
        if (e != hipSuccess) return hip_fail(e, "costate box (fp64)");
    }
    hipError_t e = launch_stage_f64(g->nd, g->space, g->dyn, a, s);
    if (e != hipSuccess) return hip_fail(e, "stage launch (fp64)");
    return HJ_OK;
}

template <>
hj_status launch<float>(hj_grid_t g, const StageArgs<float> &a, hipStream_t s)
{
    if (a.diss == kGLF) {
        hipError_t e = launch_box_f32(g->nd, g->space, a, (float *)g->box_part,
                                      (float *)g->box_dev, s);
        if (e != hipSuccess) return hip_fail(e, "costate box (fp32)");
    }
    hipError_t e = launch_stage_f32(g->nd, g->space, g->dyn, a, s);
    if (e != hipSuccess) return hip_fail(e, "stage launch (fp32)");
    return HJ_OK;
}

// What a step does beyond the free RK stages: the tube minimum with v0 in
// its last stage, the restricted update L = min(L, 0) in every stage.
struct StepKind {
    bool tube;
    bool vi;
};

StepKind step_kind(hj_mode mode) { return StepKind{mode == HJ_TUBE, mode == HJ_TUBE_VI}; }

// One stage: out = combine(vs, vb, L(vs)), then min with v0 when tube.
template <typename T>
hj_status stage(hj_grid_t g, const void *vs, const void *vb, const void *v0, void *out,
                Combine c, double dt, double wb, double w2, double den, bool tube, bool vi,
                hipStream_t s)
{
    if (g->diss == HJ_DISS_GLF) {
        hj_status st = ensure_box(g);
        if (st != HJ_OK) return st;
    }
    StageArgs<T> a = base_args<T>(g);
    a.vs = (const T *)vs;
    a.vb = (const T *)vb;
    a.v0 = (const T *)v0;
    a.out = (T *)out;
    a.combine = c;
    a.dt = T(dt);
    a.wb = T(wb);
    a.w2 = T(w2);
    a.den = T(den);
    a.tube = tube ? 1 : 0;
    a.vi = vi ? 1 : 0;
    return launch<T>(g, a, s);
}

// One TVD-RK step of size h in place on v (Sec. 5, odeCFL listing):
//   RK1  v <- v + h L(v)
//   RK2  A <- v + h L(v);  v <- (v + (A + h L(A))) / 2
//   RK3  A <- v + h L(v);  B <- (3v + (A + h L(A))) / 4;  v <- (v + 2(B + h L(B))) / 3
// followed by the tube minimum with v0 (fused in the last stage); every
// stage restricts its update in the variational-inequality tube.
template <typename T>
hj_status rk_step(hj_grid_t g, void *v, const void *v0, StepKind k, double h, hipStream_t s)
{
    hj_status st;
    if (g->order == 1) {
        if ((st = stage<T>(g, v, nullptr, v0, g->bufA, kEuler, h, 0, 0, 1, k.tube, k.vi, s)) !=
            HJ_OK)
            return st;
        HJ_HIP(hipMemcpyAsync(v, g->bufA, g->bytes(), hipMemcpyDeviceToDevice, s),
               "RK1 copy-back");
        return HJ_OK;
    }
    if ((st = stage<T>(g, v, nullptr, nullptr, g->bufA, kEuler, h, 0, 0, 1, false, k.vi, s)) !=
        HJ_OK)
        return st;
    if (g->order == 2)
        return stage<T>(g, g->bufA, v, v0, v, kBlend, h, 1.0, 1.0, 2.0, k.tube, k.vi, s);
    if ((st = stage<T>(g, g->bufA, v, nullptr, g->bufB, kBlend, h, 3.0, 1.0, 4.0, false, k.vi,
                       s)) != HJ_OK)
        return st;
    return stage<T>(g, g->bufB, v, v0, v, kBlend, h, 1.0, 2.0, 3.0, k.tube, k.vi, s);
}

// The steps hs in place on v.  In the tube-at-outputs mode the steps are free
// except the last, whose last stage takes the minimum with v0.
template <typename T>
hj_status run_steps(hj_grid_t g, void *v, const void *v0, hj_mode mode,
                    const std::vector<double> &hs, hipStream_t s)
{
    const StepKind k = step_kind(mode);
    for (size_t i = 0; i < hs.size(); ++i) {
        StepKind ki = k;
        if (mode == HJ_TUBE_OUTPUTS && i + 1 == hs.size()) ki.tube = true;
        hj_status st = rk_step<T>(g, v, v0, ki, hs[i], s);
        if (st != HJ_OK) return st;
    }
    return HJ_OK;
}

bool known_mode(hj_mode m)
{
    return m == HJ_SET || m == HJ_TUBE || m == HJ_TUBE_VI || m == HJ_TUBE_OUTPUTS;
}

bool overlap(const void *a, const void *b, size_t bytes)
{
    const uintptr_t x = uintptr_t(a), y = uintptr_t(b);
    return x < y + bytes && y < x + bytes;
}

// [a, a + na) and [b, b + nb) share a byte
bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = uintptr_t(a), y = uintptr_t(b);
    return x < y + nb && y < x + na;
}

}  // namespace

namespace hj {

hj_status solve_check(hj_grid_t g, const void *V0, const void *V_out, double t0, double tf,
                      hj_mode mode)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (!V0 || !V_out) return fail(HJ_E_ARG, "V0 and V_out must be non-NULL");
    if (!known_mode(mode)) return fail(HJ_E_ARG, "unknown mode");
    if (!(std::isfinite(t0) && std::isfinite(tf) && tf >= t0))
        return fail(HJ_E_ARG, "need finite t0 <= tf");
    if (overlap(V0, V_out, g->bytes())) return fail(HJ_E_ARG, "V_out overlaps V0");
    return HJ_OK;
}

// The body of hj_solve with the stage buffers A and B given (B unused below
// RK3): alpha (one synchronisation), the schedule, V_out <- V0 and the step
// launches, all on st.  The handle's own buffers are restored before return;
// the launches already hold A and B by value.
hj_status solve_enqueue(hj_grid_t g, const void *V0, void *V_out, double t0, double tf,
                        hj_mode mode, void *A, void *B, hipStream_t st)
{
    hj_status s = compute_alpha(g, st);
    if (s != HJ_OK) return s;
    std::vector<double> hs;
    schedule(cfl_dt(g), t0, tf, &hs);
    g->last_steps = int64_t(hs.size());
    HJ_HIP(hipMemcpyAsync(V_out, V0, g->bytes(), hipMemcpyDeviceToDevice, st), "copy V0");
    void *own_a = g->bufA, *own_b = g->bufB;
    g->bufA = A;
    g->bufB = B;
    if (g->prec == HJ_FP64)
        s = run_steps<double>(g, V_out, V0, mode, hs, st);
    else
        s = run_steps<float>(g, V_out, V0, mode, hs, st);
    g->bufA = own_a;
    g->bufB = own_b;
    return s;
}

hj_status check_result(hj_grid_t g, const void *V, size_t n, bool fp64, hipStream_t st)
{
    if (!(g->check & HJ_CHECK_FINITE)) return HJ_OK;
    for (size_t off = 0; off < n; off += size_t(1) << 30) {
        const size_t m = n - off < (size_t(1) << 30) ? n - off : (size_t(1) << 30);
        const void *p = (const char *)V + off * (fp64 ? 8 : 4);
        hipError_t e = launch_scan_nonfinite(p, fp64 ? 1 : 0, uint32_t(m), g->check_dev, st);
        if (e != hipSuccess) return hip_fail(e, "non-finite scan");
        HJ_HIP(hipMemcpyAsync(g->check_host, g->check_dev, sizeof(int), hipMemcpyDeviceToHost,
                              st),
               "non-finite scan read-back");
        HJ_HIP(hipStreamSynchronize(st), "non-finite scan synchronise");
        if (*g->check_host)
            return fail(HJ_E_NUMERIC, "the result holds NaN or infinite values");
    }
    return HJ_OK;
}

}  // namespace hj

extern "C" {

const char *hj_last_error(void) { return g_err.c_str(); }

hj_status hj_set_check(hj_grid_t g, int flags)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    if (flags & ~HJ_CHECK_FINITE) return fail(HJ_E_ARG, "unknown check flags");
    if (flags & HJ_CHECK_FINITE) {
        hj_status s = use_device(g);
        if (s != HJ_OK) return s;
        if (!g->check_dev &&
            (s = dev_alloc((void **)&g->check_dev, sizeof(int), "check flag")) != HJ_OK)
            return s;
        if (!g->check_host) {
            hipError_t e = hipHostMalloc((void **)&g->check_host, sizeof(int), 0);
            if (e != hipSuccess) return hip_fail(e, "pinned check flag");
        }
    }
    g->check = flags;
    return HJ_OK;
}

const char *hj_version(void) { return "libhj 0.1 (gfx950)"; }

hj_status hj_grid_create(int ndim, const int64_t *N, const double *lo, const double *hi,
                         uint32_t periodic_mask, hj_precision prec, hj_grid_t *out)
{
    if (!out) return fail(HJ_E_ARG, "out is NULL");
    *out = nullptr;
    if (ndim < 1 || ndim > kMaxDim) return fail(HJ_E_ARG, "ndim must be in [1, 4]");
    if (!N || !lo || !hi) return fail(HJ_E_ARG, "N, lo and hi must be non-NULL");
    if (prec != HJ_FP64 && prec != HJ_FP32) return fail(HJ_E_ARG, "unknown precision");
    if (periodic_mask >> ndim) return fail(HJ_E_ARG, "periodic_mask names an axis >= ndim");
    int64_t total = 1;
    for (int d = 0; d < ndim; ++d) {
        if (N[d] < 3) return fail(HJ_E_ARG, "every axis needs at least 3 nodes");
        if (!(std::isfinite(lo[d]) && std::isfinite(hi[d]) && lo[d] < hi[d]))
            return fail(HJ_E_ARG, "need finite lo < hi on every axis");
        total *= N[d];
        if (total >= (int64_t(1) << 31)) return fail(HJ_E_ARG, "grid exceeds 2^31 nodes");
    }
    hj_grid_s *g = new (std::nothrow) hj_grid_s();
    if (!g) return fail(HJ_E_OOM, "host allocation of the handle");
    g->nd = ndim;
    g->prec = prec;
    g->pmask = periodic_mask;
    g->total = total;
    uint32_t off = 0;
    for (int d = 0; d < ndim; ++d) {
        g->n[d] = N[d];
        g->lo[d] = lo[d];
        g->hi[d] = hi[d];
        const bool per = (periodic_mask >> d) & 1u;
        g->dx[d] = per ? (hi[d] - lo[d]) / double(N[d]) : (hi[d] - lo[d]) / double(N[d] - 1);
        g->tab_off[d] = off;
        off += uint32_t(3 * N[d]);
    }
    uint32_t st = 1;
    for (int d = ndim - 1; d >= 0; --d) {
        g->stride[d] = st;
        st *= uint32_t(g->n[d]);
    }
    // coordinate tables x_k = lo + k dx, cos x_k, sin x_k (host libm, FP64)
    std::vector<double> t64(off);
    for (int d = 0; d < ndim; ++d)
        for (int64_t k = 0; k < N[d]; ++k) {
            const double x = lo[d] + double(k) * g->dx[d];
            t64[g->tab_off[d] + k] = x;
            t64[g->tab_off[d] + N[d] + k] = std::cos(x);
            t64[g->tab_off[d] + 2 * N[d] + k] = std::sin(x);
        }
    hj_status s = HJ_OK;
    // test switch: the 64-bit-addressing form of the stage kernels whatever
    // the grid's size (the form grids of 4 GiB arrays and more take)
    g->addr64 = std::getenv("HJ_ADDR64") != nullptr;
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) s = hip_fail(e, "hipGetDevice");
    if (s == HJ_OK) s = dev_alloc((void **)&g->tab64, sizeof(double) * off, "coordinate table");
    if (s == HJ_OK) {
        e = hipMemcpy(g->tab64, t64.data(), sizeof(double) * off, hipMemcpyHostToDevice);
        if (e != hipSuccess) s = hip_fail(e, "coordinate table upload");
    }
    if (s == HJ_OK && prec == HJ_FP32) {
        std::vector<float> t32(t64.begin(), t64.end());
        s = dev_alloc((void **)&g->tab32, sizeof(float) * off, "coordinate table (fp32)");
        if (s == HJ_OK) {
            e = hipMemcpy(g->tab32, t32.data(), sizeof(float) * off, hipMemcpyHostToDevice);
            if (e != hipSuccess) s = hip_fail(e, "coordinate table upload (fp32)");
        }
    }
    if (s == HJ_OK)
        s = dev_alloc((void **)&g->partial,
                      sizeof(double) * alpha_blocks(uint32_t(total)) * ndim, "alpha partials");
    if (s == HJ_OK) s = dev_alloc((void **)&g->alpha_dev, sizeof(double) * kMaxDim, "alpha");
    if (s == HJ_OK) {
        e = hipHostMalloc((void **)&g->alpha_host, sizeof(double) * kMaxDim, 0);
        if (e != hipSuccess) s = hip_fail(e, "pinned alpha");
    }
    if (s != HJ_OK) {
        hj_grid_destroy(g);
        return s;
    }
    *out = g;
    return HJ_OK;
}

hj_status hj_set_dynamics(hj_grid_t g, hj_dyn kind, const double *params, int nparams)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    int want = -1, nd_need = 0;
    switch (kind) {
    case HJ_DYN_TRANSLATION: want = g->nd; break;
    case HJ_DYN_BALL: want = 1; break;
    case HJ_DYN_DOUBLE_INTEGRATOR: want = 1; nd_need = 2; break;
    case HJ_DYN_REL_DUBINS: want = 4; nd_need = 3; break;
    case HJ_DYN_DUBINS4D: want = 2; nd_need = 4; break;
    case HJ_DYN_ROCKETS: want = 3; nd_need = 3; break;
    default: return fail(HJ_E_ARG, "unknown dynamics");
    }
    if (nd_need && g->nd != nd_need)
        return fail(HJ_E_UNSUPPORTED, "these dynamics need ndim = " + std::to_string(nd_need));
    if (nparams != want || (want > 0 && !params))
        return fail(HJ_E_ARG, "dynamics expects " + std::to_string(want) + " parameters");
    for (int k = 0; k < nparams; ++k)
        if (!std::isfinite(params[k])) return fail(HJ_E_ARG, "non-finite dynamics parameter");
    g->dyn = kind;
    for (int k = 0; k < 8; ++k) g->prm[k] = k < nparams ? params[k] : 0.0;
    g->alpha_valid = false;
    return HJ_OK;
}

hj_status hj_set_scheme(hj_grid_t g, hj_space space, hj_time time, double cfl)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    if (space != HJ_UPWIND1 && space != HJ_ENO2 && space != HJ_ENO3 && space != HJ_WENO5)
        return fail(HJ_E_ARG, "unknown spatial scheme");
    if (time != HJ_RK1 && time != HJ_RK2 && time != HJ_RK3)
        return fail(HJ_E_ARG, "unknown RK order");
    if (!(cfl > 0.0 && cfl <= 1.0)) return fail(HJ_E_ARG, "cfl must be in (0, 1]");
    g->space = space;
    g->order = time;
    g->cfl = cfl;
    return HJ_OK;
}

hj_status hj_set_dissipation(hj_grid_t g, hj_dissipation kind)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    if (kind != HJ_DISS_LF && kind != HJ_DISS_LLF && kind != HJ_DISS_GLF)
        return fail(HJ_E_ARG, "unknown dissipation kind");
    g->diss = kind;
    return HJ_OK;
}

hj_status hj_get_schedule(hj_grid_t g, double t0, double tf, double *alpha, double *dt,
                          int64_t *n_steps, void *hip_stream)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (!(std::isfinite(t0) && std::isfinite(tf) && tf >= t0))
        return fail(HJ_E_ARG, "need finite t0 <= tf");
    if ((s = use_device(g)) != HJ_OK) return s;
    if ((s = compute_alpha(g, (hipStream_t)hip_stream)) != HJ_OK) return s;
    const double d = cfl_dt(g);
    std::vector<double> hs;
    schedule(d, t0, tf, &hs);
    if (alpha)
        for (int k = 0; k < g->nd; ++k) alpha[k] = g->alpha[k];
    if (dt) *dt = d;
    if (n_steps) *n_steps = int64_t(hs.size());
    return HJ_OK;
}

hj_status hj_get_info(hj_grid_t g, double *alpha, double *dt, int64_t *n_steps)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (!g->alpha_valid) {
        if ((s = use_device(g)) != HJ_OK) return s;
        if ((s = compute_alpha(g, nullptr)) != HJ_OK) return s;
    }
    if (alpha)
        for (int k = 0; k < g->nd; ++k) alpha[k] = g->alpha[k];
    if (dt) *dt = cfl_dt(g);
    if (n_steps) *n_steps = g->last_steps;
    return HJ_OK;
}

hj_status hj_solve(hj_grid_t g, const void *V0, void *V_out, double t0, double tf, hj_mode mode,
                   void *hip_stream)
{
    hj_status s = solve_check(g, V0, V_out, t0, tf, mode);
    if (s != HJ_OK) return s;
    if ((s = use_device(g)) != HJ_OK) return s;
    if ((s = ensure_buffers(g, g->order == 3)) != HJ_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = solve_enqueue(g, V0, V_out, t0, tf, mode, g->bufA, g->bufB, st)) != HJ_OK) return s;
    return check_result(g, V_out, size_t(g->total), g->prec == HJ_FP64, st);
}

hj_status hj_init_shapes(hj_grid_t g, void *V_out, const hj_shape *shapes, int nshapes,
                         void *hip_stream)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    if (!V_out || !shapes) return fail(HJ_E_ARG, "V_out and shapes must be non-NULL");
    if (nshapes < 1 || nshapes > kMaxShapes)
        return fail(HJ_E_ARG, "nshapes must be in [1, " + std::to_string(kMaxShapes) + "]");
    ShapeArgs a;
    std::memset(&a, 0, sizeof(a));
    const uint32_t all = (1u << g->nd) - 1u;
    for (int k = 0; k < nshapes; ++k) {
        const hj_shape &s = shapes[k];
        if (s.kind < HJ_SHAPE_SPHERE || s.kind > HJ_SHAPE_ELLIPSOID)
            return fail(HJ_E_ARG, "unknown shape kind in shape " + std::to_string(k));
        if (k > 0 && (s.op < HJ_OP_UNION || s.op > HJ_OP_SUBTRACT))
            return fail(HJ_E_ARG, "unknown shape op in shape " + std::to_string(k));
        if (s.axes & ~all) return fail(HJ_E_ARG, "shape axes name an axis >= ndim");
        ShapeDesc &d = a.s[k];
        d.kind = s.kind;
        d.op = s.op;
        d.mask = (s.kind == HJ_SHAPE_SPHERE || s.axes == 0) ? all : s.axes;
        for (int i = 0; i < kMaxDim; ++i) {
            d.center[i] = s.center[i];
            d.size[i] = s.size[i];
        }
        d.radius = s.radius;
    }
    a.tab = g->tab64;
    a.out = V_out;
    for (int d = 0; d < kMaxDim; ++d) {
        a.n[d] = uint32_t(g->n[d]);
        a.tab_off[d] = g->tab_off[d];
    }
    a.total = uint32_t(g->total);
    a.nd = g->nd;
    a.nshapes = nshapes;
    a.fp32 = g->prec == HJ_FP32 ? 1 : 0;
    hj_status s = use_device(g);
    if (s != HJ_OK) return s;
    hipError_t e = launch_shapes(a, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "shapes launch");
    return HJ_OK;
}

hj_status hj_solve_outputs(hj_grid_t g, const void *V0, void *V_outs, double t0,
                           const double *times, int ntimes, hj_mode mode, void *hip_stream)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (!V0 || !V_outs || !times) return fail(HJ_E_ARG, "V0, V_outs and times must be non-NULL");
    if (ntimes < 1) return fail(HJ_E_ARG, "need ntimes >= 1");
    if (!known_mode(mode)) return fail(HJ_E_ARG, "unknown mode");
    if (!std::isfinite(t0)) return fail(HJ_E_ARG, "non-finite t0");
    for (int k = 0; k < ntimes; ++k)
        if (!std::isfinite(times[k]) || times[k] < (k ? times[k - 1] : t0))
            return fail(HJ_E_ARG, "output times must be finite, ascending and >= t0");
    const size_t bytes = g->bytes();
    const uintptr_t a = uintptr_t(V0), b = uintptr_t(V_outs);
    if (a < b + bytes * size_t(ntimes) && b < a + bytes)
        return fail(HJ_E_ARG, "V_outs overlaps V0");
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = use_device(g)) != HJ_OK) return s;
    if ((s = ensure_buffers(g, g->order == 3)) != HJ_OK) return s;
    if ((s = compute_alpha(g, st)) != HJ_OK) return s;
    const double dt = cfl_dt(g);
    double t = t0;
    const void *prev = V0;
    g->last_steps = 0;
    for (int k = 0; k < ntimes; ++k) {
        void *out = (char *)V_outs + bytes * size_t(k);
        HJ_HIP(hipMemcpyAsync(out, prev, bytes, hipMemcpyDeviceToDevice, st), "copy V");
        std::vector<double> hs;
        schedule(dt, t, times[k], &hs);  // the interval's own loop
        g->last_steps += int64_t(hs.size());
        if (g->prec == HJ_FP64)
            s = run_steps<double>(g, out, V0, mode, hs, st);
        else
            s = run_steps<float>(g, out, V0, mode, hs, st);
        if (s != HJ_OK) return s;
        t = times[k];
        prev = out;
    }
    return check_result(g, V_outs, size_t(g->total) * size_t(ntimes), g->prec == HJ_FP64, st);
}

hj_status hj_solve_mixed(hj_grid_t g, const double *V0, double *V_out, double t0, double tf,
                         hj_mode mode, double band, void *hip_stream)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (g->prec != HJ_FP32) return fail(HJ_E_ARG, "hj_solve_mixed needs an HJ_FP32 grid");
    if (!V0 || !V_out) return fail(HJ_E_ARG, "V0 and V_out must be non-NULL");
    if (mode != HJ_SET && mode != HJ_TUBE && mode != HJ_TUBE_VI)
        return fail(HJ_E_ARG, "hj_solve_mixed takes HJ_SET, HJ_TUBE or HJ_TUBE_VI");
    if (!(std::isfinite(t0) && std::isfinite(tf) && tf >= t0))
        return fail(HJ_E_ARG, "need finite t0 <= tf");
    const size_t b64 = size_t(g->total) * sizeof(double);
    if (overlap(V0, V_out, b64)) return fail(HJ_E_ARG, "V_out overlaps V0");
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = use_device(g)) != HJ_OK) return s;
    if (!g->mixV && (s = dev_alloc(&g->mixV, g->bytes(), "mixed V")) != HJ_OK) return s;
    if (!g->mixV0 && (s = dev_alloc(&g->mixV0, g->bytes(), "mixed V0")) != HJ_OK) return s;
    hipError_t e = launch_round_to_f32(V0, (float *)g->mixV0, uint32_t(g->total), st);
    if (e != hipSuccess) return hip_fail(e, "round to fp32");
    const int check = g->check;
    g->check = 0;  // the FP64 result is checked below, not the FP32 working array
    s = hj_solve(g, g->mixV0, g->mixV, t0, tf, mode, hip_stream);
    g->check = check;
    if (s != HJ_OK) return s;
    if ((s = hj_tube_finish(g, (const float *)g->mixV, V0, V_out, mode, band, hip_stream)) !=
        HJ_OK)
        return s;
    return check_result(g, V_out, size_t(g->total), true, st);
}

hj_status hj_tube_finish(hj_grid_t g, const float *V32, const double *V0, double *V_out,
                         hj_mode mode, double band, void *hip_stream)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (g->prec != HJ_FP32) return fail(HJ_E_ARG, "hj_tube_finish needs an HJ_FP32 grid");
    if (!V32 || !V0 || !V_out) return fail(HJ_E_ARG, "V32, V0 and V_out must be non-NULL");
    if (mode != HJ_SET && mode != HJ_TUBE && mode != HJ_TUBE_VI)
        return fail(HJ_E_ARG, "hj_tube_finish takes HJ_SET, HJ_TUBE or HJ_TUBE_VI");
    if (!(band == band)) return fail(HJ_E_ARG, "band is NaN");
    const size_t b64 = size_t(g->total) * sizeof(double);
    if (overlap(V_out, b64, V32, g->bytes()) || overlap(V_out, b64, V0, b64))
        return fail(HJ_E_ARG, "V_out overlaps V32 or V0");
    if (band < 0.0) {
        double m = 0.0;
        for (int d = 0; d < g->nd; ++d) m = g->dx[d] > m ? g->dx[d] : m;
        band = 3.0 * m;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = use_device(g)) != HJ_OK) return s;
    hipError_t e = launch_finalize_f64(V32, V0, V_out, uint32_t(g->total), band,
                                       mode == HJ_TUBE ? 1 : 0, st);
    if (e != hipSuccess) return hip_fail(e, "fp64 finalize");
    return HJ_OK;
}

hj_status hj_step(hj_grid_t g, void *V, const void *V0, double *t, double tf, hj_mode mode,
                  double *dt_used, void *hip_stream)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (!V || !t) return fail(HJ_E_ARG, "V and t must be non-NULL");
    if (mode != HJ_SET && mode != HJ_TUBE && mode != HJ_TUBE_VI)
        return fail(HJ_E_ARG, "hj_step takes HJ_SET, HJ_TUBE or HJ_TUBE_VI");
    if (mode == HJ_TUBE && !V0) return fail(HJ_E_ARG, "tube mode needs V0");
    if (!(std::isfinite(*t) && std::isfinite(tf))) return fail(HJ_E_ARG, "non-finite time");
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = use_device(g)) != HJ_OK) return s;
    if ((s = ensure_buffers(g, g->order == 3)) != HJ_OK) return s;
    if (!g->alpha_valid && (s = compute_alpha(g, st)) != HJ_OK) return s;
    const double dt = cfl_dt(g);
    if (!(tf > *t)) {
        if (dt_used) *dt_used = 0.0;
        return HJ_OK;
    }
    const double h = dt < tf - *t ? dt : tf - *t;
    if (g->prec == HJ_FP64)
        s = rk_step<double>(g, V, V0, step_kind(mode), h, st);
    else
        s = rk_step<float>(g, V, V0, step_kind(mode), h, st);
    if (s != HJ_OK) return s;
    *t = *t + h;
    if (dt_used) *dt_used = h;
    return HJ_OK;
}

hj_status hj_rhs(hj_grid_t g, const void *V, void *L_out, void *hip_stream)
{
    hj_status s = check_ready(g);
    if (s != HJ_OK) return s;
    if (!V || !L_out) return fail(HJ_E_ARG, "V and L_out must be non-NULL");
    if (overlap(V, L_out, g->bytes())) return fail(HJ_E_ARG, "L_out overlaps V");
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = use_device(g)) != HJ_OK) return s;
    if (!g->alpha_valid && (s = compute_alpha(g, st)) != HJ_OK) return s;
    if (g->prec == HJ_FP64)
        return stage<double>(g, V, nullptr, nullptr, L_out, kRhs, 0, 0, 0, 1, false, false, st);
    return stage<float>(g, V, nullptr, nullptr, L_out, kRhs, 0, 0, 0, 1, false, false, st);
}

hj_status hj_grid_set_workspace(hj_grid_t g, void *A, void *B)
{
    if (!g) return fail(HJ_E_ARG, "null grid handle");
    if (!A || !B) return fail(HJ_E_ARG, "workspace buffers must be non-NULL");
    if (overlap(A, B, g->bytes())) return fail(HJ_E_ARG, "workspace buffers overlap");
    if ((hj_status)use_device(g) != HJ_OK) return HJ_E_DEVICE;
    if (g->own_bufs) {
        if (g->bufA) (void)hipFree(g->bufA);
        if (g->bufB) (void)hipFree(g->bufB);
    }
    g->bufA = A;
    g->bufB = B;
    g->own_bufs = false;
    return HJ_OK;
}

hj_status hj_grid_destroy(hj_grid_t g)
{
    if (!g) return HJ_OK;
    (void)hipSetDevice(g->device);
    if (g->tab64) (void)hipFree(g->tab64);
    if (g->tab32) (void)hipFree(g->tab32);
    if (g->own_bufs && g->bufA) (void)hipFree(g->bufA);
    if (g->own_bufs && g->bufB) (void)hipFree(g->bufB);
    if (g->mixV) (void)hipFree(g->mixV);
    if (g->box_dev) (void)hipFree(g->box_dev);
    if (g->box_part) (void)hipFree(g->box_part);
    if (g->mixV0) (void)hipFree(g->mixV0);
    if (g->partial) (void)hipFree(g->partial);
    if (g->alpha_dev) (void)hipFree(g->alpha_dev);
    if (g->alpha_host) (void)hipHostFree(g->alpha_host);
    if (g->check_dev) (void)hipFree(g->check_dev);
    if (g->check_host) (void)hipHostFree(g->check_host);
    delete g;
    return HJ_OK;
}

}  // extern "C"
