// Host-side internals of libhj shared by the single-solve and batch
// entry points (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hj.h"
#include "hj_internal.h"

struct hj_grid_s {
    int nd = 0;
    int64_t n[hj::kMaxDim] = {1, 1, 1, 1};
    double lo[hj::kMaxDim] = {0, 0, 0, 0}, hi[hj::kMaxDim] = {0, 0, 0, 0};
    double dx[hj::kMaxDim] = {1, 1, 1, 1};
    uint32_t pmask = 0;
    hj_precision prec = HJ_FP64;
    int64_t total = 0;
    uint32_t stride[hj::kMaxDim] = {0, 0, 0, 0};
    uint32_t tab_off[hj::kMaxDim] = {0, 0, 0, 0};
    int device = 0;
    bool addr64 = false;  // HJ_ADDR64 set when the grid was created (test switch)

    int dyn = -1;
    double prm[8] = {0, 0, 0, 0, 0, 0, 0, 0};

    int space = HJ_WENO5;
    int order = 3;
    double cfl = 0.8;
    int diss = HJ_DISS_LF;

    void *box_dev = nullptr;   // kGLF: the costate box of the current stage input
    void *box_part = nullptr;  // kGLF: its pass-1 partials

    double *tab64 = nullptr;   // device, FP64 tables (alpha and FP64 stages)
    float *tab32 = nullptr;    // device, FP32 tables (FP32 stages)
    void *bufA = nullptr;      // stage buffers
    void *bufB = nullptr;
    bool own_bufs = true;      // false after hj_grid_set_workspace
    void *mixV = nullptr;      // hj_solve_mixed: FP32 V0 and V
    void *mixV0 = nullptr;
    double *partial = nullptr; // alpha pass-1 partial maxima
    double *alpha_dev = nullptr;
    double *alpha_host = nullptr;  // pinned
    bool alpha_valid = false;
    double alpha[hj::kMaxDim] = {0, 0, 0, 0};
    int64_t last_steps = 0;    // RK steps of the last hj_solve / hj_solve_outputs
    int check = 0;             // HJ_CHECK_* flags (hj_set_check)
    int *check_dev = nullptr;  // device flag of the non-finite scan
    int *check_host = nullptr; // pinned read-back of it

    size_t elem() const { return prec == HJ_FP64 ? sizeof(double) : sizeof(float); }
    size_t bytes() const { return size_t(total) * elem(); }
};

namespace hj {

hj_status fail(hj_status s, const std::string &msg);
hj_status hip_fail(hipError_t e, const char *what);
hj_status dev_alloc(void **p, size_t bytes, const char *what);
hj_status use_device(hj_grid_t g);
hj_status ensure_buffers(hj_grid_t g, bool need_b);
hj_status check_ready(hj_grid_t g);
// Enqueue the alpha reduction and its read-back into pinned memory.
hj_status launch_alpha_readback(hj_grid_t g, hipStream_t s);
// After the stream has synchronised: take the read-back alpha.
void accept_alpha(hj_grid_t g);
hj_status compute_alpha(hj_grid_t g, hipStream_t s);
double cfl_dt(hj_grid_t g);
void schedule(double dt, double t0, double tf, std::vector<double> *hs);
extern const double kEpsT;
template <typename T>
StageArgs<T> base_args(hj_grid_t g);
// hj_solve's argument checks, and its body with given stage buffers
hj_status solve_check(hj_grid_t g, const void *V0, const void *V_out, double t0, double tf,
                      hj_mode mode);
// HJ_CHECK_FINITE: scan n values of V (grid precision, or FP64 when fp64) for
// NaN/Inf after the work on st, wait for it, HJ_E_NUMERIC if any
hj_status check_result(hj_grid_t g, const void *V, size_t n, bool fp64, hipStream_t st);
hj_status solve_enqueue(hj_grid_t g, const void *V0, void *V_out, double t0, double tf,
                        hj_mode mode, void *A, void *B, hipStream_t st);

}  // namespace hj

#define HJ_HIP(call, what)                                       \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hj::hip_fail(e_, (what));   \
    } while (0)
