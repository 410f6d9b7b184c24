// hj_solve_noalloc: hj_solve for callers that cannot allocate device memory.
// The stage buffers live in a static device array of this file instead of
// the handle's (hipMalloc'd on first use); everything else is hj_solve.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hj_host.h"

using namespace hj;

namespace {

// Stage buffers A and B of hj_solve_noalloc: 128 MiB on each device the
// library runs on, held until the process ends.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// The array's device address, per device (the host-side name is not one).
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

hj_status scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(HJ_E_DEVICE, "device ordinal beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "static scratch address");
        if (!p) return fail(HJ_E_DEVICE, "static scratch address is NULL");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return HJ_OK;
}

}  // namespace

extern "C" hj_status hj_solve_noalloc(hj_grid_t g, const void *V0, void *V_out, double t0,
                                      double tf, hj_mode mode, void *hip_stream)
{
    hj_status s = solve_check(g, V0, V_out, t0, tf, mode);
    if (s != HJ_OK) return s;
    if (g->diss == HJ_DISS_GLF)
        return fail(HJ_E_UNSUPPORTED,
                    "hj_solve_noalloc takes HJ_DISS_LF or HJ_DISS_LLF (GLF keeps per-stage "
                    "reduction buffers)");
    const size_t need = g->bytes() * (g->order == 3 ? 2 : 1);
    if (need > kScratchBytes)
        return fail(HJ_E_ARG, "stage buffers of " + std::to_string(need) +
                                  " bytes exceed the static scratch of " +
                                  std::to_string(kScratchBytes) + " bytes");
    if ((s = use_device(g)) != HJ_OK) return s;
    void *base = nullptr;
    if ((s = scratch_address(g->device, &base)) != HJ_OK) return s;
    // B starts on a 256-byte boundary after A
    const size_t off_b = (g->bytes() + 255) & ~size_t(255);
    if (g->order == 3 && off_b + g->bytes() > kScratchBytes)
        return fail(HJ_E_ARG, "stage buffers exceed the static scratch");
    void *a = base;
    void *b = g->order == 3 ? (void *)((char *)base + off_b) : nullptr;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((s = solve_enqueue(g, V0, V_out, t0, tf, mode, a, b, st)) != HJ_OK) return s;
    return check_result(g, V_out, size_t(g->total), g->prec == HJ_FP64, st);
}
