// Entry point without allocation: the batched ELBO + gradient whose per-item partial sums
// and work-queue counter live in a file-scope device array instead of plan memory, for
// callers that cannot allocate at the time of the call.
//
// The array below is a device symbol: its name, used in host code, is a host-side stand-in
// and not a device address.  Its address on each device is looked up once, with that
// device current (plan creation is the set-up call), and only that address is passed to
// kernels.  Every call on one device shares that device's copy, which keeps the last
// call's contents; the kernels overwrite every entry they later read (each work item
// writes all of its partial sums; the queue counter is reset by a fill kernel before
// the fused adjoint), so nothing is cleared here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "celeste.h"
#include "internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = CELESTE_NOALLOC_SCRATCH_BYTES;
constexpr size_t COUNTER_BYTES = 256;   // the queue counter, padded so the partials stay aligned
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

std::mutex g_mu;
void* g_addr[MAX_DEVICES] = {};   // device address of `scratch` on each device, once looked up

}  // namespace

namespace cel {

int noalloc_attach(int device) {
    if (device < 0 || device >= MAX_DEVICES) return CELESTE_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_addr[device]) return CELESTE_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return CELESTE_EHIP;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CELESTE_EHIP;
    g_addr[device] = ptr;
    return CELESTE_OK;
}

}  // namespace cel

extern "C" int celeste_elbo_grad_noalloc(celeste_plan* p, const double* theta, const uint8_t* active,
                                         double* elbo, double* grad, hipStream_t st) {
    if (!p || !theta || !elbo || !grad) return CELESTE_EINVAL;
    const int64_t need = cel::plan_item_count(p) * cel::NACC * (int64_t)sizeof(double);
    if (need > (int64_t)(SCRATCH_BYTES - COUNTER_BYTES)) return CELESTE_ESCRATCH;
    const int dev = cel::plan_device(p);
    if (dev < 0 || dev >= MAX_DEVICES) return CELESTE_EINVAL;
    void* base;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        base = g_addr[dev];
    }
    if (!base) return CELESTE_EINVAL;   // the plan's creation looks the address up
    char* b = static_cast<char*>(base);
    return cel::batched_elbo_grad_scratch(p, theta, active, elbo, grad,
                                          reinterpret_cast<double*>(b + COUNTER_BYTES), reinterpret_cast<int*>(b),
                                          st);
}
