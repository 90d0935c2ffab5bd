// nufft_forward_noalloc: the forward NUFFT with its two FFT ping-pong grids
// in a file-scope device array instead of the plan's workspaces, for callers
// that cannot allocate device memory at the point of the call.
//
// `scratch` is a host-side stand-in in host code: its device address is
// looked up once per device with hipGetSymbolAddress (each device holds its
// own copy at its own address) and only that address is handed to kernels.
// Every call on one device shares that device's array; nothing in it has to
// start at zero (each FFT pass writes every row that a later step reads), and
// calls that overlap on one device race.
#include <mutex>

#include "kp_internal.h"

namespace kp {

constexpr size_t kNoallocGridBytes = (size_t)16 << 20;  // per ping-pong grid
constexpr int kNoallocMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[2 * kNoallocGridBytes];

static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[kNoallocMaxDevices] = {};

// device address of this device's `scratch`
static unsigned char* noalloc_scratch() {
    int dev = 0;
    KP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) fail(KP_ERR_UNSUPPORTED, "device index beyond the no-alloc table");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        KP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(KP_ERR_HIP, "hipGetSymbolAddress returned NULL for the no-alloc scratch");
        g_noalloc_ptr[dev] = p;
    }
    return static_cast<unsigned char*>(g_noalloc_ptr[dev]);
}

}  // namespace kp

using namespace kp;

extern "C" {

int nufft_forward_noalloc(kp_plan_t plan, const void* x, void* y, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        if (!x || !y) fail(KP_ERR_INVALID_ARG, "x or y is NULL");
        Plan& P = *plan->impl;
        require_plan_device(P);
        const size_t need = sizeof(float2) * (size_t)P.Gtot * (size_t)P.C;
        if (need > kNoallocGridBytes)
            fail(KP_ERR_UNSUPPORTED, "nufft_forward_noalloc: the oversampled grid needs " + std::to_string(need) +
                                         " bytes per FFT buffer, more than the static " +
                                         std::to_string(kNoallocGridBytes) + " (use nufft_forward)");
        unsigned char* base = noalloc_scratch();
        hipStream_t s = (hipStream_t)stream;
        P.stream = s;
        FwdOpts fo;
        fo.bufs[0] = reinterpret_cast<float2*>(base);
        fo.bufs[1] = reinterpret_cast<float2*>(base + kNoallocGridBytes);
        float2* grid = forward_to_grid(P, (const float2*)x, fo, s);
        InterpArgs ia{};
        ia.mode = IO_CALLER;
        ia.out = (float2*)y;
        interp(P, grid, ia, s);
    });
}

}  // extern "C"
