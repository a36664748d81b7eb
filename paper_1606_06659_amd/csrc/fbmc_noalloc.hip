// fbmc_noalloc.hip -- the allocation-free form of the network's loss and
// gradients (fb_mlp_loss_grad_noalloc), for callers that cannot allocate.
//
// Its intermediate buffers live in one file-scope device array, `scratch`.  In
// host code that name is only a host-side stand-in: the device address of each
// GPU's copy is looked up once per device with hipGetSymbolAddress and kept in
// g_scratch[device]; only that pointer is ever passed to a kernel.
#include "libfbmc.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "fbmc_mlp.hpp"

namespace fbmc {
void set_thread_error(const char *msg);   // fbmc_host.cpp

namespace {

// Floats of scratch per row: X [F], Z1, H1, Z2, H2, dH, dZ2, dZ1 [H],
// O, dO [O], the row's loss.
constexpr int64_t kRowFloats = kMlpF + 7 * kMlpH + 2 * kMlpO + 1;
constexpr int64_t kRows = FB_NOALLOC_MAX_ROWS;
static_assert(FB_MLP_PARAMS == kMlpParams, "FB_MLP_PARAMS must match the master layout");
static_assert((kRows * 4) % 256 == 0, "every region starts 256-byte aligned");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float *g_scratch[kMaxDevices];   // device address of `scratch` per device, once looked up

}  // namespace

static __device__ __align__(256) float scratch[kRows * kRowFloats];

namespace {

int fail_noalloc(int code, const char *msg)
{
    set_thread_error(msg);
    return code;
}

// The current device's copy of `scratch`, looked up on the first call on that
// device (with it current).
hipError_t scratch_ptr(float **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = (float *)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace fbmc

using namespace fbmc;

extern "C" int fb_mlp_loss_grad_noalloc(const float *master, int32_t L, const float *phi, const float *target,
                                        int64_t B, float *loss, float *grad, void *stream)
{
    char msg[160];
    if (!master || !phi || !target || !loss || !grad)
        return fail_noalloc(FB_EINVAL, "fb_mlp_loss_grad_noalloc: a buffer pointer is NULL");
    // the weight blocks are read as float4 rows
    if (reinterpret_cast<uintptr_t>(master) % 16 != 0)
        return fail_noalloc(FB_EINVAL, "fb_mlp_loss_grad_noalloc: master is not 16-byte aligned");
    if (L < 1 || L > FB_MAX_L) {
        std::snprintf(msg, sizeof msg, "fb_mlp_loss_grad_noalloc: L = %d outside 1..%d", (int)L, FB_MAX_L);
        return fail_noalloc(FB_EINVAL, msg);
    }
    if (B < 32 || B % 32 != 0) {
        std::snprintf(msg, sizeof msg, "fb_mlp_loss_grad_noalloc: B = %lld is not a positive multiple of 32",
                      (long long)B);
        return fail_noalloc(FB_EINVAL, msg);
    }
    if (B > kRows) {
        std::snprintf(msg, sizeof msg,
                      "fb_mlp_loss_grad_noalloc: B = %lld exceeds the static scratch of %d rows "
                      "(FB_NOALLOC_MAX_ROWS); split the batch",
                      (long long)B, FB_NOALLOC_MAX_ROWS);
        return fail_noalloc(FB_EINVAL, msg);
    }
    float *s = nullptr;
    hipError_t e = scratch_ptr(&s);
    if (e != hipSuccess) {
        std::snprintf(msg, sizeof msg, "fb_mlp_loss_grad_noalloc: scratch lookup: %s", hipGetErrorString(e));
        return fail_noalloc(FB_EDEVICE, msg);
    }
    // regions of kRows rows each, at fixed offsets
    TrainBufs t;
    float *q = s;
    auto take = [&](int64_t width) {
        float *p = q;
        q += kRows * width;
        return p;
    };
    t.X = take(kMlpF);
    t.Z1 = take(kMlpH);
    t.H1 = take(kMlpH);
    t.Z2 = take(kMlpH);
    t.H2 = take(kMlpH);
    t.dH = take(kMlpH);
    t.dZ2 = take(kMlpH);
    t.dZ1 = take(kMlpH);
    t.O = take(kMlpO);
    t.dO = take(kMlpO);
    t.loss = take(1);
    t.Tg = const_cast<float *>(target);
    t.grad = grad;
    t.B = (int)B;
    const hipStream_t st = (hipStream_t)stream;
    const int64_t nx = B * kMlpF;
    hipLaunchKernelGGL(standardise_rows, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, phi, master, t.X, B);
    e = hipGetLastError();
    if (e == hipSuccess) e = mlp_forward_backward(master, t, L, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(mean_rows, dim3(1), dim3(256), 0, st, t.loss, B, loss);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        std::snprintf(msg, sizeof msg, "fb_mlp_loss_grad_noalloc: %s", hipGetErrorString(e));
        return fail_noalloc(FB_EDEVICE, msg);
    }
    return FB_OK;
}
