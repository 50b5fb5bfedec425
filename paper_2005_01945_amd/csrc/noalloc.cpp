// A gate-batch entry point that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The batched gate call needs scratch memory for the extracted N-dimensional
// samples between the blind rotation and the key switching (N + 1 words per
// gate).  Here that scratch is a fixed device array of this translation unit,
// one copy per GPU, resolved to its device address once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fhe_internal.h"
#include "kernels.h"
#include "runtime.h"

namespace fhe {

constexpr size_t kNoAllocMaxGates = 4096;

// Extracted samples of up to kNoAllocMaxGates gates (16.8 MB per GPU).  In
// host code this name is not a device address: only the pointer resolved by
// hipGetSymbolAddress below is passed to kernels.
static __device__ __align__(256) uint32_t scratch[kNoAllocMaxGates * (kN + 1)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mutex;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Resolves this device's copy of `scratch` (the device must be current);
// once per device, later calls return the kept pointer.
int noalloc_scratch(int device, uint32_t** out) {
    if (device < 0 || device >= kMaxDevices) return set_error(FHE_EDEVICE, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
        g_scratch_ptr[device] = static_cast<uint32_t*>(p);
    }
    *out = g_scratch_ptr[device];
    return FHE_OK;
}

}  // namespace fhe

using namespace fhe;

extern "C" int fhe_bootstrap_gate_batch_noalloc(fhe_ctx* ctx, const uint8_t* ops, const uint32_t* in0,
                                                const uint32_t* in1, uint32_t* out, size_t count, void* stream) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_batch_noalloc: null context");
    if (count > kNoAllocMaxGates)
        return set_error(FHE_EINVAL, "fhe_bootstrap_gate_batch_noalloc: %zu gates exceed the fixed scratch of %zu",
                         count, kNoAllocMaxGates);
    if (count == 0) return FHE_OK;
    if (!ops || !in0 || !in1 || !out) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_batch_noalloc: null buffer");
    if (!ctx->noalloc_scratch) return set_error(FHE_EDEVICE, "fhe_bootstrap_gate_batch_noalloc: no scratch");
    DeviceGuard guard(ctx->device);
    int rc = take_code_error(ctx);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)stream;
    // Under capture the caller orders its own work (an event recorded outside
    // the capture cannot be waited on inside it).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "fhe_bootstrap_gate_batch_noalloc");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (!capturing && (rc = order_begin(ctx, s))) return rc;
    dev::GateIO io{};
    io.ops = ops;
    io.in0 = in0;
    io.in1 = in1;
    io.out = out;
    io.err = ctx->err_dev;
    const dev::LaunchConfig cfg = launch_config_for(ctx, count);
    e = dev::launch_blind_rotate(ctx->keys, io, ctx->noalloc_scratch, (uint32_t)count, cfg, s);
    if (e == hipSuccess) e = dev::launch_key_switch(ctx->keys, io, ctx->noalloc_scratch, (uint32_t)count, s);
    rc = e == hipSuccess ? FHE_OK : hip_fail(e, "fhe_bootstrap_gate_batch_noalloc");
    return capturing ? rc : order_end(ctx, s, rc);
}
