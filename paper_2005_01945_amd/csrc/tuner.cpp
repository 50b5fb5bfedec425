// Launch-shape table and autotuner of the blind-rotation kernel.
//
// A circuit level is one batch of independent gates; its width decides how
// the gates should be laid onto the chip.  Wide batches want one wavefront
// per gate and two waves per SIMD (issued work per gate is what counts);
// batches narrower than the chip want each gate's CMux chain split over two
// wavefronts (latency per gate is what counts).  The tuner measures every
// shape at widths 1, 2, 4, ... and keeps the fastest per width bucket.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include "fhe.h"
#include "fhe_internal.h"
#include "runtime.h"

namespace fhe {

namespace {

constexpr dev::LaunchConfig kShapes[] = {{1, 1, 0}, {1, 2, 0}, {1, 4, 0}, {1, 8, 0}, {2, 1, 0},
                                         {1, 1, 1}, {1, 2, 1}, {1, 4, 1}, {1, 8, 1}, {2, 1, 1}, {4, 1, 1}};

bool same(const dev::LaunchConfig& a, const dev::LaunchConfig& b) {
    return a.waves_per_gate == b.waves_per_gate && a.gates_per_group == b.gates_per_group && a.arith == b.arith;
}

bool shape_valid(const fhe_launch_config& c) {
    if (c.arith > 1) return false;
    if (c.waves_per_gate == 1)
        return c.gates_per_group == 1 || c.gates_per_group == 2 || c.gates_per_group == 4 || c.gates_per_group == 8;
    if (c.waves_per_gate == 4) return c.gates_per_group == 1 && c.arith == 1;
    return c.waves_per_gate == 2 && c.gates_per_group == 1;
}

}  // namespace

int tune_bucket(size_t width) {
    int b = 0;
    while (b < kTuneBuckets - 1 && ((size_t)1 << b) < width) ++b;
    return b;
}

// Before any measurement (defaults from measurements on MI355X): two-prime
// arithmetic everywhere; four waves per gate up to one gate per CU, two
// waves per gate up to two; one wave per SIMD with the full register file
// (four gates per workgroup, one 81 KB workgroup per CU) up to four gates
// per CU; eight gates per workgroup (two waves per SIMD) beyond.
static dev::LaunchConfig default_shape(const fhe_ctx* ctx, size_t width) {
    const size_t cus = (size_t)ctx->cu_count;
    if (width <= cus) return dev::LaunchConfig{4, 1, 1};
    if (width <= 2 * cus) return dev::LaunchConfig{2, 1, 1};
    if (width <= 4 * cus) return dev::LaunchConfig{1, 4, 1};
    return dev::LaunchConfig{1, 8, 1};
}

void tune_defaults(fhe_ctx* ctx) {
    for (int b = 0; b < kTuneBuckets; ++b) ctx->tune[b] = default_shape(ctx, (size_t)1 << b);
    ctx->tune_generation++;
}

dev::LaunchConfig launch_config_for(const fhe_ctx* ctx, size_t width) {
    return ctx->tune[tune_bucket(width)];
}

}  // namespace fhe

using namespace fhe;

extern "C" int fhe_ctx_launch_config(const fhe_ctx* ctx, uint32_t width, fhe_launch_config* out) {
    if (!ctx || !out) return set_error(FHE_EINVAL, "fhe_ctx_launch_config: null argument");
    if (width == 0) return set_error(FHE_EINVAL, "fhe_ctx_launch_config: width 0");
    const dev::LaunchConfig c = launch_config_for(ctx, width);
    out->waves_per_gate = c.waves_per_gate;
    out->gates_per_group = c.gates_per_group;
    out->arith = c.arith;
    return FHE_OK;
}

extern "C" int fhe_ctx_set_launch_config(fhe_ctx* ctx, uint32_t min_width, uint32_t max_width,
                                         const fhe_launch_config* cfg) {
    if (!ctx || !cfg) return set_error(FHE_EINVAL, "fhe_ctx_set_launch_config: null argument");
    if (min_width == 0 || min_width > max_width)
        return set_error(FHE_EINVAL, "fhe_ctx_set_launch_config: empty width range [%u, %u]", min_width, max_width);
    if (!shape_valid(*cfg))
        return set_error(FHE_EINVAL,
                         "fhe_ctx_set_launch_config: unsupported shape (%u waves per gate, %u gates per group, arith %u)",
                         cfg->waves_per_gate, cfg->gates_per_group, cfg->arith);
    for (int b = tune_bucket(min_width); b <= tune_bucket(max_width); ++b)
        ctx->tune[b] = dev::LaunchConfig{cfg->waves_per_gate, cfg->gates_per_group, cfg->arith};
    ctx->tune_generation++;
    return FHE_OK;
}

extern "C" int fhe_ctx_autotune(fhe_ctx* ctx, uint32_t max_width, uint32_t reps) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_ctx_autotune: null context");
    if (max_width == 0 || reps == 0) return set_error(FHE_EINVAL, "fhe_ctx_autotune: max_width and reps must be > 0");
    const int top = tune_bucket(max_width);
    const size_t widest = (size_t)1 << top;
    DeviceGuard guard(ctx->device);
    // work of earlier calls on any stream may still use the scratch buffer
    hipError_t e0 = hipDeviceSynchronize();
    if (e0 != hipSuccess) return hip_fail(e0, "fhe_ctx_autotune");
    int rc = ctx_reserve_big(ctx, widest);
    if (rc) return rc;
    // Synthetic batch: all-zero input samples (any words are valid input).
    uint32_t *in = nullptr, *out = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc((void**)&in, widest * kLweW * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&out, widest * kLweW * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemsetAsync(in, 0, widest * kLweW * sizeof(uint32_t), ctx->stream);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    dev::GateIO io{};
    io.op_const = FHE_NAND;
    io.in0 = in;
    io.in1 = in;
    io.out = out;
    dev::LaunchConfig best_cfg[kTuneBuckets];
    for (int b = 0; b <= top && e == hipSuccess; ++b) {
        const uint32_t width = 1u << b;
        // The default shape is timed first and kept unless another one is
        // more than 2% faster, so near-ties do not flip from run to run.
        const dev::LaunchConfig incumbent = default_shape(ctx, width);
        dev::LaunchConfig order[1 + sizeof(kShapes) / sizeof(kShapes[0])];
        int n_order = 0;
        order[n_order++] = incumbent;
        for (const dev::LaunchConfig& c : kShapes)
            if (!same(c, incumbent)) order[n_order++] = c;
        float best = 0;
        for (int k = 0; k < n_order; ++k) {
            const dev::LaunchConfig& cfg = order[k];
            float fastest = 0;
            for (uint32_t r = 0; r <= reps && e == hipSuccess; ++r) {  // run 0 warms up
                e = hipEventRecord(ev[0], ctx->stream);
                if (e == hipSuccess) e = dev::launch_blind_rotate(ctx->keys, io, ctx->big, width, cfg, ctx->stream);
                if (e == hipSuccess) e = dev::launch_key_switch(ctx->keys, io, ctx->big, width, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (r > 0 && (fastest == 0 || ms < fastest)) fastest = ms;
            }
            if (e == hipSuccess && (best == 0 || fastest < 0.98f * best)) {
                best = fastest;
                best_cfg[b] = cfg;
            }
        }
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : {(void*)in, (void*)out})
        if (p) (void)hipFree(p);
    if (e != hipSuccess) return hip_fail(e, "fhe_ctx_autotune");
    for (int b = 0; b < kTuneBuckets; ++b) ctx->tune[b] = best_cfg[b <= top ? b : top];
    ctx->tune_generation++;
    return FHE_OK;
}
