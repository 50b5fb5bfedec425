// Device context and gate-bootstrapping entry points.
//
// A context keeps the cloud key resident on one GPU: the bootstrapping key
// converted once to the NTT domain (32.8 MB), the key-switching key laid out
// as 2 KB rows (50.3 MB), and the twiddle tables.  Gate batches run as two
// launches on the caller's stream: blind rotation (with the gate prologue and
// sample extraction fused in) and key switching.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fhe_internal.h"
#include "goldilocks.h"
#include "kernels.h"
#include "runtime.h"
#include "modq.h"

namespace fhe {

namespace {

constexpr int brv5h(int x) {
    return ((x & 1) << 4) | ((x & 2) << 2) | (x & 4) | ((x & 8) >> 2) | ((x & 16) >> 4);
}

}  // namespace

// The 2048-th root of unity psi with psi^32 = 8: then psi^32 and psi^64 are
// powers of two and the in-register transforms need shifts only.
uint64_t ntt_psi() {
    const uint64_t psi0 = gl::pow(7, (gl::P - 1) / 2048);  // 7 generates Z_p^*
    for (uint64_t u = 1; u < 2048; u += 2) {
        const uint64_t c = gl::pow(psi0, u);
        if (gl::pow(c, 32) == 8) return c;
    }
    return 0;
}

void make_twiddles(std::vector<uint64_t>& twf, std::vector<uint64_t>& twi) {
    const uint64_t psi = ntt_psi();
    const uint64_t ninv = gl::pow(kN, gl::P - 2);
    twf.assign(1024, 0);
    twi.assign(1024, 0);
    for (int q = 0; q < 32; ++q)
        for (int t = 0; t < 32; ++t)
            twf[q * 32 + t] = gl::pow(psi, (uint64_t)(t * (2 * brv5h(q) + 1)) % 2048);
    for (int r = 0; r < 32; ++r)
        for (int t = 0; t < 32; ++t) {
            const uint64_t e = (2048 - (uint64_t)(r * (2 * t + 1)) % 2048) % 2048;
            twi[r * 32 + t] = gl::canon(gl::mul(ninv, gl::pow(psi, e)));
        }
}

// Two-prime tables, int32 [prime][32][32] in Montgomery form: forward
// psi^(t(2 brv5(q)+1)) at [q][t], inverse psi^(-r(2j+1)) N^-1 at [r][j].
template <int I>
static void make_twiddles_q1(int32_t* twf, int32_t* twi) {
    using M = mq::Mod<I>;
    const uint64_t ninv = mq::powmod(kN, M::q - 2, M::q);
    for (int q = 0; q < 32; ++q)
        for (int t = 0; t < 32; ++t) {
            twf[q * 32 + t] = M::rform(M::psi_pow((int64_t)t * (2 * brv5h(q) + 1)));
            twi[q * 32 + t] = M::rform(M::psi_pow(-(int64_t)q * (2 * t + 1)) * ninv % M::q);
        }
}

void make_twiddles_q(std::vector<int32_t>& twf, std::vector<int32_t>& twi) {
    twf.assign(2048, 0);
    twi.assign(2048, 0);
    make_twiddles_q1<0>(twf.data(), twi.data());
    make_twiddles_q1<1>(twf.data() + 1024, twi.data() + 1024);
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    ok_ = hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
}

int hip_fail(hipError_t e, const char* what) {
    // HIP keeps a failed call's code as the thread's last error; the launch
    // checks read that word, so a refused allocation would otherwise be
    // reported again by the next successful launch
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return set_error(FHE_ENOMEM, "%s: out of device memory", what);
    return set_error(FHE_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_gfx950(int device) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return set_error(FHE_EDEVICE, "no HIP device %d", device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return set_error(FHE_EDEVICE, "cannot query HIP device %d", device);
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(FHE_EDEVICE, "device %d is %s; this library is built for gfx950", device,
                         prop.gcnArchName);
    return FHE_OK;
}

int ctx_reserve_big(fhe_ctx* ctx, size_t gates) {
    const size_t need = gates * (kN + 1);
    if (need <= ctx->big_cap) return FHE_OK;
    if (ctx->big) {
        hipError_t e = hipDeviceSynchronize();  // work in flight may still read the old buffer
        if (e != hipSuccess) return hip_fail(e, "scratch resize");
        (void)hipFree(ctx->big);
        ctx->big = nullptr;
        ctx->big_cap = 0;
    }
    size_t cap = need < (size_t)4096 * (kN + 1) ? (size_t)4096 * (kN + 1) : need;
    hipError_t e = hipMalloc((void**)&ctx->big, cap * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "scratch allocation");
    ctx->big_cap = cap;
    ctx->big_generation++;
    return FHE_OK;
}

static hipEvent_t take_event(fhe_ctx* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int take_code_error(fhe_ctx* ctx) {
    if (!ctx->err_host) return FHE_OK;
    const uint32_t v = __atomic_exchange_n(ctx->err_host, 0u, __ATOMIC_ACQ_REL);
    if (v == 0) return FHE_OK;
    return set_error(FHE_EINVAL, "an earlier batch on this context held gate code %u, not valid for its call "
                     "(its output is the all-zero sample)", v & 0xFFu);
}

int order_begin(fhe_ctx* ctx, hipStream_t s) {
    if (!ctx->order_pending || ctx->order_stream == s) return FHE_OK;
    hipError_t e = hipStreamWaitEvent(s, ctx->order, 0);
    return e == hipSuccess ? FHE_OK : hip_fail(e, "stream ordering");
}

int order_end(fhe_ctx* ctx, hipStream_t s, int rc) {
    if (rc) return rc;
    hipError_t e = hipEventRecord(ctx->order, s);
    if (e != hipSuccess) return hip_fail(e, "stream ordering");
    ctx->order_stream = s;
    ctx->order_pending = true;
    return FHE_OK;
}

int run_gate_batch(fhe_ctx* ctx, const dev::GateIO& io_in, size_t count, hipStream_t s) {
    if (count == 0) return FHE_OK;
    dev::GateIO io = io_in;
    io.err = ctx->err_dev;
    const size_t samples = io.pair_slots ? 2 * count : count;
    int rc = ctx_reserve_big(ctx, samples);
    if (rc) return rc;
    const dev::LaunchConfig cfg = launch_config_for(ctx, count);
    fhe_ctx::TimedLaunch tl{{nullptr, nullptr, nullptr}, count, cfg};
    if (ctx->timing) {
        for (auto& ev : tl.ev)
            if (!(ev = take_event(ctx))) return set_error(FHE_EDEVICE, "timing event creation failed");
        (void)hipEventRecord(tl.ev[0], s);
    }
    hipError_t e = dev::launch_blind_rotate(ctx->keys, io, ctx->big, (uint32_t)count, cfg, s);
    if (e != hipSuccess) return hip_fail(e, "blind rotation launch");
    if (ctx->timing) (void)hipEventRecord(tl.ev[1], s);
    e = dev::launch_key_switch(ctx->keys, io, ctx->big, (uint32_t)samples, s);
    if (e != hipSuccess) return hip_fail(e, "key switch launch");
    if (ctx->timing) {
        (void)hipEventRecord(tl.ev[2], s);
        ctx->timed.push_back(tl);
    }
    return FHE_OK;
}

// A batched entry point: earlier invalid codes reported, the call's work
// ordered after the context's last call on another stream.
int run_batch_call(fhe_ctx* ctx, const dev::GateIO& io, size_t count, hipStream_t s) {
    int rc = take_code_error(ctx);
    if (rc) return rc;
    rc = order_begin(ctx, s);
    if (rc) return rc;
    return order_end(ctx, s, run_gate_batch(ctx, io, count, s));
}

}  // namespace fhe

using namespace fhe;

extern "C" int fhe_ctx_create(const fhe_cloud_key* ck, int device, fhe_ctx** out) {
    if (!ck || !out) return set_error(FHE_EINVAL, "fhe_ctx_create: null argument");
    *out = nullptr;
    std::string why;
    if (!params_supported(ck->P, &why)) return set_error(FHE_EINVAL, "fhe_ctx_create: %s", why.c_str());
    int rc = check_gfx950(device);
    if (rc) return rc;
    DeviceGuard guard(device);
    if (!guard.ok()) return set_error(FHE_EDEVICE, "cannot select device %d", device);

    fhe_ctx* ctx = new (std::nothrow) fhe_ctx();
    if (!ctx) return set_error(FHE_ENOMEM, "fhe_ctx_create: out of host memory");
    ctx->device = device;
    ctx->P = ck->P;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            ctx->cu_count = prop.multiProcessorCount;
    }
    tune_defaults(ctx);

    std::vector<uint64_t> twf, twi;
    make_twiddles(twf, twi);
    std::vector<int32_t> twfq, twiq;
    make_twiddles_q(twfq, twiq);
    const size_t n = ck->P.n, N = ck->P.N;
    const size_t bk_words = n * 4 * 2 * N;
    const size_t bkd_words = n * 2 * 32 * 2 * 64;
    const size_t ksk_rows = N * kKsT * 3;

    // KS rows v = 1..3, each padded to 512 words.
    std::vector<uint32_t> ksk_dev(ksk_rows * kKskRowWords, 0u);
    for (size_t i = 0; i < N; ++i)
        for (size_t j = 0; j < kKsT; ++j)
            for (size_t v = 1; v < kKsBase; ++v)
                std::memcpy(&ksk_dev[((i * kKsT + j) * 3 + v - 1) * kKskRowWords],
                            &ck->ksk[((i * kKsT + j) * kKsBase + v) * (n + 1)], (n + 1) * sizeof(uint32_t));

    uint32_t* bk_tmp = nullptr;
    auto fail = [&](hipError_t e, const char* what) {
        int code = hip_fail(e, what);
        if (bk_tmp) (void)hipFree(bk_tmp);
        fhe_ctx_destroy(ctx);
        return code;
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) return fail(e, "stream");
    if ((e = hipEventCreateWithFlags(&ctx->order, hipEventDisableTiming)) != hipSuccess) return fail(e, "event");
    if ((e = hipHostMalloc((void**)&ctx->err_host, sizeof(uint32_t), hipHostMallocMapped)) != hipSuccess)
        return fail(e, "error word");
    *ctx->err_host = 0;
    if ((e = hipHostGetDevicePointer((void**)&ctx->err_dev, ctx->err_host, 0)) != hipSuccess)
        return fail(e, "error word");
    if ((rc = noalloc_scratch(device, &ctx->noalloc_scratch)) != FHE_OK) {
        fhe_ctx_destroy(ctx);
        return rc;
    }
    if ((e = hipMalloc((void**)&ctx->twf, 1024 * 8)) != hipSuccess) return fail(e, "twiddles");
    if ((e = hipMalloc((void**)&ctx->twi, 1024 * 8)) != hipSuccess) return fail(e, "twiddles");
    if ((e = hipMalloc((void**)&ctx->bkd, bkd_words * 8)) != hipSuccess) return fail(e, "bootstrapping key");
    if ((e = hipMalloc((void**)&ctx->bkq, bkd_words * 8)) != hipSuccess) return fail(e, "bootstrapping key");
    if ((e = hipMalloc((void**)&ctx->twfq, 2048 * 4)) != hipSuccess) return fail(e, "twiddles");
    if ((e = hipMalloc((void**)&ctx->twiq, 2048 * 4)) != hipSuccess) return fail(e, "twiddles");
    if ((e = hipMalloc((void**)&ctx->ksk, ksk_dev.size() * 4)) != hipSuccess) return fail(e, "key-switching key");
    if ((e = hipMalloc((void**)&ctx->zero_row, kKskRowWords * 4)) != hipSuccess) return fail(e, "zero row");
    if ((e = hipMalloc((void**)&bk_tmp, bk_words * 4)) != hipSuccess) return fail(e, "bootstrapping key staging");
    if ((e = hipMemcpy(ctx->twf, twf.data(), 1024 * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "upload");
    if ((e = hipMemcpy(ctx->twi, twi.data(), 1024 * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "upload");
    if ((e = hipMemcpy(ctx->twfq, twfq.data(), 2048 * 4, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "upload");
    if ((e = hipMemcpy(ctx->twiq, twiq.data(), 2048 * 4, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "upload");
    if ((e = hipMemcpy(ctx->ksk, ksk_dev.data(), ksk_dev.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "upload");
    if ((e = hipMemset(ctx->zero_row, 0, kKskRowWords * 4)) != hipSuccess) return fail(e, "upload");
    if ((e = hipMemcpy(bk_tmp, ck->bk.data(), bk_words * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "upload");
    if ((e = dev::launch_bk_prepare(bk_tmp, ctx->bkd, ctx->twf, (uint32_t)n, ctx->stream)) != hipSuccess)
        return fail(e, "bootstrapping key transform");
    if ((e = dev::launch_bk_prepare_q(bk_tmp, ctx->bkq, (const uint64_t*)ctx->twfq, (uint32_t)n, ctx->stream)) !=
        hipSuccess)
        return fail(e, "bootstrapping key transform");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return fail(e, "bootstrapping key transform");
    (void)hipFree(bk_tmp);
    bk_tmp = nullptr;

    ctx->keys.bkd = ctx->bkd;
    ctx->keys.ksk = ctx->ksk;
    ctx->keys.zero_row = ctx->zero_row;
    ctx->keys.twf = ctx->twf;
    ctx->keys.twi = ctx->twi;
    ctx->keys.bkq = ctx->bkq;
    ctx->keys.twfq = (const uint64_t*)ctx->twfq;
    ctx->keys.twiq = (const uint64_t*)ctx->twiq;
    *out = ctx;
    return FHE_OK;
}

extern "C" void fhe_ctx_destroy(fhe_ctx* ctx) {
    if (!ctx) return;
    {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        destroy_circuit_cache(ctx);
        for (auto& tl : ctx->timed)
            for (hipEvent_t ev : tl.ev) ctx->event_pool.push_back(ev);
        for (hipEvent_t ev : ctx->event_pool) (void)hipEventDestroy(ev);
        for (void* p : {(void*)ctx->bkd, (void*)ctx->ksk, (void*)ctx->zero_row, (void*)ctx->twf,
                        (void*)ctx->twi, (void*)ctx->big, (void*)ctx->bkq, (void*)ctx->twfq, (void*)ctx->twiq})
            if (p) (void)hipFree(p);
        if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
        if (ctx->order) (void)hipEventDestroy(ctx->order);
        if (ctx->err_host) (void)hipHostFree(ctx->err_host);
    }
    delete ctx;
}

extern "C" int fhe_bootstrap_gate_batch(fhe_ctx* ctx, const uint8_t* ops, const uint32_t* in0,
                                        const uint32_t* in1, uint32_t* out, size_t count, void* stream) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_batch: null context");
    if (count == 0) return FHE_OK;
    if (!ops || !in0 || !in1 || !out) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_batch: null buffer");
    if (count > (size_t)1 << 30) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_batch: count %zu too large", count);
    DeviceGuard guard(ctx->device);
    dev::GateIO io{};
    io.ops = ops;
    io.in0 = in0;
    io.in1 = in1;
    io.out = out;
    return run_batch_call(ctx, io, count, (hipStream_t)stream);
}

extern "C" int fhe_bootstrap_gate3_batch(fhe_ctx* ctx, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                                         const uint32_t* in2, uint32_t* out, size_t count, void* stream) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_bootstrap_gate3_batch: null context");
    if (count == 0) return FHE_OK;
    if (!ops || !in0 || !in1 || !in2 || !out) return set_error(FHE_EINVAL, "fhe_bootstrap_gate3_batch: null buffer");
    if (count > (size_t)1 << 30) return set_error(FHE_EINVAL, "fhe_bootstrap_gate3_batch: count %zu too large", count);
    DeviceGuard guard(ctx->device);
    dev::GateIO io{};
    io.ops = ops;
    io.in0 = in0;
    io.in1 = in1;
    io.in2 = in2;
    io.out = out;
    return run_batch_call(ctx, io, count, (hipStream_t)stream);
}

extern "C" int fhe_bootstrap_compound_batch(fhe_ctx* ctx, const uint8_t* ops0, const uint8_t* ops1,
                                            const uint32_t* in0, const uint32_t* in1, uint32_t* out0,
                                            uint32_t* out1, size_t count, void* stream) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_bootstrap_compound_batch: null context");
    if (count == 0) return FHE_OK;
    if (!ops0 || !ops1 || !in0 || !in1 || !out0 || !out1)
        return set_error(FHE_EINVAL, "fhe_bootstrap_compound_batch: null buffer");
    if (count > (size_t)1 << 29)
        return set_error(FHE_EINVAL, "fhe_bootstrap_compound_batch: count %zu too large", count);
    DeviceGuard guard(ctx->device);
    dev::GateIO io{};
    io.ops = ops0;
    io.ops1 = ops1;
    io.in0 = in0;
    io.in1 = in1;
    io.out = out0;
    io.out1 = out1;
    io.pair_slots = 1;
    return run_batch_call(ctx, io, count, (hipStream_t)stream);
}

extern "C" int fhe_ctx_check(fhe_ctx* ctx) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_ctx_check: null context");
    return take_code_error(ctx);
}

extern "C" int fhe_bootstrap_lut_batch(fhe_ctx* ctx, const uint32_t* tv, const uint32_t* in, uint32_t* out,
                                       size_t count, void* stream) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_bootstrap_lut_batch: null context");
    if (count == 0) return FHE_OK;
    if (!tv || !in || !out) return set_error(FHE_EINVAL, "fhe_bootstrap_lut_batch: null buffer");
    if (count > (size_t)1 << 30) return set_error(FHE_EINVAL, "fhe_bootstrap_lut_batch: count %zu too large", count);
    DeviceGuard guard(ctx->device);
    dev::GateIO io{};
    io.op_const = FHE_AND;  // (no combination: the sample itself is rotated)
    io.in0 = in;
    io.in1 = in;
    io.tv = tv;
    io.out = out;
    return run_batch_call(ctx, io, count, (hipStream_t)stream);
}

extern "C" int fhe_bootstrap_gate_plain(fhe_ctx* ctx, uint8_t op, const uint32_t* in0,
                                        const uint32_t* in1, uint32_t* out, void* stream) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_plain: null context");
    if (!in0 || !in1 || !out) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_plain: null buffer");
    if (op > FHE_ORYN) return set_error(FHE_EINVAL, "fhe_bootstrap_gate_plain: gate code %u", op);
    DeviceGuard guard(ctx->device);
    dev::GateIO io{};
    io.op_const = op;
    io.in0 = in0;
    io.in1 = in1;
    io.out = out;
    int rc = run_batch_call(ctx, io, 1, (hipStream_t)stream);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? FHE_OK : hip_fail(e, "fhe_bootstrap_gate_plain");
}

extern "C" int fhe_debug_valu_rate(int device, int op, double* lane_ops_per_s) {
    if (op < 0 || op > 5 || !lane_ops_per_s) return set_error(FHE_EINVAL, "fhe_debug_valu_rate: bad argument");
    int rc = check_gfx950(device);
    if (rc) return rc;
    DeviceGuard guard(device);
    const uint32_t blocks = 2048;  // eight waves per SIMD on 256 compute units
    const int iters = 2000;
    uint32_t* out = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    float best = 0;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // the first run warms up
        e = hipEventRecord(ev[0], nullptr);
        if (e == hipSuccess) e = dev::launch_valu_probe(op, out, blocks, iters, nullptr);
        if (e == hipSuccess) e = hipEventRecord(ev[1], nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (rep > 0 && (best == 0 || ms < best)) best = ms;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return hip_fail(e, "fhe_debug_valu_rate");
    *lane_ops_per_s = (double)blocks * 256 * iters * 64 / (best * 1e-3);
    return FHE_OK;
}

extern "C" int fhe_debug_cmux(int device, int arith, const uint32_t* bk_i, int32_t abar, uint32_t* acc) {
    if (!bk_i || !acc || abar < 0 || abar >= 2 * (int)kN || (arith != 0 && arith != 1))
        return set_error(FHE_EINVAL, "fhe_debug_cmux: bad argument");
    int rc = check_gfx950(device);
    if (rc) return rc;
    DeviceGuard guard(device);
    std::vector<uint64_t> twf, twi;
    if (arith == 0) {
        make_twiddles(twf, twi);
    } else {
        std::vector<int32_t> f, g;
        make_twiddles_q(f, g);
        twf.assign(1024, 0);
        twi.assign(1024, 0);
        std::memcpy(twf.data(), f.data(), 8192);
        std::memcpy(twi.data(), g.data(), 8192);
    }
    uint64_t *d_twf = nullptr, *d_twi = nullptr, *d_bkd = nullptr;
    uint32_t *d_bk = nullptr, *d_acc = nullptr;
    const size_t bk_words = 4 * 2 * kN, bkd_words = 2 * 32 * 2 * 64;
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    step(hipMalloc((void**)&d_twf, 8192));
    step(hipMalloc((void**)&d_twi, 8192));
    step(hipMalloc((void**)&d_bkd, bkd_words * 8));
    step(hipMalloc((void**)&d_bk, bk_words * 4));
    step(hipMalloc((void**)&d_acc, 2 * kN * 4));
    if (e == hipSuccess) {
        step(hipMemcpy(d_twf, twf.data(), 8192, hipMemcpyHostToDevice));
        step(hipMemcpy(d_twi, twi.data(), 8192, hipMemcpyHostToDevice));
        step(hipMemcpy(d_bk, bk_i, bk_words * 4, hipMemcpyHostToDevice));
        step(hipMemcpy(d_acc, acc, 2 * kN * 4, hipMemcpyHostToDevice));
    }
    if (e == hipSuccess)
        step(arith == 0 ? dev::launch_bk_prepare(d_bk, d_bkd, d_twf, 1, nullptr)
                        : dev::launch_bk_prepare_q(d_bk, d_bkd, d_twf, 1, nullptr));
    dev::DeviceKeys K{};
    if (arith == 0) {
        K.twf = d_twf;
        K.twi = d_twi;
    } else {
        K.twfq = d_twf;
        K.twiq = d_twi;
    }
    if (e == hipSuccess) step(dev::launch_debug_cmux(K, arith, d_bkd, abar, d_acc, nullptr));
    if (e == hipSuccess) step(hipDeviceSynchronize());
    if (e == hipSuccess) step(hipMemcpy(acc, d_acc, 2 * kN * 4, hipMemcpyDeviceToHost));
    for (void* p : {(void*)d_twf, (void*)d_twi, (void*)d_bkd, (void*)d_bk, (void*)d_acc})
        if (p) (void)hipFree(p);
    return e == hipSuccess ? FHE_OK : hip_fail(e, "fhe_debug_cmux");
}

extern "C" int fhe_ctx_set_timing(fhe_ctx* ctx, int enable) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_ctx_set_timing: null context");
    ctx->timing = enable != 0;
    return FHE_OK;
}

// Waits for every recorded launch pair, hands each one's figures to `sink`
// and recycles the events.
template <class Sink>
static int drain_timed(fhe_ctx* ctx, const char* name, Sink&& sink) {
    DeviceGuard guard(ctx->device);
    int rc = FHE_OK;
    for (auto& tl : ctx->timed) {
        hipError_t e = hipEventSynchronize(tl.ev[2]);
        float a = 0, b = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&a, tl.ev[0], tl.ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, tl.ev[1], tl.ev[2]);
        if (e != hipSuccess && rc == FHE_OK) rc = hip_fail(e, name);
        sink(tl, (double)a, (double)b);
        for (hipEvent_t ev : tl.ev) ctx->event_pool.push_back(ev);
    }
    ctx->timed.clear();
    return rc;
}

extern "C" int fhe_ctx_timing(fhe_ctx* ctx, double* br_ms, double* ks_ms, uint64_t* launches,
                              uint64_t* gates) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_ctx_timing: null context");
    double br = 0, ks = 0;
    uint64_t g = 0, n = 0;
    int rc = drain_timed(ctx, "fhe_ctx_timing", [&](const fhe_ctx::TimedLaunch& tl, double a, double b) {
        br += a;
        ks += b;
        g += tl.gates;
        ++n;
    });
    if (br_ms) *br_ms = br;
    if (ks_ms) *ks_ms = ks;
    if (launches) *launches = n;
    if (gates) *gates = g;
    return rc;
}

extern "C" int fhe_ctx_timing_launches(fhe_ctx* ctx, fhe_launch_record* out, size_t max, size_t* count) {
    if (!ctx || !count || (max && !out)) return set_error(FHE_EINVAL, "fhe_ctx_timing_launches: null argument");
    size_t n = 0;
    int rc = drain_timed(ctx, "fhe_ctx_timing_launches", [&](const fhe_ctx::TimedLaunch& tl, double a, double b) {
        if (n < max)
            out[n] = fhe_launch_record{tl.gates, tl.cfg.waves_per_gate, tl.cfg.gates_per_group, tl.cfg.arith, 0, a, b};
        ++n;
    });
    *count = n;
    return rc;
}

extern "C" int fhe_ctx_set_graphs(fhe_ctx* ctx, int enable) {
    if (!ctx) return set_error(FHE_EINVAL, "fhe_ctx_set_graphs: null context");
    ctx->use_graphs = enable != 0;
    return FHE_OK;
}
