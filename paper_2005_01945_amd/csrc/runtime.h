// Context state and helpers shared by the runtime, circuit and serving sources.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "fhe_internal.h"
#include "kernels.h"

namespace fhe {
struct CircuitCache;
// Launch-shape table: bucket b holds the blind-rotation shape of batches of
// width w with 2^(b-1) < w <= 2^b; the last bucket also holds every wider one.
constexpr int kTuneBuckets = 16;
}

struct fhe_ctx {
    int device = 0;
    fhe_params P{};
    hipStream_t stream = nullptr;  // internal stream (key preparation)
    uint64_t* bkd = nullptr;
    uint32_t* ksk = nullptr;
    uint32_t* zero_row = nullptr;
    uint64_t* twf = nullptr;
    uint64_t* twi = nullptr;
    uint64_t* bkq = nullptr;   // BK for the two-prime NTT
    int32_t* twfq = nullptr;   // two-prime twiddle tables [2][1024]
    int32_t* twiq = nullptr;
    uint32_t* big = nullptr;  // extracted samples of the gates in flight, [gates][N+1]
    size_t big_cap = 0;       // words
    uint64_t big_generation = 0;  // bumped on every reallocation of big (captured graphs hold it)
    bool use_graphs = true;       // replay circuit level schedules as captured HIP graphs
    int cu_count = 256;
    fhe::dev::LaunchConfig tune[fhe::kTuneBuckets]{};  // launch shape per width bucket
    uint64_t tune_generation = 0;  // bumped on every change of `tune` (captured graphs hold it)
    fhe::dev::DeviceKeys keys{};
    fhe::CircuitCache* circuits = nullptr;
    // per-phase timing: events {before BR, after BR, after KS} per launch pair
    bool timing = false;
    struct TimedLaunch {
        hipEvent_t ev[3];
        uint64_t gates;
        fhe::dev::LaunchConfig cfg;
    };
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    // Calls on different streams share the scratch buffer and the circuit
    // pools: each call records `order` on its stream, and a call on another
    // stream first waits for it.
    hipEvent_t order = nullptr;
    hipStream_t order_stream = nullptr;
    bool order_pending = false;
    // Invalid gate codes met by a kernel (0 = none), pinned host memory the
    // kernels write through err_dev.
    uint32_t* err_host = nullptr;
    uint32_t* err_dev = nullptr;
    // This device's fixed scratch array of the allocation-free entry point
    // (noalloc.cpp), resolved when the context is created.
    uint32_t* noalloc_scratch = nullptr;
};

namespace fhe {

// Makes `dev` current for the lifetime of the guard, restoring the caller's.
class DeviceGuard {
  public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    bool ok() const { return ok_; }

  private:
    int prev_ = -1;
    bool ok_ = false;
};

int hip_fail(hipError_t e, const char* what);
int check_gfx950(int device);
uint64_t ntt_psi();
void make_twiddles(std::vector<uint64_t>& twf, std::vector<uint64_t>& twi);
void make_twiddles_q(std::vector<int32_t>& twf, std::vector<int32_t>& twi);
int ctx_reserve_big(fhe_ctx* ctx, size_t gates);
// Launch-shape table (tuner.cpp).
int tune_bucket(size_t width);
void tune_defaults(fhe_ctx* ctx);
dev::LaunchConfig launch_config_for(const fhe_ctx* ctx, size_t width);
// Enqueues blind rotation + key switching of `count` gates on stream s
// (io.pair_slots: two extracted samples per gate).
int run_gate_batch(fhe_ctx* ctx, const dev::GateIO& io, size_t count, hipStream_t s);
// Cross-stream ordering of a call's work (not used inside graph capture):
// order_begin makes s wait for the context's last call on another stream,
// order_end records the call's completion on s.
int order_begin(fhe_ctx* ctx, hipStream_t s);
int order_end(fhe_ctx* ctx, hipStream_t s, int rc);
// Device address of this device's fixed scratch array (noalloc.cpp); the
// device must be current.
int noalloc_scratch(int device, uint32_t** out);
// FHE_EINVAL (and clears the word) when a kernel met an invalid gate code.
int take_code_error(fhe_ctx* ctx);
// run_gate_batch for an entry point: reports earlier invalid codes, orders
// the work after the context's last call on another stream.
int run_batch_call(fhe_ctx* ctx, const dev::GateIO& io, size_t count, hipStream_t s);
void destroy_circuit_cache(fhe_ctx* ctx);

}  // namespace fhe
