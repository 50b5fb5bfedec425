// Serving runtime: continuous batching of gate and circuit jobs (every circuit
// of the circuit entry points) on one context.
//
// A worker thread owns the context while the server lives.  Each tick it
//  1. admits queued jobs, in arrival order, whose samples (inputs, every gate
//     output) fit the pool left under the HBM budget, and copies their inputs
//     into the pool;
//  2. gathers the next ASAP level of every running job into one descriptor
//     batch and runs it as one blind-rotation + key-switching launch pair
//     (jobs of different kinds and depths share the launch);
//  3. copies the outputs of jobs whose last level ran to the caller's buffer
//     and frees their pool samples.
// Every tick goes to one stream, so a tick's gates see the outputs of the
// previous ones and freed samples are reused only after their last reader.
// A job's progress does not depend on device results, so the worker builds
// and enqueues the next tick while earlier ones still run (up to kRing ticks
// in flight, each with its own descriptor buffers and completion event): the
// device is never idle between ticks.  A job is done when the event of its
// last tick has completed.  Jobs that arrive meanwhile join the next tick.  A
// gate's arithmetic does not depend on the other gates of its launch, so a
// job's result is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "circuit_ir.h"
#include "fhe_internal.h"
#include "runtime.h"

namespace fhe {
namespace {

using Clock = std::chrono::steady_clock;

// A circuit laid out for serving: local wire -> pool slot with the inputs
// first, then the outputs (contiguous, so one copy returns them), then the
// other gate outputs; gates grouped by ASAP level.
struct ServeShape {
    uint32_t na = 0, nb = 0, nout = 0, slots = 0;
    std::vector<uint8_t> op;                        // per gate
    std::vector<uint32_t> in0, in1, out;            // pool slots per gate
    std::vector<uint32_t> in2;                      // third input (kNoWire: none)
    bool three = false;                             // any three-input gate
    std::vector<std::vector<uint32_t>> levels;      // gate indices per level
};

ServeShape make_shape(int kind, uint32_t op, uint32_t w, uint32_t rows, uint32_t cols) {
    ServeShape S;
    if (kind == FHE_JOB_GATE) {
        S.na = S.nb = S.nout = 1;
        S.slots = 3;
        S.op = {(uint8_t)op};
        S.in0 = {0};
        S.in1 = {1};
        S.in2 = {kNoWire};
        S.out = {2};
        S.levels = {{0}};
        return S;
    }
    int ck = kMatvec;
    switch (kind) {
    case FHE_JOB_ADD: ck = kAdd; break;
    case FHE_JOB_MUL: ck = kMul; break;
    case FHE_JOB_MUL_TREE: ck = kMulTree; break;
    case FHE_JOB_ADD_FA: ck = kAddFa; break;
    case FHE_JOB_ADD_NUMBERWISE: ck = kAddNumberwise; break;
    case FHE_JOB_KARATSUBA: ck = kKaratsuba; break;
    case FHE_JOB_MATMUL: ck = kMatmul; break;
    default: break;
    }
    const Circuit c = build_circuit(ck, w, rows, cols);
    uint32_t depth = 0;
    const std::vector<uint32_t> glev = asap_levels(c, &depth);
    S.na = c.na;
    S.nb = c.nb;
    S.nout = (uint32_t)c.outputs.size();
    std::vector<uint32_t> slot(c.wires(), UINT32_MAX);
    for (uint32_t k = 0; k < c.na + c.nb; ++k) slot[k] = k;
    for (uint32_t j = 0; j < S.nout; ++j) slot[c.outputs[j]] = c.na + c.nb + j;
    uint32_t next = c.na + c.nb + S.nout;
    for (const Gate& g : c.gates)
        if (slot[g.out] == UINT32_MAX) slot[g.out] = next++;
    S.slots = next;
    S.levels.assign(depth, {});
    for (size_t k = 0; k < c.gates.size(); ++k) {
        const Gate& g = c.gates[k];
        S.op.push_back(g.op);
        S.in0.push_back(slot[g.in0]);
        S.in1.push_back(slot[g.in1]);
        S.in2.push_back(g.in2 != kNoWire ? slot[g.in2] : kNoWire);
        S.three |= g.in2 != kNoWire;
        S.out.push_back(slot[g.out]);
        S.levels[glev[k] - 1].push_back((uint32_t)k);
    }
    return S;
}

enum JobState { kQueued = 0, kRunning = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

struct Job {
    fhe_job spec;
    const ServeShape* shape = nullptr;
    uint64_t ticket = 0;
    int state = kQueued;
    int error = FHE_OK;
    bool cancel = false;
    uint64_t base = 0;      // first pool slot
    uint32_t level = 0;     // next level to run
    Clock::time_point submitted, admitted, finished;
};

// First-fit allocator over pool slots.
class SlotAllocator {
  public:
    explicit SlotAllocator(uint64_t n) { free_[0] = n; }
    bool alloc(uint64_t n, uint64_t* at) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *at = it->first;
                const uint64_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t at, uint64_t n) {
        used_ -= n;
        auto it = free_.emplace(at, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;  // start -> length
    uint64_t used_ = 0;
};

}  // namespace
}  // namespace fhe

using namespace fhe;

namespace fhe {
namespace {
// One tick in flight: its descriptors (device, and pinned staging the upload
// reads from), the event recorded after its work, the jobs it finishes.
struct Tick {
    uint4* d_desc = nullptr;
    uint4* h_desc = nullptr;
    uint32_t* d_desc3 = nullptr;  // third inputs
    uint32_t* h_desc3 = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t gates = 0;
    std::vector<Job*> finishing;
};
constexpr int kRing = 3;
}  // namespace
}  // namespace fhe

struct fhe_server {
    fhe_ctx* ctx = nullptr;
    uint64_t capacity = 0;   // pool samples
    uint32_t* pool = nullptr;
    hipStream_t stream = nullptr;
    Tick ring[kRing];
    int next_tick = 0;
    std::deque<int> inflight;  // ring indices in launch order
    std::unique_ptr<SlotAllocator> slots;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job*> queue;
    std::vector<Job*> running;
    std::unordered_map<uint64_t, Job*> jobs;
    std::map<std::tuple<int, uint32_t, uint32_t, uint32_t, uint32_t>, ServeShape> shapes;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    uint64_t jobs_done = 0, gates_done = 0, launches = 0;
    int fatal = FHE_OK;
};

namespace {

const ServeShape* shape_for(fhe_server* S, const fhe_job& j) {
    const uint32_t op = j.kind == FHE_JOB_GATE ? j.op : 0;
    const uint32_t w = j.kind == FHE_JOB_GATE ? 1 : j.width;
    const uint32_t rows = j.kind == FHE_JOB_MATVEC || j.kind == FHE_JOB_MATMUL ? j.rows : 0;
    const uint32_t cols = j.kind == FHE_JOB_MATVEC ? j.cols : 0;
    auto key = std::make_tuple((int)j.kind, op, w, rows, cols);
    auto it = S->shapes.find(key);
    if (it == S->shapes.end()) it = S->shapes.emplace(key, make_shape(j.kind, op, w, rows, cols)).first;
    return &it->second;
}

void free_tick(Tick& T) {
    if (T.d_desc) (void)hipFree(T.d_desc);
    if (T.h_desc) (void)hipHostFree(T.h_desc);
    if (T.d_desc3) (void)hipFree(T.d_desc3);
    if (T.h_desc3) (void)hipHostFree(T.h_desc3);
    T.d_desc = nullptr;
    T.h_desc = nullptr;
    T.d_desc3 = nullptr;
    T.h_desc3 = nullptr;
    T.cap = 0;
}

// Descriptor room for n gates in tick T (T is not in flight).
int ensure_desc(Tick& T, size_t n) {
    if (n <= T.cap) return FHE_OK;
    size_t cap = std::max<size_t>(n, 2 * T.cap);
    cap = std::max<size_t>(cap, 4096);
    free_tick(T);
    hipError_t e = hipMalloc((void**)&T.d_desc, cap * sizeof(uint4));
    if (e == hipSuccess) e = hipHostMalloc((void**)&T.h_desc, cap * sizeof(uint4), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&T.d_desc3, cap * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&T.h_desc3, cap * sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "serving descriptors");
    T.cap = cap;
    return FHE_OK;
}

uint32_t pool_wire(uint64_t slot) { return (3u << 30) | (uint32_t)slot; }

// Marks the jobs of completed ticks done (blocking on the oldest tick when
// `block`); returns a device error, if any.  Called without the lock.
int reap(fhe_server* S, bool block) {
    int rc = FHE_OK;
    while (!S->inflight.empty()) {
        Tick& T = S->ring[S->inflight.front()];
        hipError_t e = block ? hipEventSynchronize(T.done) : hipEventQuery(T.done);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) rc = hip_fail(e, "serving tick");
        block = false;
        const Clock::time_point now = Clock::now();
        std::lock_guard<std::mutex> lk(S->mu);
        for (Job* j : T.finishing) {
            if (rc == FHE_OK) {
                j->state = kDone;
                j->finished = now;
                S->jobs_done++;
            } else {
                j->state = kFailed;
                j->error = rc;
            }
        }
        S->gates_done += rc == FHE_OK ? T.gates : 0;
        T.finishing.clear();
        T.busy = false;
        S->inflight.pop_front();
        if (rc != FHE_OK) S->fatal = rc;
        S->cv.notify_all();
    }
    return rc;
}

void fail_running(fhe_server* S, int rc) {
    for (Job* j : S->running) {
        j->state = kFailed;
        j->error = rc;
        S->slots->release(j->base, j->shape->slots);
    }
    S->running.clear();
    S->fatal = rc;
    S->cv.notify_all();
}

void worker_loop(fhe_server* S) {
    (void)hipSetDevice(S->ctx->device);
    const size_t W = kLweW;
    for (;;) {
        if (reap(S, false) != FHE_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            fail_running(S, S->fatal);
        }
        Tick* T = nullptr;
        size_t ngates = 0;
        bool three = false;
        int rc = FHE_OK;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // retire cancelled running jobs (ticks already enqueued may still
            // write their samples; anything reusing them is enqueued later)
            for (auto it = S->running.begin(); it != S->running.end();) {
                Job* j = *it;
                if (j->cancel) {
                    S->slots->release(j->base, j->shape->slots);
                    j->state = kCancelled;
                    it = S->running.erase(it);
                    S->cv.notify_all();
                } else {
                    ++it;
                }
            }
            // admission in arrival order
            while (!S->queue.empty()) {
                Job* j = S->queue.front();
                if (j->cancel) {
                    j->state = kCancelled;
                    S->queue.pop_front();
                    S->cv.notify_all();
                    continue;
                }
                uint64_t at = 0;
                if (!S->slots->alloc(j->shape->slots, &at)) break;
                j->base = at;
                j->state = kRunning;
                j->admitted = Clock::now();
                const size_t na = j->shape->na, nb = j->shape->nb;
                hipError_t e = hipMemcpyAsync(S->pool + at * W, j->spec.in0, na * W * 4, hipMemcpyDeviceToDevice, S->stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(S->pool + (at + na) * W, j->spec.in1, nb * W * 4, hipMemcpyDeviceToDevice, S->stream);
                if (e != hipSuccess) {
                    S->slots->release(at, j->shape->slots);
                    j->state = kFailed;
                    j->error = hip_fail(e, "serving input copy");
                    S->queue.pop_front();
                    S->cv.notify_all();
                    continue;
                }
                S->queue.pop_front();
                S->running.push_back(j);
            }
            if (S->running.empty()) {
                if (S->inflight.empty()) {
                    if (S->stop) return;
                    S->cv.wait_for(lk, std::chrono::milliseconds(2));
                    continue;
                }
                lk.unlock();
                reap(S, true);  // nothing new to launch: wait for the oldest tick
                continue;
            }
            T = &S->ring[S->next_tick];
            if (T->busy) {  // kRing ticks in flight: wait for the oldest
                lk.unlock();
                reap(S, true);
                continue;
            }
            for (Job* j : S->running) ngates += j->shape->levels[j->level].size();
            rc = ensure_desc(*T, ngates);
            if (rc != FHE_OK) {
                fail_running(S, rc);
                continue;
            }
            size_t k = 0;
            T->finishing.clear();
            for (auto it = S->running.begin(); it != S->running.end();) {
                Job* j = *it;
                const ServeShape& sh = *j->shape;
                three |= sh.three;
                for (uint32_t g : sh.levels[j->level]) {
                    T->h_desc3[k] = sh.in2[g] != kNoWire ? pool_wire(j->base + sh.in2[g]) : 0u;
                    T->h_desc[k++] = make_uint4(sh.op[g], pool_wire(j->base + sh.in0[g]),
                                                pool_wire(j->base + sh.in1[g]), pool_wire(j->base + sh.out[g]));
                }
                if (++j->level == sh.levels.size()) {
                    // last level: its output copy is enqueued with this tick,
                    // before anything that could reuse its samples
                    T->finishing.push_back(j);
                    S->slots->release(j->base, sh.slots);
                    it = S->running.erase(it);
                } else {
                    ++it;
                }
            }
            S->launches++;
        }
        // one launch pair for the whole frontier, then the finished jobs' outputs
        hipError_t e = hipMemcpyAsync(T->d_desc, T->h_desc, ngates * sizeof(uint4), hipMemcpyHostToDevice, S->stream);
        if (e == hipSuccess && three)
            e = hipMemcpyAsync(T->d_desc3, T->h_desc3, ngates * sizeof(uint32_t), hipMemcpyHostToDevice, S->stream);
        rc = e == hipSuccess ? FHE_OK : hip_fail(e, "serving descriptor upload");
        if (rc == FHE_OK) {
            dev::GateIO io{};
            io.desc = T->d_desc;
            io.desc3 = three ? T->d_desc3 : nullptr;
            io.region[3] = S->pool;
            rc = run_gate_batch(S->ctx, io, ngates, S->stream);
        }
        for (Job* j : T->finishing) {
            if (rc != FHE_OK) break;
            const ServeShape& sh = *j->shape;
            e = hipMemcpyAsync(j->spec.out, S->pool + (j->base + sh.na + sh.nb) * W, (size_t)sh.nout * W * 4,
                               hipMemcpyDeviceToDevice, S->stream);
            if (e != hipSuccess) rc = hip_fail(e, "serving output copy");
        }
        if (rc == FHE_OK) {
            e = hipEventRecord(T->done, S->stream);
            if (e != hipSuccess) rc = hip_fail(e, "serving tick event");
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (rc != FHE_OK) {
            for (Job* j : T->finishing) {
                j->state = kFailed;
                j->error = rc;
            }
            T->finishing.clear();
            fail_running(S, rc);
            continue;
        }
        T->gates = ngates;
        T->busy = true;
        S->inflight.push_back(S->next_tick);
        S->next_tick = (S->next_tick + 1) % kRing;
    }
}

}  // namespace

extern "C" int fhe_serve_create(fhe_ctx* ctx, size_t hbm_budget_bytes, fhe_server** out) {
    if (!ctx || !out) return set_error(FHE_EINVAL, "fhe_serve_create: null argument");
    *out = nullptr;
    const uint64_t capacity = hbm_budget_bytes / (kLweW * 4);
    if (capacity < 3) return set_error(FHE_EINVAL, "fhe_serve_create: budget below one gate job");
    if (capacity >= (1ull << 30)) return set_error(FHE_EINVAL, "fhe_serve_create: budget above 2^30 samples");
    DeviceGuard guard(ctx->device);
    fhe_server* S = new (std::nothrow) fhe_server();
    if (!S) return set_error(FHE_ENOMEM, "fhe_serve_create: out of host memory");
    S->ctx = ctx;
    S->capacity = capacity;
    // work of earlier calls on the context (any stream) completes first
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMalloc((void**)&S->pool, capacity * kLweW * 4);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    for (Tick& T : S->ring)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&T.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "fhe_serve_create");
        if (S->pool) (void)hipFree(S->pool);
        if (S->stream) (void)hipStreamDestroy(S->stream);
        for (Tick& T : S->ring)
            if (T.done) (void)hipEventDestroy(T.done);
        delete S;
        return rc;
    }
    S->slots.reset(new SlotAllocator(capacity));
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return FHE_OK;
}

extern "C" int fhe_serve_submit(fhe_server* S, const fhe_job* job, uint64_t* ticket) {
    if (!S || !job || !ticket) return set_error(FHE_EINVAL, "fhe_serve_submit: null argument");
    const fhe_job& j = *job;
    if (j.kind > FHE_JOB_MATMUL) return set_error(FHE_EINVAL, "fhe_serve_submit: job kind %u", j.kind);
    if (j.kind == FHE_JOB_GATE && j.op > FHE_ORYN) return set_error(FHE_EINVAL, "fhe_serve_submit: gate code %u", j.op);
    if (j.kind != FHE_JOB_GATE && (j.width < 1 || j.width > 64))
        return set_error(FHE_EINVAL, "fhe_serve_submit: width %u", j.width);
    if (j.kind == FHE_JOB_MATVEC && (j.rows == 0 || j.cols == 0 || j.rows > 4096 || j.cols > 4096))
        return set_error(FHE_EINVAL, "fhe_serve_submit: matrix %ux%u", j.rows, j.cols);
    if (j.kind == FHE_JOB_MATMUL && (j.rows == 0 || j.rows > 64))
        return set_error(FHE_EINVAL, "fhe_serve_submit: matrix dimension %u", j.rows);
    if (j.kind == FHE_JOB_KARATSUBA && j.width < 2)
        return set_error(FHE_EINVAL, "fhe_serve_submit: Karatsuba width %u", j.width);
    if (!j.in0 || !j.in1 || !j.out) return set_error(FHE_EINVAL, "fhe_serve_submit: null buffer");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return set_error(S->fatal, "fhe_serve_submit: server stopped after a device error");
    const ServeShape* sh = shape_for(S, j);
    if (sh->slots > S->capacity)
        return set_error(FHE_EBUSY, "fhe_serve_submit: job needs %u samples, budget holds %llu", sh->slots,
                         (unsigned long long)S->capacity);
    Job* J = new Job();
    J->spec = j;
    J->shape = sh;
    J->ticket = S->next_ticket++;
    J->submitted = Clock::now();
    S->jobs[J->ticket] = J;
    S->queue.push_back(J);
    *ticket = J->ticket;
    S->cv.notify_all();
    return FHE_OK;
}

extern "C" int fhe_serve_poll(fhe_server* S, uint64_t ticket, int* state, double* latency_ms) {
    if (!S || !state) return set_error(FHE_EINVAL, "fhe_serve_poll: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return set_error(FHE_EINVAL, "fhe_serve_poll: unknown ticket %llu", (unsigned long long)ticket);
    Job* J = it->second;
    *state = J->state;
    if (latency_ms)
        *latency_ms = J->state == kDone
                          ? std::chrono::duration<double, std::milli>(J->finished - J->submitted).count()
                          : -1.0;
    if (J->state == kCancelled) return set_error(FHE_ECANCELED, "fhe_serve_poll: job %llu was cancelled", (unsigned long long)ticket);
    if (J->state == kFailed) return set_error(J->error, "fhe_serve_poll: job %llu failed", (unsigned long long)ticket);
    return FHE_OK;
}

extern "C" int fhe_serve_job_times(fhe_server* S, uint64_t ticket, double* queue_ms, double* service_ms) {
    if (!S) return set_error(FHE_EINVAL, "fhe_serve_job_times: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end())
        return set_error(FHE_EINVAL, "fhe_serve_job_times: unknown ticket %llu", (unsigned long long)ticket);
    const Job* J = it->second;
    if (J->state != kDone)
        return set_error(FHE_EINVAL, "fhe_serve_job_times: job %llu is not done", (unsigned long long)ticket);
    using ms = std::chrono::duration<double, std::milli>;
    if (queue_ms) *queue_ms = ms(J->admitted - J->submitted).count();
    if (service_ms) *service_ms = ms(J->finished - J->admitted).count();
    return FHE_OK;
}

extern "C" int fhe_serve_wait(fhe_server* S, uint64_t ticket, double timeout_s) {
    if (!S) return set_error(FHE_EINVAL, "fhe_serve_wait: null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return set_error(FHE_EINVAL, "fhe_serve_wait: unknown ticket");
    Job* J = it->second;
    const auto deadline = Clock::now() + std::chrono::duration<double>(timeout_s);
    while (J->state == kQueued || J->state == kRunning) {
        if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout && (J->state == kQueued || J->state == kRunning))
            return set_error(FHE_EBUSY, "fhe_serve_wait: job %llu not done after %.1f s", (unsigned long long)ticket, timeout_s);
    }
    if (J->state == kCancelled) return set_error(FHE_ECANCELED, "fhe_serve_wait: job cancelled");
    if (J->state == kFailed) return set_error(J->error, "fhe_serve_wait: job failed");
    return FHE_OK;
}

extern "C" int fhe_serve_cancel(fhe_server* S, uint64_t ticket) {
    if (!S) return set_error(FHE_EINVAL, "fhe_serve_cancel: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return set_error(FHE_EINVAL, "fhe_serve_cancel: unknown ticket");
    if (it->second->state == kQueued || it->second->state == kRunning) it->second->cancel = true;
    S->cv.notify_all();
    return FHE_OK;
}

extern "C" int fhe_serve_stats(fhe_server* S, uint64_t* jobs_done, uint64_t* gates_done, uint64_t* launches,
                               uint64_t* pool_bytes_in_use, uint64_t* jobs_waiting) {
    if (!S) return set_error(FHE_EINVAL, "fhe_serve_stats: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (jobs_done) *jobs_done = S->jobs_done;
    if (gates_done) *gates_done = S->gates_done;
    if (launches) *launches = S->launches;
    if (pool_bytes_in_use) *pool_bytes_in_use = S->slots->used() * kLweW * 4;
    if (jobs_waiting) *jobs_waiting = S->queue.size();
    return FHE_OK;
}

extern "C" void fhe_serve_destroy(fhe_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (Job* j : S->queue) j->cancel = true;
        for (Job* j : S->running) j->cancel = true;
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    {
        DeviceGuard guard(S->ctx->device);
        (void)hipStreamSynchronize(S->stream);
        if (S->pool) (void)hipFree(S->pool);
        for (Tick& T : S->ring) {
            free_tick(T);
            if (T.done) (void)hipEventDestroy(T.done);
        }
        if (S->stream) (void)hipStreamDestroy(S->stream);
    }
    for (auto& kv : S->jobs) delete kv.second;
    delete S;
}
