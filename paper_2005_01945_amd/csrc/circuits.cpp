// Circuits on encrypted integers as device-resident plans: one batched
// launch pair per level over every instance, descriptor arrays into four
// buffer regions (the caller's two input buffers, the caller's output
// buffer and a pool of intermediate samples owned by the cached plan),
// captured HIP graphs.  The circuits themselves and their level schedules
// are built in circuit_build.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "fhe_internal.h"
#include "circuit_ir.h"
#include "runtime.h"

namespace fhe {

// A scheduled, device-resident plan for (kind, width, rows, cols, count).
struct Plan {
    uint32_t levels = 0;
    uint64_t gates = 0;
    std::vector<uint32_t> level_off, level_width;  // into desc
    uint4* desc = nullptr;                         // device descriptors
    uint32_t* desc3 = nullptr;                     // third-input wire ids (circuits with three-input gates)
    uint32_t* pool = nullptr;                      // intermediate samples
    uint32_t max_width = 0;
    uint64_t region_samples[4] = {0, 0, 0, 0};     // samples per region over all instances
    bool pair_slots = false;                       // compound nodes: two extracted samples per rotation
};

// A level schedule captured as a HIP graph for one set of caller buffers.
struct CapturedRun {
    hipGraphExec_t exec = nullptr;
    uint64_t big_generation = 0;
    uint64_t tune_generation = 0;
    uint64_t last_use = 0;
};

struct CircuitCache {
    std::map<std::tuple<int, uint32_t, uint32_t, uint32_t, size_t>, Plan> plans;
    std::map<std::tuple<const Plan*, const void*, const void*, const void*>, CapturedRun> graphs;
    std::map<uint32_t, Circuit> custom;  // caller-defined circuits by id (plans: kind kCustom, rows = id)
    uint32_t next_custom = 1;
    uint64_t clock = 0;
};

constexpr int kCustom = 1000;

constexpr size_t kMaxGraphs = 64;

namespace {

constexpr uint32_t kRegionA = 0, kRegionB = 1, kRegionR = 2, kRegionPool = 3;

uint32_t wire_id(uint32_t region, uint64_t index) { return (region << 30) | (uint32_t)index; }

int build_plan(fhe_ctx* ctx, int kind, uint32_t w, uint32_t rows, uint32_t cols, size_t count, Plan* P) {
    const Circuit c = kind == kCustom ? ctx->circuits->custom.at(rows) : build_circuit(kind, w, rows, cols);
    uint32_t depth = 0;
    const std::vector<uint32_t> asap = asap_levels(c, &depth);
    const bool pairs = c.has_compound();  // (balance_levels keeps such circuits at ASAP levels)
    const std::vector<uint32_t> glev = balance_levels(c, asap, depth, count, 8 * (uint64_t)ctx->cu_count);
    const uint32_t nw = c.wires();
    // Local wire -> (region, index within instance) for one instance.
    std::vector<uint32_t> region(nw, kRegionPool), local(nw, 0);
    for (uint32_t k = 0; k < c.na; ++k) { region[k] = kRegionA; local[k] = k; }
    for (uint32_t k = 0; k < c.nb; ++k) { region[c.na + k] = kRegionB; local[c.na + k] = k; }
    for (size_t j = 0; j < c.outputs.size(); ++j) { region[c.outputs[j]] = kRegionR; local[c.outputs[j]] = (uint32_t)j; }
    uint32_t npool = 0;
    for (const Gate& g : c.gates)
        if (region[g.out] == kRegionPool) local[g.out] = npool++;
    const uint64_t per_region[4] = {c.na, c.nb, (uint64_t)c.outputs.size(), npool};
    for (int r = 0; r < 4; ++r) P->region_samples[r] = per_region[r] * count;
    for (int r = 0; r < 4; ++r)
        if (per_region[r] * count >= (1ull << 30))
            return set_error(FHE_EINVAL, "circuit too large for one plan (%llu samples in a region)",
                             (unsigned long long)(per_region[r] * count));

    auto gid = [&](uint32_t wl, size_t inst) {
        return wire_id(region[wl], (uint64_t)inst * per_region[region[wl]] + local[wl]);
    };
    std::vector<std::vector<uint32_t>> by_level(depth + 1);
    for (size_t k = 0; k < c.gates.size(); ++k) by_level[glev[k]].push_back((uint32_t)k);
    std::vector<uint4> desc;
    std::vector<uint32_t> desc3;
    bool three = pairs;
    for (const Gate& g : c.gates) three |= g.in2 != kNoWire;
    desc.reserve(c.gates.size() * count);
    P->levels = depth;
    P->gates = c.bootstraps() * count;
    P->pair_slots = pairs;
    for (uint32_t L = 1; L <= depth; ++L) {
        P->level_off.push_back((uint32_t)desc.size());
        for (size_t inst = 0; inst < count; ++inst)
            for (uint32_t k : by_level[L]) {
                const Gate& g = c.gates[k];
                if (g.second) continue;  // emitted with its first output
                const bool comp = k + 1 < c.gates.size() && c.gates[k + 1].second;
                const uint32_t op = comp ? (dev::kCompoundFlag | g.op | (uint32_t)c.gates[k + 1].op << 8) : g.op;
                desc.push_back(make_uint4(op, gid(g.in0, inst), gid(g.in1, inst), gid(g.out, inst)));
                if (three)
                    desc3.push_back(comp ? gid(c.gates[k + 1].out, inst) : g.in2 != kNoWire ? gid(g.in2, inst) : 0u);
            }
        const uint32_t wdt = (uint32_t)(desc.size() - P->level_off.back());
        P->level_width.push_back(wdt);
        P->max_width = std::max(P->max_width, wdt);
    }
    hipError_t e = hipMalloc((void**)&P->desc, std::max<size_t>(desc.size(), 1) * sizeof(uint4));
    if (e != hipSuccess) return hip_fail(e, "circuit descriptors");
    e = hipMemcpy(P->desc, desc.data(), desc.size() * sizeof(uint4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "circuit descriptors");
    if (three) {
        e = hipMalloc((void**)&P->desc3, std::max<size_t>(desc3.size(), 1) * sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail(e, "circuit descriptors");
        e = hipMemcpy(P->desc3, desc3.data(), desc3.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "circuit descriptors");
    }
    if (npool) {
        e = hipMalloc((void**)&P->pool, (size_t)npool * count * kLweW * sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail(e, "circuit pool");
    }
    return ctx_reserve_big(ctx, (size_t)P->max_width * (pairs ? 2 : 1));
}

void free_plan(Plan& P) {
    if (P.desc) (void)hipFree(P.desc);
    if (P.desc3) (void)hipFree(P.desc3);
    if (P.pool) (void)hipFree(P.pool);
    P.desc = nullptr;
    P.desc3 = nullptr;
    P.pool = nullptr;
}

int get_plan(fhe_ctx* ctx, int kind, uint32_t w, uint32_t rows, uint32_t cols, size_t count, Plan** out) {
    if (!ctx->circuits) ctx->circuits = new CircuitCache();
    auto key = std::make_tuple(kind, w, rows, cols, count);
    auto it = ctx->circuits->plans.find(key);
    if (it != ctx->circuits->plans.end()) {
        *out = &it->second;
        return FHE_OK;
    }
    Plan P;
    int rc = build_plan(ctx, kind, w, rows, cols, count, &P);
    if (rc) {
        free_plan(P);
        return rc;
    }
    *out = &(ctx->circuits->plans[key] = P);
    return FHE_OK;
}

int enqueue_levels(fhe_ctx* ctx, const Plan* P, dev::GateIO io, hipStream_t s) {
    io.pair_slots = P->pair_slots ? 1 : 0;
    for (uint32_t L = 0; L < P->levels; ++L) {
        io.desc = P->desc + P->level_off[L];
        io.desc3 = P->desc3 ? P->desc3 + P->level_off[L] : nullptr;
        int rc = run_gate_batch(ctx, io, P->level_width[L], s);
        if (rc) return rc;
    }
    return FHE_OK;
}

void drop_graph(CapturedRun& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
}

// Captures the level schedule of P over these buffers on the context's own
// stream (kernel launches only) and instantiates it.
int capture_levels(fhe_ctx* ctx, const Plan* P, const dev::GateIO& io, CapturedRun* out) {
    int rc = ctx_reserve_big(ctx, (size_t)P->max_width * (P->pair_slots ? 2 : 1));  // none while capturing
    if (rc) return rc;
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    rc = enqueue_levels(ctx, P, io, ctx->stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->stream, &graph);
    if (rc == FHE_OK && e != hipSuccess) rc = hip_fail(e, "graph capture");
    if (rc == FHE_OK) {
        e = hipGraphInstantiate(&out->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "graph instantiation");
    }
    if (graph) (void)hipGraphDestroy(graph);
    out->big_generation = ctx->big_generation;
    out->tune_generation = ctx->tune_generation;
    return rc;
}

int run_circuit(fhe_ctx* ctx, int kind, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                uint32_t w, uint32_t rows, uint32_t cols, hipStream_t s, const char* name) {
    if (!ctx) return set_error(FHE_EINVAL, "%s: null context", name);
    if (w < 1 || w > 64) return set_error(FHE_EINVAL, "%s: width %u not in 1..64", name, w);
    if (count == 0) return FHE_OK;
    if (!A || !B || !R) return set_error(FHE_EINVAL, "%s: null buffer", name);
    DeviceGuard guard(ctx->device);
    Plan* P = nullptr;
    int rc = get_plan(ctx, kind, w, rows, cols, count, &P);
    if (rc) return rc;
    dev::GateIO io{};
    io.region[kRegionA] = const_cast<uint32_t*>(A);
    io.region[kRegionB] = const_cast<uint32_t*>(B);
    io.region[kRegionR] = R;
    io.region[kRegionPool] = P->pool;
    rc = order_begin(ctx, s);
    if (rc) return rc;
    if (!ctx->use_graphs || ctx->timing) return order_end(ctx, s, enqueue_levels(ctx, P, io, s));

    CircuitCache& C = *ctx->circuits;
    auto key = std::make_tuple((const Plan*)P, (const void*)A, (const void*)B, (const void*)R);
    CapturedRun& g = C.graphs[key];
    if (g.exec && (g.big_generation != ctx->big_generation || g.tune_generation != ctx->tune_generation))
        drop_graph(g);  // scratch moved or launch shapes changed
    if (!g.exec) {
        if (C.graphs.size() > kMaxGraphs) {  // evict the least recently used other entry
            auto victim = C.graphs.end();
            for (auto it = C.graphs.begin(); it != C.graphs.end(); ++it)
                if (it->first != key && (victim == C.graphs.end() || it->second.last_use < victim->second.last_use))
                    victim = it;
            if (victim != C.graphs.end()) {
                drop_graph(victim->second);
                C.graphs.erase(victim);
            }
        }
        CapturedRun& slot = C.graphs[key];
        rc = capture_levels(ctx, P, io, &slot);
        if (rc) {
            drop_graph(slot);
            C.graphs.erase(key);
            return rc;
        }
    }
    CapturedRun& run = C.graphs[key];
    run.last_use = ++C.clock;
    hipError_t e = hipGraphLaunch(run.exec, s);
    return order_end(ctx, s, e == hipSuccess ? FHE_OK : hip_fail(e, "graph launch"));
}

}  // namespace

// Frees the plans and graphs of caller-defined circuit `id` and forgets it.
static void drop_custom(fhe_ctx* ctx, uint32_t id) {
    CircuitCache& C = *ctx->circuits;
    for (auto it = C.plans.begin(); it != C.plans.end();) {
        if (std::get<0>(it->first) == kCustom && std::get<2>(it->first) == id) {
            const Plan* P = &it->second;
            for (auto g = C.graphs.begin(); g != C.graphs.end();) {
                if (std::get<0>(g->first) == P) {
                    drop_graph(g->second);
                    g = C.graphs.erase(g);
                } else {
                    ++g;
                }
            }
            free_plan(it->second);
            it = C.plans.erase(it);
        } else {
            ++it;
        }
    }
    C.custom.erase(id);
}

void destroy_circuit_cache(fhe_ctx* ctx) {
    if (!ctx->circuits) return;
    for (auto& kv : ctx->circuits->graphs) drop_graph(kv.second);
    for (auto& kv : ctx->circuits->plans) free_plan(kv.second);
    delete ctx->circuits;
    ctx->circuits = nullptr;
}

}  // namespace fhe

using namespace fhe;

extern "C" int fhe_add(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                       uint32_t width, void* stream) {
    return run_circuit(ctx, kAdd, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_add");
}

extern "C" int fhe_add_fa(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                          uint32_t width, void* stream) {
    return run_circuit(ctx, kAddFa, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_add_fa");
}

extern "C" int fhe_add_compound(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                                uint32_t width, void* stream) {
    return run_circuit(ctx, kAddCompound, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_add_compound");
}

extern "C" int fhe_add_numberwise(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                                  uint32_t width, void* stream) {
    return run_circuit(ctx, kAddNumberwise, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_add_numberwise");
}

extern "C" int fhe_mul(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                       uint32_t width, void* stream) {
    return run_circuit(ctx, kMul, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_mul");
}

extern "C" int fhe_mul_tree(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                            uint32_t width, void* stream) {
    return run_circuit(ctx, kMulTree, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_mul_tree");
}

extern "C" int fhe_mul_karatsuba(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                                 uint32_t width, void* stream) {
    if (width < 2) return set_error(FHE_EINVAL, "fhe_mul_karatsuba: width %u below 2", width);
    return run_circuit(ctx, kKaratsuba, A, B, R, count, width, 0, 0, (hipStream_t)stream, "fhe_mul_karatsuba");
}

extern "C" int fhe_matvec(fhe_ctx* ctx, const uint32_t* M, const uint32_t* x, uint32_t* y, uint32_t rows,
                          uint32_t cols, uint32_t width, void* stream) {
    if (rows == 0 || cols == 0) return set_error(FHE_EINVAL, "fhe_matvec: empty matrix");
    return run_circuit(ctx, kMatvec, M, x, y, 1, width, rows, cols, (hipStream_t)stream, "fhe_matvec");
}

extern "C" int fhe_matmul(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* C, uint32_t n,
                          uint32_t width, void* stream) {
    if (n == 0 || n > 64) return set_error(FHE_EINVAL, "fhe_matmul: dimension %u not in 1..64", n);
    return run_circuit(ctx, kMatmul, A, B, C, 1, width, n, 0, (hipStream_t)stream, "fhe_matmul");
}

// ---------------------------------------------------------------------------
// Caller-defined circuits.
// ---------------------------------------------------------------------------
struct fhe_circuit {
    fhe_ctx* ctx = nullptr;
    uint32_t id = 0, n_inputs = 0, n_outputs = 0;
};

extern "C" int fhe_circuit_create(fhe_ctx* ctx, const fhe_gate_node* gates, uint32_t n_gates, uint32_t n_inputs,
                                  const uint32_t* outputs, uint32_t n_outputs, fhe_circuit** out) {
    if (!ctx || !out || (n_gates && !gates) || !outputs)
        return set_error(FHE_EINVAL, "fhe_circuit_create: null argument");
    *out = nullptr;
    if (n_inputs == 0 || n_outputs == 0 || n_gates == 0 || n_inputs >= (1u << 24) || n_gates >= (1u << 24))
        return set_error(FHE_EINVAL, "fhe_circuit_create: %u inputs, %u gates, %u outputs", n_inputs, n_gates,
                         n_outputs);
    Circuit c;
    c.na = n_inputs;
    c.nb = 0;
    for (uint32_t k = 0; k < n_gates; ++k) {
        const fhe_gate_node& g = gates[k];
        const uint32_t lim = n_inputs + k;  // wires defined before gate k
        const bool three = g.op == FHE_MAJ || g.op == FHE_XOR3;
        if (g.op > FHE_XOR3 || g.in0 >= lim || g.in1 >= lim || (three && g.in2 >= lim))
            return set_error(FHE_EINVAL, "fhe_circuit_create: gate %u (op %u) reads a wire not defined before it", k,
                             g.op);
        c.gates.push_back({g.op, g.in0, g.in1, lim, three ? g.in2 : kNoWire});
    }
    std::vector<bool> seen(n_inputs + n_gates, false);
    for (uint32_t j = 0; j < n_outputs; ++j) {
        if (outputs[j] < n_inputs || outputs[j] >= n_inputs + n_gates || seen[outputs[j]])
            return set_error(FHE_EINVAL, "fhe_circuit_create: output %u must be a distinct gate output", j);
        seen[outputs[j]] = true;
        c.outputs.push_back(outputs[j]);
    }
    fhe_circuit* h = new (std::nothrow) fhe_circuit();
    if (!h) return set_error(FHE_ENOMEM, "fhe_circuit_create: out of host memory");
    if (!ctx->circuits) ctx->circuits = new CircuitCache();
    h->ctx = ctx;
    h->id = ctx->circuits->next_custom++;
    h->n_inputs = n_inputs;
    h->n_outputs = n_outputs;
    ctx->circuits->custom[h->id] = std::move(c);
    *out = h;
    return FHE_OK;
}

extern "C" int fhe_circuit_run(fhe_circuit* c, const uint32_t* in, uint32_t* out, size_t count, void* stream) {
    if (!c) return set_error(FHE_EINVAL, "fhe_circuit_run: null circuit");
    return run_circuit(c->ctx, kCustom, in, in, out, count, 1, c->id, 0, (hipStream_t)stream, "fhe_circuit_run");
}

extern "C" void fhe_circuit_destroy(fhe_circuit* c) {
    if (!c) return;
    if (c->ctx && c->ctx->circuits) {
        DeviceGuard guard(c->ctx->device);
        (void)hipDeviceSynchronize();  // runs may still be in flight on callers' streams
        drop_custom(c->ctx, c->id);
    }
    delete c;
}

// ---------------------------------------------------------------------------
// Test support: the schedule of a circuit entry point's plan and the words
// its wires hold after a run (teacher-forced checks of sampled gates).
// ---------------------------------------------------------------------------
static int debug_plan_lookup(fhe_ctx* ctx, int kind, uint32_t width, uint32_t rows, uint32_t cols,
                             uint64_t count, Plan** P, const char* name) {
    if (!ctx) return set_error(FHE_EINVAL, "%s: null context", name);
    const bool one = kind == kMatvec || kind == kMatmul;
    if (kind < 0 || kind > kLastKind || width < 1 || width > 64 || count == 0 || count > (1ull << 30) ||
        (kind == kKaratsuba && width < 2) || (kind == kMatvec && (rows == 0 || cols == 0)) ||
        (kind == kMatmul && (rows == 0 || rows > 64)) || (one && count != 1))
        return set_error(FHE_EINVAL, "%s: bad arguments", name);
    if (!one) rows = cols = 0;
    if (kind == kMatmul) cols = 0;
    DeviceGuard guard(ctx->device);
    return get_plan(ctx, kind, width, rows, cols, count, P);
}

extern "C" int fhe_debug_plan(fhe_ctx* ctx, int kind, uint32_t width, uint32_t rows, uint32_t cols, uint64_t count,
                              uint32_t* gates_out, uint64_t max_gates, uint32_t* level_off, uint32_t max_levels,
                              uint64_t* n_gates, uint32_t* n_levels) {
    Plan* P = nullptr;
    int rc = debug_plan_lookup(ctx, kind, width, rows, cols, count, &P, "fhe_debug_plan");
    if (rc) return rc;
    if (n_gates) *n_gates = P->gates;
    if (n_levels) *n_levels = P->levels;
    if (level_off) {
        if (max_levels < P->levels + 1) return set_error(FHE_EINVAL, "fhe_debug_plan: %u level offsets do not fit",
                                                         P->levels + 1);
        for (uint32_t L = 0; L < P->levels; ++L) level_off[L] = P->level_off[L];
        level_off[P->levels] = (uint32_t)P->gates;
    }
    if (gates_out) {
        if (max_gates < P->gates) return set_error(FHE_EINVAL, "fhe_debug_plan: %llu gates do not fit",
                                                   (unsigned long long)P->gates);
        DeviceGuard guard(ctx->device);
        std::vector<uint4> d(P->gates);
        std::vector<uint32_t> d3(P->desc3 ? P->gates : 0);
        hipError_t e = hipMemcpy(d.data(), P->desc, d.size() * sizeof(uint4), hipMemcpyDeviceToHost);
        if (e == hipSuccess && P->desc3)
            e = hipMemcpy(d3.data(), P->desc3, d3.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "fhe_debug_plan");
        for (size_t g = 0; g < d.size(); ++g) {
            const bool three =
                P->desc3 && (d[g].x == FHE_MAJ || d[g].x == FHE_XOR3 || (d[g].x & dev::kCompoundFlag) != 0);
            uint32_t* o = gates_out + 5 * g;
            o[0] = d[g].x;
            o[1] = d[g].y;
            o[2] = d[g].z;
            o[3] = d[g].w;
            o[4] = three ? d3[g] : kNoWire;
        }
    }
    return FHE_OK;
}

extern "C" int fhe_debug_read_wires(fhe_ctx* ctx, int kind, uint32_t width, uint32_t rows, uint32_t cols,
                                    uint64_t count, const uint32_t* A, const uint32_t* B, const uint32_t* R,
                                    const uint32_t* wires, size_t n, uint32_t* words_out) {
    Plan* P = nullptr;
    int rc = debug_plan_lookup(ctx, kind, width, rows, cols, count, &P, "fhe_debug_read_wires");
    if (rc) return rc;
    if (n && (!wires || !words_out)) return set_error(FHE_EINVAL, "fhe_debug_read_wires: null buffer");
    const uint32_t* base[4] = {A, B, R, P->pool};
    DeviceGuard guard(ctx->device);
    hipError_t e = hipDeviceSynchronize();  // runs may be in flight on any stream
    if (e != hipSuccess) return hip_fail(e, "fhe_debug_read_wires");
    for (size_t i = 0; i < n; ++i) {
        const uint32_t region = wires[i] >> 30;
        const uint64_t idx = wires[i] & 0x3FFFFFFFu;
        if (!base[region] || idx >= P->region_samples[region])
            return set_error(FHE_EINVAL, "fhe_debug_read_wires: wire %zu (0x%08x) is not a wire of this plan", i,
                             wires[i]);
        e = hipMemcpy(words_out + i * kLweW, base[region] + idx * kLweW, kLweW * sizeof(uint32_t),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "fhe_debug_read_wires");
    }
    return FHE_OK;
}
