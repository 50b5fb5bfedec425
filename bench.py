"""Benchmark: bootstrapped gates/s on one MI355X, batched vs plain, plus the
latency of one 32-bit multiplication.

One step = one batched 32-bit multiplication of 256 encrypted pairs
(shift-and-add keeping the low 32 bits: 722,944 bootstrapped gates in 120
levels, each level one launch pair), with inputs resident in HBM.  The
batched 16-bit addition of 1024 pairs (75,776 gates) and the 64x64 16-bit
matrix-vector product (2,952,576 gates) are timed as legs beside it.  Prints
one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config add16|mul32|matvec]
                  [--plain-reps R] [--mul-samples S] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402  (seeded plaintext inputs only)

# Algorithmic work of one gate bootstrap, in 32-bit integer lane operations,
# for the radix-2 NTT form of the method: 500 CMux x (6 NTT-1024 of 5,120
# butterflies + 8 x 1,024 pointwise products + their sums).
#   arith 0 (NTT over p = 2^64 - 2^32 + 1): 26 lane-ops per modmul (four
#     32x32->64 products and the reduction), 4 per modular add/sub.
#   arith 1 (NTT modulo two 28-bit primes): per prime, 3 per Montgomery
#     modmul and 1 per add/sub; plus the CRT recombination of the 2 x 1,024
#     output coefficients (7 each).
MODMUL_PER_CMUX = 6 * 5120 + 8 * 1024
MODADD_PER_CMUX = 6 * 5120 * 2 + 8 * 1024
LANE_OPS_PER_GATE = {
    0: 500 * (26 * MODMUL_PER_CMUX + 4 * MODADD_PER_CMUX),
    1: 500 * (2 * (3 * MODMUL_PER_CMUX + MODADD_PER_CMUX) + 7 * 2 * 1024),
}
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit integer op per lane-cycle.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Key switching gathers rows of the key-switching key: per gate 1,024 input
# coefficients x 8 base-4 digits, three quarters of them non-zero on average,
# each selecting one 501-word row (2,004 B).  The 50 MB key is far larger
# than one XCD's 4 MB L2 but rows are shared by the gates of a launch, so the
# gathers are served mostly from L2: the roof is the aggregate L2 bandwidth,
# 8 XCDs x 16 channels x 128 B per clock x 2.4 GHz.
KS_BYTES_PER_GATE = 1024 * 8 * 3 // 4 * 501 * 4
L2_PEAK_TBS = 8 * 16 * 128 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blind_rotate_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2005_01945_amd", "csrc", f)
               for f in ("kernels.hip", "goldilocks.h", "modq.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, gates_per_launch):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none for it or the kernel source changed since the
    counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash() or t.get("kernel") != kernel:
        return None
    return round(t["bytes_per_gate"] * gates_per_launch)


def host_threads():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def level1_sample(sk, config, count):
    """`count` gates of the first level of a workload: its operand-bit gates
    (AND of a_i, b_j for the multiplier; XOR / AND of a_i, b_i for the adder),
    on fresh encryptions of the workload's operands."""
    if config == "add16":
        wl = workloads.AddWorkload()
        pairs = [(op, c, i, i) for c in range(wl.count) for i in range(wl.width) for op in (4, 0)]
    else:
        wl = workloads.MulWorkload()
        pairs = [(0, c, j, i) for c in range(wl.count) for i in range(wl.width) for j in range(wl.width - i)]
    a, b = wl.operands()
    pairs = pairs[:count]
    used = sorted({p[1] for p in pairs})
    ca = sk.encrypt_uint(a[used], wl.width, nonce=0)
    cb = sk.encrypt_uint(b[used], wl.width, nonce=1 << 40)
    row = {c: k for k, c in enumerate(used)}
    ops = np.array([p[0] for p in pairs], np.uint8)
    i0 = np.stack([ca[row[p[1]], p[2]] for p in pairs])
    i1 = np.stack([cb[row[p[1]], p[3]] for p in pairs])
    return ops, i0, i1


def cpu_baseline(sk, config, sample_gates, single_gates, gates_per_step):
    """The oracle on the host cores (all threads, then one) on level-1 gates of
    the benchmark's workload; every bootstrap costs the same, so the per-gate
    rate extrapolates to whole workloads (labelled as extrapolated)."""
    import oracle
    K = oracle.Keys(0)
    sample = "add16" if config == "add16" else "mul32"
    ops, i0, i1 = level1_sample(sk, sample, sample_gates)
    threads = host_threads()
    t0 = time.perf_counter()
    K.bootstrap(ops, i0, i1, threads=threads)
    dt = time.perf_counter() - t0
    rate = len(ops) / dt
    t0 = time.perf_counter()
    K.bootstrap(ops[:single_gates], i0[:single_gates], i1[:single_gates], threads=1)
    dt1 = time.perf_counter() - t0
    rate1 = single_gates / dt1
    full = {name: round(g / rate / 3600, 2) for name, g in gates_per_step.items()}
    return {"value": round(rate, 3), "unit": "gates/s", "cores": threads, "kind": "oracle",
            "single_core_gates_per_s": round(rate1, 3), "cpu_model": cpu_model(),
            "sample": f"{len(ops)} gates of level 1 of the {sample} workload on {threads} threads ({dt:.1f} s), "
                      f"{single_gates} of them on one thread ({dt1:.1f} s); every bootstrap does the same work",
            "extrapolated_full_config_hours": full}


def cpu_parallel_leg(sk, ck, config, sample_gates, gpu_value):
    """The paper's CPU parallel framework (Sec. IV) on the host's cores: a
    batch of level-1 gates of the benchmark's workload (one gate per thread),
    16 add16 pairs (numbers across threads, bits in carry order) and one
    16-bit multiplication (ANDs across threads, accumulation in order)."""
    from paper_2005_01945_amd import cpupar
    bk, ksk = ck.export()
    cp = cpupar.CpuParallel(bk, ksk)
    threads = host_threads()
    ops, i0, i1 = level1_sample(sk, "add16" if config == "add16" else "mul32", sample_gates)
    t0 = time.perf_counter()
    cp.bootstrap(ops, i0, i1, threads=threads)
    dt = time.perf_counter() - t0
    rate = len(ops) / dt
    wl = workloads.AddWorkload(count=16)
    a, b = wl.operands()
    ca, cb = sk.encrypt_uint(a, 16, nonce=7 << 48), sk.encrypt_uint(b, 16, nonce=(7 << 48) + 4096)
    t0 = time.perf_counter()
    r = cp.add(ca, cb, 16, threads=threads)
    add_s = time.perf_counter() - t0
    if not np.array_equal(sk.decrypt_uint(r, 16), (a + b) % (1 << 16)):
        raise SystemExit("bench: CPU parallel additions decrypt wrongly")
    ma, mb = workloads.uniform_uints(16, 1, 16), workloads.uniform_uints(17, 1, 16)
    cma, cmb = sk.encrypt_uint(ma, 16, nonce=8 << 48), sk.encrypt_uint(mb, 16, nonce=(8 << 48) + 64)
    t0 = time.perf_counter()
    r = cp.mul(cma, cmb, 16, threads=threads)
    mul_s = time.perf_counter() - t0
    if sk.decrypt_uint(r, 16)[0] != (int(ma[0]) * int(mb[0])) % (1 << 16):
        raise SystemExit("bench: CPU parallel multiplication decrypts wrongly")
    return {"kind": "the paper's CPU parallel framework (Sec. IV): one gate per core, two-prime NTT products",
            "gates_per_s": round(rate, 2), "cores": threads,
            "sample": f"{len(ops)} level-1 gates of the benchmark's workload in {dt:.1f} s",
            "add16_x16": {"s": round(add_s, 2), "adds_per_s": round(16 / add_s, 2)},
            "mul16_latency_s": round(mul_s, 2),
            "gpu_batched_over_cpu_parallel": round(gpu_value / rate, 1)}


JOB_GATES = None


def serving_leg(F, sk, ctx, rate_gates_per_s, n_jobs, budget_bytes, seed=3):
    """Poisson stream of mixed jobs (single gates, add16, add32, mul32 with
    tree accumulation, 8x8 8-bit matvec) offered at rate_gates_per_s; every
    job is checked against plaintext arithmetic after the run."""
    import torch
    kinds = {"gate": (F.FHE_JOB_GATE, 1), "add16": (F.FHE_JOB_ADD, 16), "add32": (F.FHE_JOB_ADD, 32),
             "mul32": (F.FHE_JOB_MUL_TREE, 32), "matvec8": (F.FHE_JOB_MATVEC, 8)}
    gates_of = {"gate": 1, "add16": F.fhe_circuit_shape("add", 16)[0], "add32": F.fhe_circuit_shape("add", 32)[0],
                "mul32": F.fhe_circuit_shape("mul_tree", 32)[0], "matvec8": F.fhe_circuit_shape("matvec", 8, 8, 8)[0]}
    mean_gates = sum(p * gates_of[k] for k, p in zip(workloads.JOB_KINDS, workloads.JOB_MIX))
    jobs = workloads.job_stream(seed, n_jobs, rate_gates_per_s / mean_gates)
    prepared = []
    nonce = 1 << 56
    for j in jobs:
        kind, w = kinds[j.kind]
        if j.kind == "gate":
            a = sk.encrypt_bits(j.a, nonce=nonce); b = sk.encrypt_bits(j.b, nonce=nonce + 1); nonce += 2
            shape, rows, cols = (1, F.WORDS), 0, 0
            a_, b_ = int(j.a[0]), int(j.b[0])
            want = [[a_ & b_, 1 - (a_ & b_), a_ | b_, 1 - (a_ | b_), a_ ^ b_, 1 - (a_ ^ b_),
                     (1 - a_) & b_, a_ & (1 - b_), (1 - a_) | b_, a_ | (1 - b_)][j.op]]
        elif j.kind == "matvec8":
            a = sk.encrypt_uint(j.a.reshape(-1), w, nonce=nonce); nonce += 64 * w
            b = sk.encrypt_uint(j.b, w, nonce=nonce); nonce += 8 * w
            shape, rows, cols = (8, w, F.WORDS), 8, 8
            want = list((j.a @ j.b) % (1 << w))
        else:
            a = sk.encrypt_uint(j.a, w, nonce=nonce); b = sk.encrypt_uint(j.b, w, nonce=nonce + w); nonce += 2 * w
            shape, rows, cols = (w, F.WORDS), 0, 0
            x, y = int(j.a[0]), int(j.b[0])
            want = [((x + y) if kind == F.FHE_JOB_ADD else (x * y)) % (1 << w)]
        prepared.append(dict(j=j, kind=kind, w=w, rows=rows, cols=cols, da=F.to_device(a), db=F.to_device(b),
                             out=torch.zeros(shape, dtype=torch.int32, device="cuda"), want=want))
    torch.cuda.synchronize()
    srv = F.Server(ctx, budget_bytes)
    t0 = time.perf_counter()
    tickets = []
    for p in prepared:
        delay = p["j"].arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(F.fhe_serve_submit(srv, p["kind"], p["da"], p["db"], p["out"], op=p["j"].op,
                                          width=p["w"], rows=p["rows"], cols=p["cols"]))
    for t in tickets:
        F.fhe_serve_wait(srv, t, 1200)
    t1 = time.perf_counter()
    stats = F.fhe_serve_stats(srv)
    lat, wait, serv = {}, {}, {}
    bad = 0
    for p, t in zip(prepared, tickets):
        st, ms = F.fhe_serve_poll(srv, t)
        q, v = F.fhe_serve_job_times(srv, t)
        k = p["j"].kind
        lat.setdefault(k, []).append(ms)
        wait.setdefault(k, []).append(q)
        serv.setdefault(k, []).append(v)
        host = F.to_host(p["out"])
        dec = sk.decrypt_bits(host) if p["kind"] == F.FHE_JOB_GATE else sk.decrypt_uint(host, p["w"])
        bad += list(dec) != list(p["want"])
    srv.close()
    if bad:
        raise SystemExit(f"bench: {bad} served jobs decrypted wrongly")
    total_gates = sum(gates_of[p["j"].kind] for p in prepared)
    span = prepared[-1]["j"].arrival_s - prepared[0]["j"].arrival_s

    def pct(v):
        return {"p50": round(float(np.percentile(v, 50)), 1), "p99": round(float(np.percentile(v, 99)), 1)}

    served = total_gates / (t1 - t0)
    offered = total_gates / span if span > 0 else rate_gates_per_s
    return {"jobs": len(prepared), "gates": total_gates, "offered_gates_per_s": round(offered, 1),
            "served_gates_per_s": round(served, 1), "served_over_offered": round(served / offered, 3),
            "wall_s": round(t1 - t0, 2), "launches": stats["launches"], "hbm_budget_bytes": budget_bytes,
            "mul32_circuit": "tree accumulation (Sec. V-B-2), 62 levels",
            "latency_ms": {k: {**pct(v), "n": len(v)} for k, v in sorted(lat.items())},
            "queue_ms": {k: pct(v) for k, v in sorted(wait.items())},
            "service_ms": {k: pct(v) for k, v in sorted(serv.items())}}


def prepare_config(F, sk, ctx, name, stream):
    """Encrypted operands resident in HBM and the step of workload `name`."""
    import torch
    if name in ("add16", "mul32"):
        wl = workloads.AddWorkload() if name == "add16" else workloads.MulWorkload()
        a, b = wl.operands()
        width, count = wl.width, wl.count
        ca, cb = sk.encrypt_uint(a, width, nonce=0), sk.encrypt_uint(b, width, nonce=1 << 40)
        dA, dB = F.to_device(ca), F.to_device(cb)
        dR = torch.empty_like(dA)
        kind = "add" if name == "add16" else "mul"
        fn = F.fhe_add if name == "add16" else F.fhe_mul
        step = lambda: fn(ctx, dA, dB, dR, count, width, stream)
        gates, levels, _ = F.fhe_circuit_shape(kind, width)
        expect = (a + b) % (1 << width) if name == "add16" else (a.astype(object) * b.astype(object)) % (1 << width)
        label = (f"batched {width}-bit ripple-carry addition" if name == "add16"
                 else f"batched {width}-bit shift-and-add multiplication (low {width} bits)")
        workload = {"workload": label, "pairs": count, "width": width, "gates_per_step": gates * count,
                    "levels": levels}
        gates_per_step = gates * count
    else:
        wl = workloads.MatvecWorkload()
        M, x = wl.operands()
        width = wl.width
        cm = sk.encrypt_uint(M.reshape(-1), width, nonce=0)
        cx = sk.encrypt_uint(x, width, nonce=1 << 40)
        dA, dB = F.to_device(cm), F.to_device(cx)
        dR = torch.empty((wl.rows, width, F.WORDS), dtype=torch.int32, device="cuda")
        step = lambda: F.fhe_matvec(ctx, dA, dB, dR, wl.rows, wl.cols, width, stream)
        gates, levels, _ = F.fhe_circuit_shape("matvec", width, wl.rows, wl.cols)
        expect = (M @ x) % (1 << width)
        workload = {"workload": f"encrypted {wl.rows}x{wl.cols} matrix-vector product, {width}-bit",
                    "rows": wl.rows, "cols": wl.cols, "width": width, "gates_per_step": gates, "levels": levels}
        gates_per_step = gates

    def verify():
        got = sk.decrypt_uint(F.to_host(dR), width).astype(object)
        return np.array_equal(got, np.asarray(expect).reshape(-1).astype(object))

    return dict(name=name, step=step, gates_per_step=gates_per_step, levels=levels, workload=workload,
                verify=verify, dA=dA, dB=dB, dR=dR, width=width)


def roofline_of(records):
    """Roofline object of the blind-rotation shape with the most device time
    in `records` (per-launch HIP events on the launch stream)."""
    by_shape = {}
    for r in records:
        e = by_shape.setdefault(r["shape"], {"launches": 0, "gates": 0, "ms": 0.0})
        e["launches"] += 1
        e["gates"] += r["gates"]
        e["ms"] += r["blind_rotate_ms"]
    shape = max(by_shape, key=lambda k: by_shape[k]["ms"])
    dom = by_shape[shape]
    gates_per_launch = dom["gates"] / dom["launches"]
    avg_launch_ms = dom["ms"] / dom["launches"]
    achieved = LANE_OPS_PER_GATE[shape[2]] * gates_per_launch / (avg_launch_ms / 1e3) / 1e12
    kernel = f"k_blind_rotate_pair<{shape[2]}>" if shape[0] == 2 else f"k_blind_rotate<{shape[1]}, {shape[2]}>"
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(kernel, gates_per_launch),
                "kernel": kernel, "launches": dom["launches"], "avg_launch_ms": round(avg_launch_ms, 3),
                "gates_per_launch": round(gates_per_launch, 1)}
    per_shape = {f"{k[0]}x{k[1]}/arith{k[2]}": {"launches": v["launches"], "gates": v["gates"], "ms": round(v["ms"], 3)}
                 for k, v in sorted(by_shape.items())}
    return roofline, per_shape, shape


def key_switch_roof(records):
    """Key switching against the aggregate L2 bandwidth: algorithmic bytes =
    the expected 6,144 non-zero digit rows of 2,004 B gathered per gate."""
    gates = sum(r["gates"] for r in records)
    ms = sum(r["key_switch_ms"] for r in records)
    if not gates or ms <= 0:
        return None
    achieved = KS_BYTES_PER_GATE * gates / (ms / 1e3) / 1e12
    return {"bound": "l2", "achieved": round(achieved, 3), "peak": round(L2_PEAK_TBS, 2), "unit": "TB/s",
            "frac": round(achieved / L2_PEAK_TBS, 4), "ms": round(ms, 3), "gates": gates}


def time_config(F, ctx, cfg, steps, warmup):
    """Warm-up, then `steps` timed steps with per-launch events."""
    import torch
    for _ in range(warmup):
        cfg["step"]()
    torch.cuda.synchronize()
    F.fhe_ctx_timing(ctx)  # drop anything recorded so far
    F.fhe_ctx_set_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cfg["step"]()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    F.fhe_ctx_set_timing(ctx, False)
    records = F.fhe_ctx_timing_launches(ctx)
    if not cfg["verify"]():
        raise SystemExit(f"bench: {cfg['name']}: decrypted results differ from plaintext arithmetic")
    ms = (t1 - t0) * 1e3 / steps
    roofline, per_shape, shape = roofline_of(records)
    br = sum(r["blind_rotate_ms"] for r in records)
    ks = sum(r["key_switch_ms"] for r in records)
    return {"gates_per_s": round(cfg["gates_per_step"] / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
            "steps": steps, "warmup": warmup, "config": cfg["workload"],
            "phase_ms_per_step": {"blind_rotate": round(br / steps, 3), "key_switch": round(ks / steps, 3)},
            "launches_per_step": len(records) // max(steps, 1), "roofline": roofline,
            "key_switch_roofline": key_switch_roof(records), "timed_by_shape": per_shape,
            "_shape": shape}


def latency(fn, samples):
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(samples):
        s0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out.append(time.perf_counter() - s0)
    return {"p50_ms": round(1e3 * float(np.median(out)), 2), "p99_ms": round(1e3 * float(np.percentile(out, 99)), 2),
            "samples": len(out)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="mul32", choices=["add16", "mul32", "matvec"],
                    help="workload of `value` (default: the 256-pair 32-bit multiplication)")
    ap.add_argument("--leg-steps", type=int, default=5, help="timed steps of the add16 leg")
    ap.add_argument("--matvec-steps", type=int, default=1, help="timed steps of the matvec leg (0: skip)")
    ap.add_argument("--graph-steps", type=int, default=2, help="steps replayed from the captured HIP graphs")
    ap.add_argument("--plain-reps", type=int, default=50)
    ap.add_argument("--mul-samples", type=int, default=50)
    ap.add_argument("--circuit-samples", type=int, default=5)
    ap.add_argument("--compound-samples", type=int, default=10,
                    help="samples of the compound-gate against two-single-gates comparison (0: skip)")
    ap.add_argument("--cpu-sample-gates", type=int, default=768)
    ap.add_argument("--cpu-single-gates", type=int, default=48)
    ap.add_argument("--tune-max-width", type=int, default=4096,
                    help="autotune launch shapes up to this batch width before warmup (0 keeps the defaults)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-parallel-gates", type=int, default=3072,
                    help="gates of the CPU parallel framework leg (0 skips the leg)")
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs in the serving leg (0 skips it)")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load of the serving leg as a fraction of the batched throughput")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--small-budget-jobs", type=int, default=400,
                    help="jobs of a second serving run under a small HBM budget (0 skips it)")
    ap.add_argument("--small-budget-mib", type=float, default=256.0)
    ap.add_argument("--goldilocks-steps", type=int, default=1,
                    help="add16 steps timed once more with the NTT over 2^64 - 2^32 + 1 (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the gates of a level are "
              "independent, so several GPUs would each take a share of every level", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_01945_amd as F

    sk, ck = F.fhe_keygen(0)
    ctx = F.Context(ck, 0)
    stream = torch.cuda.current_stream()
    tuning_s = None
    if args.tune_max_width > 0:
        log(f"autotuning launch shapes up to width {args.tune_max_width}")
        t = time.perf_counter()
        F.fhe_ctx_autotune(ctx, args.tune_max_width, 1)
        tuning_s = round(time.perf_counter() - t, 2)
    shapes = [[1 << b, *F.fhe_ctx_launch_config(ctx, 1 << b)] for b in range(16)]
    log(f"launch shapes [bucket width, waves/gate, gates/group, arith]: {shapes}")

    # issue rates of the VALU instruction classes of the blind rotation (the
    # per-class peaks behind the roofline's 39.32 T: one 32-bit operation per
    # lane per cycle at 2.4 GHz)
    valu_rates = {name: round(F.fhe_debug_valu_rate(op) / 1e12, 2) for op, name in enumerate(F.VALU_CLASSES)}
    log(f"VALU issue rates (T lane-ops/s): {valu_rates}")

    # --- the measured workload (`value`) ---
    main_cfg = prepare_config(F, sk, ctx, args.config, stream)
    log(f"config {args.config}: {main_cfg['gates_per_step']} gates/step, {main_cfg['levels']} levels; "
        f"warmup {args.warmup}, timing {args.steps} steps")
    res = time_config(F, ctx, main_cfg, args.steps, args.warmup)
    ms_per_step = res["ms_per_step"]
    value = main_cfg["gates_per_step"] / (ms_per_step / 1e3)
    log(f"{ms_per_step:.1f} ms/step, {value:.0f} gates/s; phases {res['phase_ms_per_step']}")

    # the same steps replayed from the captured HIP graphs (timing off)
    graph_ms_per_step = None
    if args.graph_steps > 0:
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.graph_steps):
            main_cfg["step"]()
        torch.cuda.synchronize()
        graph_ms_per_step = (time.perf_counter() - g0) * 1e3 / args.graph_steps
        log(f"graph replay: {graph_ms_per_step:.1f} ms/step")

    # one step with the inputs copied in from pinned host memory and the
    # results copied out (the PCIe-inclusive rate; not `value`)
    dA, dB, dR = main_cfg["dA"], main_cfg["dB"], main_cfg["dR"]
    hA, hB = dA.cpu().pin_memory(), dB.cpu().pin_memory()
    hR = torch.empty(dR.shape, dtype=dR.dtype).pin_memory()
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    dA.copy_(hA, non_blocking=True)
    dB.copy_(hB, non_blocking=True)
    main_cfg["step"]()
    hR.copy_(dR, non_blocking=True)
    torch.cuda.synchronize()
    e2e_ms = (time.perf_counter() - e0) * 1e3
    end_to_end = {"gates_per_s": round(main_cfg["gates_per_step"] / (e2e_ms / 1e3), 1), "ms_per_step": round(e2e_ms, 1),
                  "bytes_in": int(hA.numel() + hB.numel()) * 4, "bytes_out": int(hR.numel()) * 4}
    log(f"with host transfers: {end_to_end}")
    if not main_cfg["verify"]():
        raise SystemExit("bench: results after the host-transfer step differ from plaintext arithmetic")
    del hA, hB, hR

    # --- the other batched workloads, each timed with its own roofline ---
    legs = {}
    add_cfg = main_cfg if args.config == "add16" else prepare_config(F, sk, ctx, "add16", stream)
    if args.config != "add16" and args.leg_steps > 0:
        log(f"leg add16: {add_cfg['gates_per_step']} gates/step, warmup 1, {args.leg_steps} steps")
        legs["add16"] = time_config(F, ctx, add_cfg, args.leg_steps, 1)
        log(f"leg add16: {legs['add16']['gates_per_s']} gates/s")
    if args.config != "matvec" and args.matvec_steps > 0:
        mv = prepare_config(F, sk, ctx, "matvec", stream)
        log(f"leg matvec: {mv['gates_per_step']} gates/step, warmup 1, {args.matvec_steps} steps")
        legs["matvec"] = time_config(F, ctx, mv, args.matvec_steps, 1)
        log(f"leg matvec: {legs['matvec']['gates_per_s']} gates/s")
        del mv
        torch.cuda.empty_cache()
    if args.config != "mul32" and args.leg_steps > 0:
        mc = prepare_config(F, sk, ctx, "mul32", stream)
        log(f"leg mul32: {mc['gates_per_step']} gates/step, warmup 1, 1 step")
        legs["mul32"] = time_config(F, ctx, mc, 1, 1)
        del mc
    for v in legs.values():
        v.pop("_shape", None)

    # the add16 step once more with the NTT over the Goldilocks prime
    # 2^64 - 2^32 + 1 (one wave per gate, four gates per workgroup), against
    # its own algorithmic count; then the tuned shapes are put back
    goldilocks = None
    if args.goldilocks_steps > 0:
        saved = [F.fhe_ctx_launch_config(ctx, 1 << b) for b in range(16)]
        F.fhe_ctx_set_launch_config(ctx, 1, 1 << 31, (1, 4, 0))
        add_cfg["step"]()
        torch.cuda.synchronize()
        F.fhe_ctx_timing(ctx)
        F.fhe_ctx_set_timing(ctx, True)
        gs0 = time.perf_counter()
        for _ in range(args.goldilocks_steps):
            add_cfg["step"]()
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - gs0) * 1e3 / args.goldilocks_steps
        F.fhe_ctx_set_timing(ctx, False)
        grec = [r for r in F.fhe_ctx_timing_launches(ctx) if r["shape"] == (1, 4, 0)]
        g_gates = sum(r["gates"] for r in grec)
        g_br = sum(r["blind_rotate_ms"] for r in grec)
        g_ach = LANE_OPS_PER_GATE[0] * g_gates / (g_br / 1e3) / 1e12
        goldilocks = {"workload": "add16 x 1024", "gates_per_s": round(add_cfg["gates_per_step"] / (g_ms / 1e3), 1),
                      "ms_per_step": round(g_ms, 1), "kernel": "k_blind_rotate<4, 0>", "achieved": round(g_ach, 3),
                      "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s", "frac": round(g_ach / VALU_PEAK_TOPS, 4)}
        for b, shp in enumerate(saved):
            F.fhe_ctx_set_launch_config(ctx, 1 << b, 1 << b, shp)
        if not add_cfg["verify"]():
            raise SystemExit("bench: Goldilocks-path results differ from plaintext arithmetic")
        log(f"Goldilocks NTT: {goldilocks}")

    # compound gates (Sec. V-A-3, Fig. 5c): the XOR and the AND of the same
    # inputs from one blind rotation, against the two single gates in one batch
    compound = None
    if args.compound_samples > 0:
        compound = {}
        for n in (1, 32, 2048):
            a_bits, b_bits = workloads.bits(80, n), workloads.bits(81, n)
            c0 = sk.encrypt_bits(a_bits, nonce=(1 << 51) + 10 * n)
            c1 = sk.encrypt_bits(b_bits, nonce=(1 << 51) + 10 * n + 4096)
            d0, d1 = F.to_device(c0), F.to_device(c1)
            d00, d11 = torch.cat([d0, d0]), torch.cat([d1, d1])
            ox = torch.full((n,), F.XOR, dtype=torch.uint8, device="cuda")
            oa = torch.full((n,), F.AND, dtype=torch.uint8, device="cuda")
            oxa = torch.cat([ox, oa])
            o0, o1, o2 = torch.empty_like(d0), torch.empty_like(d0), torch.empty_like(d00)
            single = latency(lambda: F.fhe_bootstrap_gate_batch(ctx, oxa, d00, d11, o2, 2 * n, stream),
                             args.compound_samples)
            comp = latency(lambda: F.fhe_bootstrap_compound_batch(ctx, ox, oa, d0, d1, o0, o1, n, stream),
                           args.compound_samples)
            assert (sk.decrypt_bits(F.to_host(o0)) == (a_bits ^ b_bits)).all()
            assert (sk.decrypt_bits(F.to_host(o1)) == (a_bits & b_bits)).all()
            assert (sk.decrypt_bits(F.to_host(o2)) == np.concatenate([a_bits ^ b_bits, a_bits & b_bits])).all()
            compound[f"{n}_pairs"] = {"compound_ms": comp["p50_ms"], "two_single_gates_ms": single["p50_ms"],
                                      "single_over_compound": round(single["p50_ms"] / comp["p50_ms"], 2)}
        wl = workloads.AddWorkload()
        aA, aB, aR = add_cfg["dA"], add_cfg["dB"], add_cfg["dR"]
        ca16 = latency(lambda: F.fhe_add_compound(ctx, aA, aB, aR, wl.count, wl.width, stream), 2)
        assert add_cfg["verify"]()
        rot = F.fhe_circuit_shape("add_compound", wl.width)[0] * wl.count
        add_ms = legs["add16"]["ms_per_step"] if "add16" in legs else ms_per_step if args.config == "add16" else None
        compound["add16_x1024"] = {"compound_ms": ca16["p50_ms"], "rotations": rot,
                                   "two_input_gates_ms": add_ms,
                                   "two_input_gates": F.fhe_circuit_shape("add", wl.width)[0] * wl.count}
        log(f"compound gates: {compound}")

    if args.copy_calibration_mib > 0:
        src = torch.empty(args.copy_calibration_mib << 18, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: {args.copy_calibration_mib} MiB read + written")

    # plain path: one gate per launch, synchronous (NAND on the four input pairs)
    plain = None
    a_bits, b_bits = workloads.truth_table_inputs()
    p0 = F.to_device(sk.encrypt_bits(a_bits, nonce=1 << 50))
    p1 = F.to_device(sk.encrypt_bits(b_bits, nonce=(1 << 50) + 100))
    pout = torch.empty_like(p0)
    lat = []
    for rep in range(args.plain_reps + 1 if args.plain_reps > 0 else 0):
        for g in range(4):
            s0 = time.perf_counter()
            F.fhe_bootstrap_gate_plain(ctx, F.NAND, p0[g], p1[g], pout[g], stream)
            if rep > 0:  # the first round is warmup
                lat.append(time.perf_counter() - s0)
    if lat:
        assert list(sk.decrypt_bits(F.to_host(pout))) == [1, 1, 1, 0]
        plain = {"gates_per_s": round(len(lat) / sum(lat), 2), "p50_ms": round(1e3 * float(np.median(lat)), 3),
                 "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3), "gates": len(lat),
                 "reps": args.plain_reps, "batched_over_plain": round(value / (len(lat) / sum(lat)), 1)}
        log(f"plain: {plain}")

    # latency of one 32-bit multiplication: shift-and-add (120 levels), tree
    # accumulation (62 levels, same 2,824 gates), Karatsuba (full product)
    mul = mul_tree = mul_kara = None
    if args.mul_samples > 0:
        ma = workloads.uniform_uints(11, 1, 32)
        mb = workloads.uniform_uints(12, 1, 32)
        mA = F.to_device(sk.encrypt_uint(ma, 32, nonce=1 << 52))
        mB = F.to_device(sk.encrypt_uint(mb, 32, nonce=(1 << 52) + 64))
        mR = torch.empty_like(mA)
        mR2 = torch.empty((1, 64, mA.shape[-1]), dtype=mA.dtype, device=mA.device)
        want = (int(ma[0]) * int(mb[0])) % (1 << 32)
        mul = latency(lambda: F.fhe_mul(ctx, mA, mB, mR, 1, 32, stream), args.mul_samples)
        assert sk.decrypt_uint(F.to_host(mR), 32)[0] == want
        mul.update(zip(("gates", "levels"), F.fhe_circuit_shape("mul", 32)[:2]))
        log(f"mul32 latency: {mul}")
        mul_tree = latency(lambda: F.fhe_mul_tree(ctx, mA, mB, mR, 1, 32, stream), args.mul_samples)
        assert sk.decrypt_uint(F.to_host(mR), 32)[0] == want
        mul_tree.update(zip(("gates", "levels"), F.fhe_circuit_shape("mul_tree", 32)[:2]))
        log(f"mul32 (tree accumulation) latency: {mul_tree}")
        mul_kara = latency(lambda: F.fhe_mul_karatsuba(ctx, mA, mB, mR2, 1, 32, stream), args.mul_samples)
        assert sk.decrypt_uint(F.to_host(mR2), 64)[0] == int(ma[0]) * int(mb[0])
        mul_kara.update(zip(("gates", "levels"), F.fhe_circuit_shape("karatsuba", 32)[:2]))
        mul_kara["product_bits"] = 64
        log(f"mul32 Karatsuba (64-bit product) latency: {mul_kara}")

    # latency of other circuits of the paper, one instance each: the 16-bit
    # adders (ripple carry, eqs. (1)-(2); full-adder gates; number-wise, GPU_n)
    # and the 4 x 4 16-bit matrix product by Cannon's algorithm
    circuits = None
    if args.circuit_samples > 0:
        ca = workloads.uniform_uints(13, 1, 16)
        cb = workloads.uniform_uints(14, 1, 16)
        cA = F.to_device(sk.encrypt_uint(ca, 16, nonce=(1 << 52) + 128))
        cB = F.to_device(sk.encrypt_uint(cb, 16, nonce=(1 << 52) + 160))
        cR = torch.empty_like(cA)
        rng = np.random.default_rng(15)
        MA = rng.integers(0, 1 << 16, (4, 4)).astype(np.uint64)
        MB = rng.integers(0, 1 << 16, (4, 4)).astype(np.uint64)
        dMA = F.to_device(sk.encrypt_uint(MA.reshape(-1), 16, nonce=(1 << 52) + 1024))
        dMB = F.to_device(sk.encrypt_uint(MB.reshape(-1), 16, nonce=(1 << 52) + 2048))
        dMC = torch.empty_like(dMA)
        cl = {"add16": (lambda: F.fhe_add(ctx, cA, cB, cR, 1, 16, stream), ("add", 16, 0)),
              "add16_full_adder_gates": (lambda: F.fhe_add_fa(ctx, cA, cB, cR, 1, 16, stream), ("add_fa", 16, 0)),
              "add16_numberwise": (lambda: F.fhe_add_numberwise(ctx, cA, cB, cR, 1, 16, stream),
                                   ("add_numberwise", 16, 0)),
              "matmul4x4_16": (lambda: F.fhe_matmul(ctx, dMA, dMB, dMC, 4, 16, stream), ("matmul", 16, 4))}
        circuits = {}
        for name, (fn, shape) in cl.items():
            r = latency(fn, args.circuit_samples)
            r.update(zip(("gates", "levels"), F.fhe_circuit_shape(shape[0], shape[1], shape[2])[:2]))
            circuits[name] = r
        assert sk.decrypt_uint(F.to_host(cR), 16)[0] == (int(ca[0]) + int(cb[0])) % (1 << 16)
        got = sk.decrypt_uint(F.to_host(dMC).reshape(16, 16, -1), 16).reshape(4, 4).astype(object)
        assert (got == (MA.astype(object) @ MB.astype(object)) % (1 << 16)).all()
        # the 1024 add16 pairs through full-adder gates (MAJ, XOR3): additions
        # per second against the two-input circuit's
        wl = workloads.AddWorkload()
        aA, aB, aR = add_cfg["dA"], add_cfg["dB"], add_cfg["dR"]
        fa = latency(lambda: F.fhe_add_fa(ctx, aA, aB, aR, wl.count, wl.width, stream), 1)
        assert add_cfg["verify"]()
        g_fa = F.fhe_circuit_shape("add_fa", wl.width)[0] * wl.count
        add_ms = legs["add16"]["ms_per_step"] if "add16" in legs else ms_per_step if args.config == "add16" else None
        circuits["add16_x1024_batched"] = {
            "two_input_gates": None if add_ms is None else {"ms": add_ms, "adds_per_s": round(wl.count / (add_ms / 1e3), 1)},
            "full_adder_gates": {"ms": fa["p50_ms"], "adds_per_s": round(wl.count / (fa["p50_ms"] / 1e3), 1),
                                 "gates": g_fa, "gates_per_s": round(g_fa / (fa["p50_ms"] / 1e3), 1)}}
        log(f"circuit latency: {circuits}")
    del add_cfg

    serving = None
    if args.serve_jobs > 0:
        log(f"serving: {args.serve_jobs} jobs at {args.serve_load:.2f} x {value:.0f} gates/s ({args.config})")
        serving = serving_leg(F, sk, ctx, args.serve_load * value, args.serve_jobs,
                              int(args.serve_budget_gib * (1 << 30)))
        serving["offered_as"] = f"{args.serve_load} x the batched {args.config} rate"
        log(f"serving: {serving}")
    if args.serve_jobs > 0 and args.small_budget_jobs > 0:
        log(f"serving under a {args.small_budget_mib:.0f} MiB budget: {args.small_budget_jobs} jobs")
        small = serving_leg(F, sk, ctx, args.serve_load * value, args.small_budget_jobs,
                            int(args.small_budget_mib * (1 << 20)), seed=5)
        serving["small_budget"] = small
        log(f"serving, small budget: {small}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        full = {"add16 x 1024": F.fhe_circuit_shape("add", 16)[0] * 1024,
                "mul32 x 256": F.fhe_circuit_shape("mul", 32)[0] * 256,
                "matvec 64x64": F.fhe_circuit_shape("matvec", 16, 64, 64)[0]}
        cpu = cpu_baseline(sk, args.config, args.cpu_sample_gates, args.cpu_single_gates, full)
        log(f"cpu baseline: {cpu}")

    cpu_par = None
    if not args.no_cpu_baseline and args.cpu_parallel_gates > 0:
        log("CPU parallel framework (Sec. IV)")
        cpu_par = cpu_parallel_leg(sk, ck, args.config, args.cpu_parallel_gates, value)
        log(f"CPU parallel framework: {cpu_par}")

    shape = res.pop("_shape")
    dtype = ("u32 (Torus32) / i32 residues mod two 28-bit primes (NTT)" if shape[2] == 1
             else "u32 (Torus32) / u64 (NTT mod 2^64-2^32+1)")
    line = {
        "metric": "bootstrapped gates/sec on 1 MI355X (batched vs plain) + p50/p99 latency per 32-bit mul",
        "value": round(value, 1), "unit": "gates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "graph_ms_per_step": None if graph_ms_per_step is None else round(graph_ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": main_cfg["workload"],
        "plain": plain, "mul32_latency": mul, "mul32_tree_latency": mul_tree,
        "mul32_karatsuba_latency": mul_kara, "batched_legs": legs, "circuit_latency": circuits,
        "goldilocks_ntt": goldilocks, "compound_gates": compound, "with_host_transfers": end_to_end,
        "serving": serving,
        "phase_ms_per_step": res["phase_ms_per_step"],
        "key_switch_roofline": res["key_switch_roofline"],
        "launch_shapes": {"tuned": tuning_s is not None, "tuning_s": tuning_s, "buckets": shapes,
                          "timed_by_shape": res["timed_by_shape"]},
        "roofline": res["roofline"], "valu_class_rates_tops": valu_rates,
        "cpu_baseline": cpu, "cpu_parallel_framework": cpu_par,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
