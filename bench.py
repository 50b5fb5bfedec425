"""Benchmark: bootstrapped gates/s on one MI355X, batched vs plain, plus the
latency of one 32-bit multiplication.

One step = one batched 16-bit ripple-carry addition of 1024 encrypted pairs
(75,776 bootstrapped gates in 30 levels, each level one launch pair), with
inputs resident in HBM.  Prints one JSON line.

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


def cpu_baseline(sk, a, b, width, sample_gates):
    """The oracle on the host cores, on the first level of the same addition
    workload (independent XOR/AND gates of fresh inputs)."""
    import oracle
    K = oracle.Keys(0)
    ca = sk.encrypt_uint(a[: sample_gates], width, nonce=0)
    cb = sk.encrypt_uint(b[: sample_gates], width, nonce=1 << 40)
    ops, i0, i1 = [], [], []
    for c in range(sample_gates):
        for bit in range(width):
            for op in (4, 0):  # XOR, AND of (a_i, b_i)
                if len(ops) < sample_gates:
                    ops.append(op)
                    i0.append(ca[c, bit])
                    i1.append(cb[c, bit])
    threads = host_threads()
    t0 = time.perf_counter()
    K.bootstrap(ops, np.array(i0), np.array(i1), threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(len(ops) / dt, 3), "unit": "gates/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(ops)} gates of level 1 of the add16 workload (XOR/AND of fresh inputs), "
                      f"{dt:.1f} s on {threads} threads; per-gate work is identical on every level"}


JOB_GATES = None


def serving_leg(F, sk, ctx, rate_gates_per_s, n_jobs, budget_bytes, seed=3):
    """Poisson stream of mixed jobs (single gates, add16, add32, mul32, 8x8
    8-bit matvec) offered at rate_gates_per_s; every job is checked against
    plaintext arithmetic after the run."""
    import torch
    import workloads
    kinds = {"gate": (F.FHE_JOB_GATE, 1, 1), "add16": (F.FHE_JOB_ADD, 16, None), "add32": (F.FHE_JOB_ADD, 32, None),
             "mul32": (F.FHE_JOB_MUL, 32, None), "matvec8": (F.FHE_JOB_MATVEC, 8, None)}
    gates_of = {"gate": 1, "add16": F.fhe_circuit_shape("add", 16)[0], "add32": F.fhe_circuit_shape("add", 32)[0],
                "mul32": F.fhe_circuit_shape("mul", 32)[0], "matvec8": F.fhe_circuit_shape("matvec", 8, 8, 8)[0]}
    mean_gates = sum(p * gates_of[k] for k, p in zip(workloads.JOB_KINDS, workloads.JOB_MIX))
    jobs = workloads.job_stream(seed, n_jobs, rate_gates_per_s / mean_gates)
    prepared = []
    nonce = 1 << 56
    for j in jobs:
        kind, w, _ = kinds[j.kind]
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
    lat = {}
    bad = 0
    for p, t in zip(prepared, tickets):
        st, ms = F.fhe_serve_poll(srv, t)
        lat.setdefault(p["j"].kind, []).append(ms)
        host = F.to_host(p["out"])
        dec = sk.decrypt_bits(host) if p["kind"] == F.FHE_JOB_GATE else sk.decrypt_uint(host, p["w"])
        bad += list(dec) != list(p["want"])
    srv.close()
    if bad:
        raise SystemExit(f"bench: {bad} served jobs decrypted wrongly")
    total_gates = sum(gates_of[p["j"].kind] for p in prepared)
    return {"jobs": len(prepared), "gates": total_gates, "offered_gates_per_s": round(rate_gates_per_s, 1),
            "served_gates_per_s": round(total_gates / (t1 - t0), 1), "wall_s": round(t1 - t0, 2),
            "launches": stats["launches"], "hbm_budget_bytes": budget_bytes,
            "latency_ms": {k: {"p50": round(float(np.percentile(v, 50)), 1), "p99": round(float(np.percentile(v, 99)), 1),
                                "n": len(v)} for k, v in sorted(lat.items())}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="add16", choices=["add16", "mul32", "matvec"])
    ap.add_argument("--plain-reps", type=int, default=5)
    ap.add_argument("--mul-samples", type=int, default=5)
    ap.add_argument("--cpu-sample-gates", type=int, default=768)
    ap.add_argument("--tune-max-width", type=int, default=4096,
                    help="autotune launch shapes up to this batch width before warmup (0 keeps the defaults)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs in the serving leg (0 skips it)")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load of the serving leg as a fraction of the batched throughput")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--goldilocks-steps", type=int, default=1,
                    help="steps timed once more with the NTT over 2^64 - 2^32 + 1 (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the gates of a level are "
              "independent, so several GPUs would each take a share of every level", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_01945_amd as F
    import workloads

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

    if args.config == "add16":
        wl = workloads.AddWorkload()
        a, b = wl.operands()
        width, count = wl.width, wl.count
        ca, cb = sk.encrypt_uint(a, width, nonce=0), sk.encrypt_uint(b, width, nonce=1 << 40)
        dA, dB = F.to_device(ca), F.to_device(cb)
        dR = torch.empty_like(dA)
        step = lambda: F.fhe_add(ctx, dA, dB, dR, count, width, stream)
        gates, levels, _ = F.fhe_circuit_shape("add", width)
        expect = (a + b) % (1 << width)
        workload = {"workload": f"batched {width}-bit ripple-carry addition", "pairs": count,
                    "width": width, "gates_per_step": gates * count, "levels": levels}
    elif args.config == "mul32":
        wl = workloads.MulWorkload()
        a, b = wl.operands()
        width, count = wl.width, wl.count
        ca, cb = sk.encrypt_uint(a, width, nonce=0), sk.encrypt_uint(b, width, nonce=1 << 40)
        dA, dB = F.to_device(ca), F.to_device(cb)
        dR = torch.empty_like(dA)
        step = lambda: F.fhe_mul(ctx, dA, dB, dR, count, width, stream)
        gates, levels, _ = F.fhe_circuit_shape("mul", width)
        expect = (a * b) % (1 << width)
        workload = {"workload": f"batched {width}-bit shift-and-add multiplication", "pairs": count,
                    "width": width, "gates_per_step": gates * count, "levels": levels}
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
        count = 1
        expect = (M @ x) % (1 << width)
        workload = {"workload": f"encrypted {wl.rows}x{wl.cols} matrix-vector product, {width}-bit",
                    "rows": wl.rows, "cols": wl.cols, "width": width, "gates_per_step": gates, "levels": levels}
    gates_per_step = gates * count

    log(f"config {args.config}: {gates_per_step} gates/step, {levels} levels; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    F.fhe_ctx_timing(ctx)  # drop anything recorded so far
    F.fhe_ctx_set_timing(ctx, True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    F.fhe_ctx_set_timing(ctx, False)
    records = F.fhe_ctx_timing_launches(ctx)
    br_ms = sum(r["blind_rotate_ms"] for r in records)
    ks_ms = sum(r["key_switch_ms"] for r in records)
    launches = len(records)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = gates_per_step / (ms_per_step / 1e3)
    log(f"{ms_per_step:.1f} ms/step, {value:.0f} gates/s; blind rotation {br_ms:.1f} ms, "
        f"key switch {ks_ms:.1f} ms over {launches} launches")

    # the same steps replayed from the captured HIP graphs (timing off)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    graph_ms_per_step = (time.perf_counter() - g0) * 1e3 / args.steps
    log(f"graph replay: {graph_ms_per_step:.1f} ms/step")

    # one step with the inputs copied in from pinned host memory and the
    # results copied out (the PCIe-inclusive rate; not `value`)
    hA = dA.cpu().pin_memory()
    hB = dB.cpu().pin_memory()
    hR = torch.empty(dR.shape, dtype=dR.dtype).pin_memory()
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    dA.copy_(hA, non_blocking=True)
    dB.copy_(hB, non_blocking=True)
    step()
    hR.copy_(dR, non_blocking=True)
    torch.cuda.synchronize()
    e2e_ms = (time.perf_counter() - e0) * 1e3
    end_to_end = {"gates_per_s": round(gates_per_step / (e2e_ms / 1e3), 1), "ms_per_step": round(e2e_ms, 1),
                  "bytes_in": int(hA.numel() + hB.numel()) * 4, "bytes_out": int(hR.numel()) * 4}
    log(f"with host transfers: {end_to_end}")

    got = sk.decrypt_uint(F.to_host(dR), width)
    if not np.array_equal(got, np.asarray(expect).reshape(-1).astype(np.uint64)):
        raise SystemExit("bench: decrypted results differ from plaintext arithmetic")

    # roofline of the dominant kernel (the blind-rotation shape with the most
    # device time in the timed region), from its launches there
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
    dtype = ("u32 (Torus32) / i32 residues mod two 28-bit primes (NTT)" if shape[2] == 1
             else "u32 (Torus32) / u64 (NTT mod 2^64-2^32+1)")
    kernel = f"k_blind_rotate_pair<{shape[2]}>" if shape[0] == 2 else f"k_blind_rotate<{shape[1]}, {shape[2]}>"
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(kernel, gates_per_launch),
                "kernel": kernel, "launches": dom["launches"], "avg_launch_ms": round(avg_launch_ms, 3),
                "gates_per_launch": round(gates_per_launch, 1)}
    per_shape = {f"{k[0]}x{k[1]}/arith{k[2]}": {"launches": v["launches"], "gates": v["gates"], "ms": round(v["ms"], 3)}
                 for k, v in sorted(by_shape.items())}

    # the same step with the NTT over the Goldilocks prime 2^64 - 2^32 + 1 (one
    # wave per gate, four gates per workgroup), against its own algorithmic
    # count; then the tuned shapes are put back
    goldilocks = None
    if args.goldilocks_steps > 0:
        saved = [F.fhe_ctx_launch_config(ctx, 1 << b) for b in range(16)]
        F.fhe_ctx_set_launch_config(ctx, 1, 1 << 31, (1, 4, 0))
        step()
        torch.cuda.synchronize()
        F.fhe_ctx_timing(ctx)
        F.fhe_ctx_set_timing(ctx, True)
        gs0 = time.perf_counter()
        for _ in range(args.goldilocks_steps):
            step()
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - gs0) * 1e3 / args.goldilocks_steps
        F.fhe_ctx_set_timing(ctx, False)
        grec = [r for r in F.fhe_ctx_timing_launches(ctx) if r["shape"] == (1, 4, 0)]
        g_gates = sum(r["gates"] for r in grec)
        g_br = sum(r["blind_rotate_ms"] for r in grec)
        g_ach = LANE_OPS_PER_GATE[0] * g_gates / (g_br / 1e3) / 1e12
        goldilocks = {"gates_per_s": round(gates_per_step / (g_ms / 1e3), 1), "ms_per_step": round(g_ms, 1),
                      "kernel": "k_blind_rotate<4, 0>", "achieved": round(g_ach, 3), "peak": round(VALU_PEAK_TOPS, 2),
                      "unit": "TOP/s", "frac": round(g_ach / VALU_PEAK_TOPS, 4)}
        for b, shp in enumerate(saved):
            F.fhe_ctx_set_launch_config(ctx, 1 << b, 1 << b, shp)
        if not np.array_equal(sk.decrypt_uint(F.to_host(dR), width), np.asarray(expect).reshape(-1).astype(np.uint64)):
            raise SystemExit("bench: Goldilocks-path results differ from plaintext arithmetic")
        log(f"Goldilocks NTT: {goldilocks}")

    if args.copy_calibration_mib > 0:
        src = torch.empty(args.copy_calibration_mib << 18, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: {args.copy_calibration_mib} MiB read + written")

    # plain path: one gate per launch, synchronous
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
                 "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3), "gates": len(lat)}
        log(f"plain: {plain}")

    # latency of one 32-bit multiplication: shift-and-add (120 levels) and with
    # the partial products summed by a tree (62 levels), same 2,824 gates
    mul = mul_tree = mul_kara = None
    if args.mul_samples > 0:
        ma = workloads.uniform_uints(11, 1, 32)
        mb = workloads.uniform_uints(12, 1, 32)
        mA = F.to_device(sk.encrypt_uint(ma, 32, nonce=1 << 52))
        mB = F.to_device(sk.encrypt_uint(mb, 32, nonce=(1 << 52) + 64))
        mR = torch.empty_like(mA)

        def mul_latency(fn, kind):
            fn(ctx, mA, mB, mR, 1, 32, stream)
            torch.cuda.synchronize()
            ml = []
            for _ in range(args.mul_samples):
                s0 = time.perf_counter()
                fn(ctx, mA, mB, mR, 1, 32, stream)
                torch.cuda.synchronize()
                ml.append(time.perf_counter() - s0)
            assert sk.decrypt_uint(F.to_host(mR), 32)[0] == (int(ma[0]) * int(mb[0])) % (1 << 32)
            gates, levels, _ = F.fhe_circuit_shape(kind, 32)
            return {"p50_ms": round(1e3 * float(np.median(ml)), 1),
                    "p99_ms": round(1e3 * float(np.percentile(ml, 99)), 1),
                    "samples": len(ml), "gates": gates, "levels": levels}

        mul = mul_latency(F.fhe_mul, "mul")
        log(f"mul32 latency: {mul}")
        mul_tree = mul_latency(F.fhe_mul_tree, "mul_tree")
        log(f"mul32 (tree accumulation) latency: {mul_tree}")
        # Karatsuba (Sec. III-B-2): all 64 bits of the product
        mR2 = torch.empty((1, 64, mA.shape[-1]), dtype=mA.dtype, device=mA.device)
        F.fhe_mul_karatsuba(ctx, mA, mB, mR2, 1, 32, stream)
        torch.cuda.synchronize()
        kl = []
        for _ in range(args.mul_samples):
            s0 = time.perf_counter()
            F.fhe_mul_karatsuba(ctx, mA, mB, mR2, 1, 32, stream)
            torch.cuda.synchronize()
            kl.append(time.perf_counter() - s0)
        assert sk.decrypt_uint(F.to_host(mR2), 64)[0] == int(ma[0]) * int(mb[0])
        kg, klv, _ = F.fhe_circuit_shape("karatsuba", 32)
        mul_kara = {"p50_ms": round(1e3 * float(np.median(kl)), 1), "p99_ms": round(1e3 * float(np.percentile(kl, 99)), 1),
                    "samples": len(kl), "gates": kg, "levels": klv, "product_bits": 64}
        log(f"mul32 Karatsuba (64-bit product) latency: {mul_kara}")

    # latency of other circuits of the paper, one instance each: the 16-bit
    # adders (ripple carry, eqs. (1)-(2); number-wise, GPU_n) and the 4 x 4
    # 16-bit matrix product by Cannon's algorithm
    circuits = None
    if args.mul_samples > 0:
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
        legs = {"add16": (lambda: F.fhe_add(ctx, cA, cB, cR, 1, 16, stream), ("add", 16, 0)),
                "add16_full_adder_gates": (lambda: F.fhe_add_fa(ctx, cA, cB, cR, 1, 16, stream), ("add_fa", 16, 0)),
                "add16_numberwise": (lambda: F.fhe_add_numberwise(ctx, cA, cB, cR, 1, 16, stream),
                                     ("add_numberwise", 16, 0)),
                "matmul4x4_16": (lambda: F.fhe_matmul(ctx, dMA, dMB, dMC, 4, 16, stream), ("matmul", 16, 4))}
        circuits = {}
        for name, (fn, shape) in legs.items():
            fn()
            torch.cuda.synchronize()
            tl = []
            for _ in range(args.mul_samples):
                s0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                tl.append(time.perf_counter() - s0)
            g, lv, _ = F.fhe_circuit_shape(shape[0], shape[1], shape[2])
            circuits[name] = {"p50_ms": round(1e3 * float(np.median(tl)), 1), "gates": g, "levels": lv}
        assert sk.decrypt_uint(F.to_host(cR), 16)[0] == (int(ca[0]) + int(cb[0])) % (1 << 16)
        got = sk.decrypt_uint(F.to_host(dMC).reshape(16, 16, -1), 16).reshape(4, 4).astype(object)
        assert (got == (MA.astype(object) @ MB.astype(object)) % (1 << 16)).all()
        log(f"circuit latency: {circuits}")
        if args.config == "add16":
            # the benchmark's 1024 add16 pairs through full-adder gates (MAJ,
            # XOR3): additions per second against the two-input circuit's
            F.fhe_add_fa(ctx, dA, dB, dR, count, width, stream)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            F.fhe_add_fa(ctx, dA, dB, dR, count, width, stream)
            torch.cuda.synchronize()
            fa_s = time.perf_counter() - s0
            assert (sk.decrypt_uint(F.to_host(dR), width) == (wl.operands()[0] + wl.operands()[1]) % (1 << width)).all()
            g_fa = F.fhe_circuit_shape("add_fa", width)[0] * count
            circuits["add16_x1024_batched"] = {
                "two_input_gates": {"ms": round(ms_per_step, 1), "adds_per_s": round(count / (ms_per_step / 1e3), 1)},
                "full_adder_gates": {"ms": round(1e3 * fa_s, 1), "adds_per_s": round(count / fa_s, 1),
                                     "gates": g_fa, "gates_per_s": round(g_fa / fa_s, 1)}}
            log(f"add16 x 1024 batched: {circuits['add16_x1024_batched']}")

    serving = None
    if args.serve_jobs > 0:
        log(f"serving: {args.serve_jobs} jobs at {args.serve_load:.2f} x {value:.0f} gates/s")
        serving = serving_leg(F, sk, ctx, args.serve_load * value, args.serve_jobs,
                              int(args.serve_budget_gib * (1 << 30)))
        log(f"serving: {serving}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(sk, workloads.AddWorkload().operands()[0], workloads.AddWorkload().operands()[1],
                           16, args.cpu_sample_gates)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "bootstrapped gates/sec on 1 MI355X (batched vs plain) + p50/p99 latency per 32-bit mul",
        "value": round(value, 1), "unit": "gates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "graph_ms_per_step": round(graph_ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": workload,
        "plain": plain, "mul32_latency": mul, "mul32_tree_latency": mul_tree,
        "mul32_karatsuba_latency": mul_kara, "circuit_latency": circuits, "goldilocks_ntt": goldilocks,
        "with_host_transfers": end_to_end,
        "serving": serving,
        "phase_ms_per_step": {"blind_rotate": round(br_ms / args.steps, 3), "key_switch": round(ks_ms / args.steps, 3)},
        "launch_shapes": {"tuned": tuning_s is not None, "tuning_s": tuning_s, "buckets": shapes,
                          "timed_by_shape": per_shape},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
