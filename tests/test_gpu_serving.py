"""Serving (continuous batching): every job's output is byte-identical alone
and in a mix, equal to the same job run through its own entry point and to
the oracle, decrypts to the plaintext result, and admission respects the HBM
budget (queueing when full, refusing what can never fit)."""
import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    sk, ck = F.fhe_keygen(0)
    return sk, F.Context(ck, 0)


def make_jobs(sk):
    """A small mix: two gates, an add16, an add32, a mul8 (shift-and-add and
    tree accumulation), 8-bit additions with full-adder gates and number-wise,
    a 6-bit Karatsuba product, a 2x3 4-bit matvec and a 2x2 3-bit matmul."""
    import torch
    jobs = []
    nonce = 3_000_000
    for k, op in enumerate([F.NAND, F.XOR]):
        a = sk.encrypt_bits([k & 1], nonce=nonce); nonce += 1
        b = sk.encrypt_bits([1], nonce=nonce); nonce += 1
        jobs.append(dict(kind=F.FHE_JOB_GATE, op=op, a=a, b=b, shape=(1, F.WORDS),
                         want=[[1 - (k & 1), (k & 1) ^ 1][k]], width=1))
    for kind, w, x, y in [(F.FHE_JOB_ADD, 16, 51234, 40000), (F.FHE_JOB_ADD, 32, 4000000000, 500000000),
                          (F.FHE_JOB_MUL, 8, 201, 77), (F.FHE_JOB_MUL_TREE, 8, 201, 77),
                          (F.FHE_JOB_ADD_FA, 8, 200, 99), (F.FHE_JOB_ADD_NUMBERWISE, 8, 255, 1),
                          (F.FHE_JOB_KARATSUBA, 6, 61, 45)]:
        a = sk.encrypt_uint([x], w, nonce=nonce); nonce += w
        b = sk.encrypt_uint([y], w, nonce=nonce); nonce += w
        if kind in (F.FHE_JOB_ADD, F.FHE_JOB_ADD_FA, F.FHE_JOB_ADD_NUMBERWISE):
            res, ow = (x + y) % (1 << w), w
        elif kind == F.FHE_JOB_KARATSUBA:
            res, ow = x * y, 2 * w
        else:
            res, ow = (x * y) % (1 << w), w
        jobs.append(dict(kind=kind, op=0, a=a, b=b, shape=(ow, F.WORDS), want=[res], width=w, out_width=ow))
    M = np.array([[3, 9, 15], [7, 1, 12]], np.uint64)
    v = np.array([5, 11, 2], np.uint64)
    a = sk.encrypt_uint(M.reshape(-1), 4, nonce=nonce); nonce += 24
    b = sk.encrypt_uint(v, 4, nonce=nonce); nonce += 12
    jobs.append(dict(kind=F.FHE_JOB_MATVEC, op=0, a=a, b=b, shape=(2, 4, F.WORDS), want=list((M @ v) % 16),
                     width=4, rows=2, cols=3))
    A = np.array([[5, 7], [2, 6]], np.uint64)
    B = np.array([[3, 1], [4, 7]], np.uint64)
    a = sk.encrypt_uint(A.reshape(-1), 3, nonce=nonce); nonce += 12
    b = sk.encrypt_uint(B.reshape(-1), 3, nonce=nonce); nonce += 12
    jobs.append(dict(kind=F.FHE_JOB_MATMUL, op=0, a=a, b=b, shape=(4, 3, F.WORDS),
                     want=list(((A @ B) % 8).reshape(-1)), width=3, rows=2))
    for j in jobs:
        j["da"], j["db"] = F.to_device(j["a"]), F.to_device(j["b"])
    torch.cuda.synchronize()
    return jobs


def submit(srv, j, out):
    return F.fhe_serve_submit(srv, j["kind"], j["da"], j["db"], out, op=j["op"], width=j["width"],
                              rows=j.get("rows", 0), cols=j.get("cols", 0))


def test_alone_equals_mix_and_decrypts(env):
    import torch
    sk, ctx = env
    jobs = make_jobs(sk)
    srv = F.Server(ctx, 1 << 30)
    try:
        alone = []
        for j in jobs:
            out = torch.zeros(j["shape"], dtype=torch.int32, device="cuda")
            log(f"serving alone: kind {j['kind']} width {j['width']}")
            t = submit(srv, j, out)
            F.fhe_serve_wait(srv, t, 300)
            st, lat = F.fhe_serve_poll(srv, t)
            assert st == F.FHE_JOB_DONE and lat > 0
            q, v = F.fhe_serve_job_times(srv, t)
            assert q >= 0 and v > 0 and abs(q + v - lat) < 1e-6 * max(lat, 1.0) + 1e-3
            alone.append(F.to_host(out))
        outs = [torch.zeros(j["shape"], dtype=torch.int32, device="cuda") for j in jobs]
        log("serving: all jobs in one mix")
        tickets = [submit(srv, j, o) for j, o in zip(jobs, outs)]
        for t in tickets:
            F.fhe_serve_wait(srv, t, 300)
        for j, o, a in zip(jobs, outs, alone):
            got = F.to_host(o)
            np.testing.assert_array_equal(got, a)
            dec = sk.decrypt_uint(got, j.get("out_width", j["width"])) if j["kind"] != F.FHE_JOB_GATE \
                else sk.decrypt_bits(got)
            assert list(dec) == list(j["want"]), (j["kind"], list(dec), j["want"])
        stats = F.fhe_serve_stats(srv)
        assert stats["jobs_done"] == 2 * len(jobs) and stats["pool_bytes_in_use"] == 0
    finally:
        srv.close()
    # The server runs its own slot layout and level order; a gate's words do
    # not depend on either, so every served job must give the words of its
    # direct entry point and of the oracle.
    K = oracle.Keys(0)
    for j, a in zip(jobs, alone):
        log(f"served job kind {j['kind']} width {j['width']}: direct entry point and oracle")
        np.testing.assert_array_equal(a, direct_run(ctx, j))
        np.testing.assert_array_equal(a.reshape(-1, F.WORDS), oracle_run(K, j).reshape(-1, F.WORDS))


def direct_run(ctx, j):
    """The job through its own entry point (no server)."""
    import torch
    out = torch.zeros(j["shape"], dtype=torch.int32, device="cuda")
    k, w, da, db = j["kind"], j["width"], j["da"], j["db"]
    if k == F.FHE_JOB_GATE:
        ops = torch.tensor([j["op"]], dtype=torch.uint8, device="cuda")
        F.fhe_bootstrap_gate_batch(ctx, ops, da, db, out, 1)
    elif k == F.FHE_JOB_MATVEC:
        F.fhe_matvec(ctx, da, db, out, j["rows"], j["cols"], w)
    elif k == F.FHE_JOB_MATMUL:
        F.fhe_matmul(ctx, da, db, out, j["rows"], w)
    else:
        fn = {F.FHE_JOB_ADD: F.fhe_add, F.FHE_JOB_MUL: F.fhe_mul, F.FHE_JOB_MUL_TREE: F.fhe_mul_tree,
              F.FHE_JOB_ADD_FA: F.fhe_add_fa, F.FHE_JOB_ADD_NUMBERWISE: F.fhe_add_numberwise,
              F.FHE_JOB_KARATSUBA: F.fhe_mul_karatsuba}[k]
        fn(ctx, da, db, out, 1, w)
    torch.cuda.synchronize()
    return F.to_host(out)


def oracle_run(K, j):
    k, w, a, b = j["kind"], j["width"], j["a"], j["b"]
    if k == F.FHE_JOB_GATE:
        return K.bootstrap([j["op"]], a, b)
    if k == F.FHE_JOB_MATVEC:
        return K.matvec(a, b, j["rows"], j["cols"], w)
    if k == F.FHE_JOB_MATMUL:
        return K.matmul(a, b, j["rows"], w)
    fn = {F.FHE_JOB_ADD: K.add, F.FHE_JOB_MUL: K.mul, F.FHE_JOB_MUL_TREE: K.mul_tree, F.FHE_JOB_ADD_FA: K.add_fa,
          F.FHE_JOB_ADD_NUMBERWISE: K.add_numberwise, F.FHE_JOB_KARATSUBA: K.karatsuba}[k]
    return fn(a.reshape(1, w, -1), b.reshape(1, w, -1), w)


def test_small_budget_queues_and_refuses(env):
    import torch
    sk, ctx = env
    jobs = make_jobs(sk)
    add32 = jobs[3]
    need = (2 * 32 + F.fhe_circuit_shape("add", 32)[0]) * F.WORDS * 4
    srv = F.Server(ctx, need + 1000)  # room for one add32 at a time
    try:
        outs = [torch.zeros(add32["shape"], dtype=torch.int32, device="cuda") for _ in range(3)]
        log("serving: three add32 jobs through a budget that holds one")
        tickets = [submit(srv, add32, o) for o in outs]
        states = [F.fhe_serve_poll(srv, t)[0] for t in tickets]
        assert states.count(F.FHE_JOB_RUNNING) <= 1
        for t in tickets:
            F.fhe_serve_wait(srv, t, 300)
        ref = F.to_host(outs[0])
        for o in outs[1:]:
            np.testing.assert_array_equal(F.to_host(o), ref)
        matvec = next(j for j in jobs if j["kind"] == F.FHE_JOB_MATVEC)  # larger than the budget
        with pytest.raises(F.FheError) as e:
            submit(srv, matvec, torch.zeros(matvec["shape"], dtype=torch.int32, device="cuda"))
        assert e.value.code == F.FHE_EBUSY
    finally:
        srv.close()


def test_cancel_queued_job(env):
    import torch
    sk, ctx = env
    jobs = make_jobs(sk)
    add32 = jobs[3]
    need = (2 * 32 + F.fhe_circuit_shape("add", 32)[0]) * F.WORDS * 4
    srv = F.Server(ctx, need + 1000)
    try:
        o1 = torch.zeros(add32["shape"], dtype=torch.int32, device="cuda")
        o2 = torch.zeros(add32["shape"], dtype=torch.int32, device="cuda")
        t1 = submit(srv, add32, o1)
        t2 = submit(srv, add32, o2)
        F.fhe_serve_cancel(srv, t2)
        F.fhe_serve_wait(srv, t1, 300)
        with pytest.raises(F.FheError) as e:
            F.fhe_serve_wait(srv, t2, 300)
        assert e.value.code == F.FHE_ECANCELED
        assert F.fhe_serve_stats(srv)["pool_bytes_in_use"] == 0
    finally:
        srv.close()


def test_device_allocation_failure_is_enomem(env):
    """A server whose HBM budget exceeds the device (400 GiB against 288 GB)
    fails with FHE_ENOMEM from its pool allocation, and the context keeps
    working: a gate batch afterwards is bit-exact with the oracle."""
    import torch
    sk, ctx = env
    with pytest.raises(F.FheError) as e:
        F.Server(ctx, 400 << 30)
    assert e.value.code == F.FHE_ENOMEM
    a, b = workloads.truth_table_inputs()
    c0, c1 = sk.encrypt_bits(a, nonce=3_900_000), sk.encrypt_bits(b, nonce=3_900_100)
    ops = torch.tensor([F.NAND, F.XOR, F.AND, F.OR], dtype=torch.uint8, device="cuda")
    d0, d1 = F.to_device(c0), F.to_device(c1)
    out = torch.empty_like(d0)
    F.fhe_bootstrap_gate_batch(ctx, ops, d0, d1, out, 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(F.to_host(out), oracle.Keys(0).bootstrap([F.NAND, F.XOR, F.AND, F.OR], c0, c1))
