"""Captured level schedules: a circuit replayed from its HIP graph gives the
same words as the eager launches, on every replay, with eager work and
synchronizations in between; a graph is recaptured when the scratch buffer it
refers to moves."""
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


def test_graph_replays_match_eager(env):
    import torch
    sk, ctx = env
    w, count = 5, 3
    a = workloads.uniform_uints(90, count, w)
    b = workloads.uniform_uints(91, count, w)
    ca, cb = sk.encrypt_uint(a, w, nonce=4_000_000), sk.encrypt_uint(b, w, nonce=4_100_000)
    dA, dB = F.to_device(ca), F.to_device(cb)
    eager = torch.empty_like(dA)
    F.fhe_ctx_set_graphs(ctx, False)
    log("add5 x 3 eager")
    F.fhe_add(ctx, dA, dB, eager, count, w)
    torch.cuda.synchronize()
    want = F.to_host(eager)
    np.testing.assert_array_equal(want, oracle.Keys(0).add(ca, cb, w))
    F.fhe_ctx_set_graphs(ctx, True)
    out = torch.empty_like(dA)
    for rep in range(3):
        out.zero_()
        log(f"add5 x 3 graph replay {rep}")
        F.fhe_add(ctx, dA, dB, out, count, w)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(F.to_host(out), want)
        # eager work between replays
        F.fhe_ctx_set_graphs(ctx, False)
        F.fhe_mul(ctx, dA, dB, eager, count, w)
        torch.cuda.synchronize()
        F.fhe_ctx_set_graphs(ctx, True)
    np.testing.assert_array_equal(sk.decrypt_uint(want, w), (a + b) % (1 << w))


def test_graph_recaptured_after_scratch_grows(env):
    import torch
    sk, ctx = env
    w = 3
    a = workloads.uniform_uints(92, 2, w)
    b = workloads.uniform_uints(93, 2, w)
    dA = F.to_device(sk.encrypt_uint(a, w, nonce=4_200_000))
    dB = F.to_device(sk.encrypt_uint(b, w, nonce=4_300_000))
    out = torch.empty_like(dA)
    F.fhe_ctx_set_graphs(ctx, True)
    F.fhe_mul(ctx, dA, dB, out, 2, w)
    torch.cuda.synchronize()
    first = F.to_host(out)
    # a batch wider than any seen so far reallocates the scratch buffer
    n = 9000
    log(f"gate batch of {n} (scratch grows)")
    ops = torch.full((n,), F.XOR, dtype=torch.uint8, device="cuda")
    bits = F.to_device(sk.encrypt_bits(workloads.bits(94, n), nonce=4_400_000))
    big_out = torch.empty_like(bits)
    F.fhe_bootstrap_gate_batch(ctx, ops, bits, bits, big_out, n)
    torch.cuda.synchronize()
    out.zero_()
    log("mul3 graph after scratch growth")
    F.fhe_mul(ctx, dA, dB, out, 2, w)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(F.to_host(out), first)
    np.testing.assert_array_equal(sk.decrypt_uint(first, w), (a * b) % (1 << w))
    # XOR of a bit with itself is 0
    assert not sk.decrypt_bits(F.to_host(big_out)).any()
