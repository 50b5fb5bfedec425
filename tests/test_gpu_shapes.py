"""Launch shapes and the autotuner: every blind-rotation shape (one wave per
gate with 1, 2, 4 or 8 gates per workgroup, or two or four waves per gate;
NTT over the Goldilocks prime or modulo two 28-bit primes) gives the
oracle's words bit for bit, and the tuner only ever stores such shapes."""
import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads

pytestmark = pytest.mark.gpu
WIDEST = 1 << 31


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    sk, ck = F.fhe_keygen(0)
    return sk, F.Context(ck, 0), oracle.Keys(0)


def run_batch(ctx, ops, c0, c1):
    import torch
    d_ops = torch.from_numpy(np.asarray(ops, np.uint8).copy()).cuda()
    d0, d1 = F.to_device(c0), F.to_device(c1)
    out = torch.empty_like(d0)
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d0, d1, out, len(ops))
    torch.cuda.synchronize()
    return F.to_host(out)


def test_every_shape_bit_exact(env):
    """9 gates (a ragged last workgroup for 2 and 4 gates per group), all ten
    gate codes, fresh inputs."""
    sk, ctx, K = env
    n = 9
    ops = workloads.gate_ops(70, n)
    c0 = sk.encrypt_bits(workloads.bits(71, n), nonce=5_000_000)
    c1 = sk.encrypt_bits(workloads.bits(72, n), nonce=5_100_000)
    want = K.bootstrap(ops, c0, c1, threads=8)
    try:
        for shape in F.SHAPES:
            F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, shape)
            assert F.fhe_ctx_launch_config(ctx, n) == shape
            log(f"{n} gates, shape {shape}")
            np.testing.assert_array_equal(run_batch(ctx, ops, c0, c1), want)
    finally:
        F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, (1, 4, 0))


@pytest.mark.parametrize("shape", [(2, 1, 0), (2, 1, 1), (1, 4, 1), (4, 1, 1)])
def test_shape_on_circuit_output(env, shape):
    """Gates whose inputs are themselves gate outputs (noisier, key-switched
    samples), against the oracle."""
    sk, ctx, K = env
    n = 6
    ops = workloads.gate_ops(73, n)
    c0 = K.bootstrap(workloads.gate_ops(74, n), sk.encrypt_bits(workloads.bits(75, n), nonce=5_200_000),
                     sk.encrypt_bits(workloads.bits(76, n), nonce=5_300_000), threads=8)
    c1 = sk.encrypt_bits(workloads.bits(77, n), nonce=5_400_000)
    want = K.bootstrap(ops, c0, c1, threads=8)
    try:
        F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, shape)
        log(f"{n} gates on gate outputs, shape {shape}")
        np.testing.assert_array_equal(run_batch(ctx, ops, c0, c1), want)
    finally:
        F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, (1, 4, 0))


def test_shape_ranges_and_errors(env):
    _, ctx, _ = env
    F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, (1, 4, 0))
    F.fhe_ctx_set_launch_config(ctx, 1, 8, (2, 1, 1))
    assert [F.fhe_ctx_launch_config(ctx, w) for w in (1, 5, 8, 9, 1 << 20)] == \
        [(2, 1, 1), (2, 1, 1), (2, 1, 1), (1, 4, 0), (1, 4, 0)]
    for bad in [(1, 3, 0), (2, 2, 0), (3, 1, 0), (0, 1, 0), (1, 4, 2), (4, 1, 0), (4, 2, 1)]:
        with pytest.raises(F.FheError):
            F.fhe_ctx_set_launch_config(ctx, 1, 4, bad)
    with pytest.raises(F.FheError):
        F.fhe_ctx_set_launch_config(ctx, 5, 4, (1, 1, 0))
    with pytest.raises(F.FheError):
        F.fhe_ctx_launch_config(ctx, 0)
    F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, (1, 4, 0))


def test_autotune_then_circuit(env):
    """The tuner stores a valid shape in every bucket, and a circuit replayed
    from a graph captured before tuning is recaptured with the new shapes and
    gives the same words."""
    import torch
    sk, ctx, _ = env
    w, count = 4, 3
    a = workloads.uniform_uints(78, count, w)
    b = workloads.uniform_uints(79, count, w)
    dA = F.to_device(sk.encrypt_uint(a, w, nonce=5_500_000))
    dB = F.to_device(sk.encrypt_uint(b, w, nonce=5_600_000))
    F.fhe_ctx_set_graphs(ctx, True)
    before = torch.empty_like(dA)
    log("add4 x 3 before tuning")
    F.fhe_add(ctx, dA, dB, before, count, w)
    torch.cuda.synchronize()
    log("autotune up to 16 gates")
    F.fhe_ctx_autotune(ctx, 16, 1)
    shapes = [F.fhe_ctx_launch_config(ctx, 1 << b) for b in range(16)]
    assert all(s in F.SHAPES for s in shapes)
    assert all(s == shapes[4] for s in shapes[4:])  # wider buckets take the widest measured one's
    after = torch.empty_like(dA)
    log("add4 x 3 after tuning")
    F.fhe_add(ctx, dA, dB, after, count, w)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(F.to_host(after), F.to_host(before))
    np.testing.assert_array_equal(sk.decrypt_uint(F.to_host(after), w), (a + b) % (1 << w))
    F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, (1, 4, 0))
