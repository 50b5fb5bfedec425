"""GPU parity of gate bootstrapping: the HIP path through the C ABI against the
CPU oracle, ciphertext word for ciphertext word (bit-exact: the NTT over
p = 2^64 - 2^32 + 1 is exact, so no tolerance applies)."""
import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads

pytestmark = pytest.mark.gpu
M32 = 1 << 32


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    sk, ck = F.fhe_keygen(0)
    ctx = F.Context(ck, 0)
    return sk, ctx, oracle.Keys(0)


def run_batch(ctx, ops, c0, c1):
    import torch
    d_ops = torch.from_numpy(np.asarray(ops, np.uint8).copy()).cuda()
    d0, d1 = F.to_device(c0), F.to_device(c1)
    out = torch.empty_like(d0)
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d0, d1, out, len(ops))
    torch.cuda.synchronize()
    return F.to_host(out)


def cmux_case(bk, abar, acc):
    got = F.fhe_debug_cmux(bk, abar, acc)
    want = oracle.cmux(bk, abar, acc)
    np.testing.assert_array_equal(got, want)


def test_cmux_random():
    g = np.random.default_rng(0)
    for abar in (1, 513, 1024, 2047):
        log(f"debug_cmux random abar={abar}")
        bk = g.integers(0, M32, (4, 2, 1024), dtype=np.uint64).astype(np.uint32)
        acc = g.integers(0, M32, (2, 1024), dtype=np.uint64).astype(np.uint32)
        cmux_case(bk, abar, acc)


def test_cmux_extreme_magnitudes():
    """All digits -512 (acc = 0xC0100400, abar = N gives D = -2 acc = -offset)
    against key words -2^31: every product coefficient reaches 2^52."""
    log("debug_cmux extreme")
    bk = np.full((4, 2, 1024), 0x80000000, np.uint32)
    acc = np.full((2, 1024), 0xC0100400, np.uint32)
    cmux_case(bk, 1024, acc)
    bk2 = np.full((4, 2, 1024), 0x7FFFFFFF, np.uint32)
    cmux_case(bk2, 1024, acc)
    acc3 = np.full((2, 1024), 0x3FEFFC00, np.uint32)  # digits +511 ... mixed signs
    cmux_case(bk, 1024, acc3)


def test_cmux_zero_rotation_and_zero_key():
    log("debug_cmux zero")
    g = np.random.default_rng(1)
    bk = g.integers(0, M32, (4, 2, 1024), dtype=np.uint64).astype(np.uint32)
    acc = g.integers(0, M32, (2, 1024), dtype=np.uint64).astype(np.uint32)
    cmux_case(bk, 0, acc)
    cmux_case(np.zeros_like(bk), 700, acc)


def test_truth_tables_bit_exact(env):
    sk, ctx, K = env
    a_bits, b_bits = workloads.truth_table_inputs()
    ops = np.repeat(np.arange(10, dtype=np.uint8), 4)
    A = np.tile(a_bits, 10)
    B = np.tile(b_bits, 10)
    c0 = sk.encrypt_bits(A, nonce=1000)
    c1 = sk.encrypt_bits(B, nonce=2000)
    np.testing.assert_array_equal(c0, K.encrypt_bits(A, nonce=1000))
    log("gate batch: 10 gates x 4 input pairs")
    got = run_batch(ctx, ops, c0, c1)
    want = K.bootstrap(ops, c0, c1)
    np.testing.assert_array_equal(got, want)
    truth = [[a & b, 1 - (a & b), a | b, 1 - (a | b), a ^ b, 1 - (a ^ b),
              (1 - a) & b, a & (1 - b), (1 - a) | b, a | (1 - b)][op]
             for op, a, b in zip(ops, A.astype(int), B.astype(int))]
    np.testing.assert_array_equal(sk.decrypt_bits(got), truth)


@pytest.mark.parametrize("count", [1, 3, 5, 9])
def test_ragged_batches(env, count):
    sk, ctx, K = env
    ops = workloads.gate_ops(100 + count, count)
    A = workloads.bits(200 + count, count)
    B = workloads.bits(300 + count, count)
    c0 = sk.encrypt_bits(A, nonce=10_000 * count)
    c1 = sk.encrypt_bits(B, nonce=10_000 * count + 5000)
    log(f"gate batch ragged count={count}")
    got = run_batch(ctx, ops, c0, c1)
    np.testing.assert_array_equal(got, K.bootstrap(ops, c0, c1))


def test_plain_path_nand(env):
    import torch
    sk, ctx, K = env
    a_bits, b_bits = workloads.truth_table_inputs()
    c0 = sk.encrypt_bits(a_bits, nonce=50_000)
    c1 = sk.encrypt_bits(b_bits, nonce=60_000)
    d0, d1 = F.to_device(c0), F.to_device(c1)
    out = torch.empty_like(d0)
    for g in range(4):
        log(f"plain NAND pair {g}")
        F.fhe_bootstrap_gate_plain(ctx, F.NAND, d0[g], d1[g], out[g])
    got = F.to_host(out)
    np.testing.assert_array_equal(got, K.bootstrap([F.NAND] * 4, c0, c1))
    np.testing.assert_array_equal(sk.decrypt_bits(got), [1, 1, 1, 0])


def test_empty_batch_and_repeat_determinism(env):
    import torch
    sk, ctx, K = env
    e = torch.empty((0, F.WORDS), dtype=torch.int32, device="cuda")
    ops0 = torch.empty(0, dtype=torch.uint8, device="cuda")
    F.fhe_bootstrap_gate_batch(ctx, ops0, e, e, e, 0)
    ops = workloads.gate_ops(7, 8)
    c0 = sk.encrypt_bits(workloads.bits(8, 8), nonce=70_000)
    c1 = sk.encrypt_bits(workloads.bits(9, 8), nonce=80_000)
    log("determinism: same batch twice")
    assert np.array_equal(run_batch(ctx, ops, c0, c1), run_batch(ctx, ops, c0, c1))
