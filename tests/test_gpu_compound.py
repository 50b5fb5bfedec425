"""Compound gates (two symmetric gates of the same inputs from one blind
rotation), the compound ripple-carry adder, the reporting of invalid gate
codes, and calls on two streams, all through the C ABI against the oracle
(bit-exact) or against single-stream results."""
import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads
from sampled import check_sampled_levels

pytestmark = pytest.mark.gpu
SYM = [F.AND, F.NAND, F.OR, F.NOR, F.XOR, F.XNOR]
WIDEST = 1 << 31


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    sk, ck = F.fhe_keygen(0)
    return sk, F.Context(ck, 0), oracle.Keys(0)


def truth(op, a, b):
    a, b = np.asarray(a, int), np.asarray(b, int)
    return np.array([a & b, 1 - (a & b), a | b, 1 - (a | b), a ^ b, 1 - (a ^ b)])[op]


def run_compound(ctx, ops0, ops1, c0, c1, stream=None):
    import torch
    d_o0 = torch.from_numpy(np.asarray(ops0, np.uint8).copy()).cuda()
    d_o1 = torch.from_numpy(np.asarray(ops1, np.uint8).copy()).cuda()
    d0, d1 = F.to_device(c0), F.to_device(c1)
    out0, out1 = torch.empty_like(d0), torch.empty_like(d0)
    F.fhe_bootstrap_compound_batch(ctx, d_o0, d_o1, d0, d1, out0, out1, len(ops0), stream)
    torch.cuda.synchronize()
    return F.to_host(out0), F.to_host(out1)


def oracle_compound(K, ops0, ops1, c0, c1):
    ops = np.stack([ops0, ops1], axis=1).astype(np.uint8)
    out = K.bootstrap_compound(ops, c0, c1)
    return out[:, 0], out[:, 1]


def all_pairs():
    """Every ordered pair of symmetric codes on each of the four input pairs."""
    o0, o1, a, b = [], [], [], []
    for x in SYM:
        for y in SYM:
            for u in (0, 1):
                for v in (0, 1):
                    o0.append(x); o1.append(y); a.append(u); b.append(v)
    return (np.array(o0, np.uint8), np.array(o1, np.uint8), np.array(a, np.uint8), np.array(b, np.uint8))


def test_compound_every_code_pair_bit_exact(env):
    """36 code pairs x 4 input pairs (144 compound gates, 288 outputs):
    bit-exact against the oracle, every output decrypting to its gate."""
    sk, ctx, K = env
    o0, o1, a, b = all_pairs()
    c0 = sk.encrypt_bits(a, nonce=40_000_000)
    c1 = sk.encrypt_bits(b, nonce=40_100_000)
    log(f"compound: {len(o0)} gates")
    g0, g1 = run_compound(ctx, o0, o1, c0, c1)
    np.testing.assert_array_equal(sk.decrypt_bits(g0), [truth(o, x, y) for o, x, y in zip(o0, a, b)])
    np.testing.assert_array_equal(sk.decrypt_bits(g1), [truth(o, x, y) for o, x, y in zip(o1, a, b)])
    w0, w1 = oracle_compound(K, o0, o1, c0, c1)
    np.testing.assert_array_equal(g0, w0)
    np.testing.assert_array_equal(g1, w1)


@pytest.mark.parametrize("shape", [(1, 8, 1), (1, 4, 0), (2, 1, 1), (2, 1, 0), (4, 1, 1)])
def test_compound_every_shape_on_gate_outputs(env, shape):
    """Compound gates whose inputs are outputs of compound gates (the noisier
    weighted samples), in every kind of blind-rotation kernel (one wave per
    gate in both arithmetics, two and four waves per gate)."""
    sk, ctx, K = env
    n = 11
    o0 = np.array(SYM * 2, np.uint8)[:n]
    o1 = np.array(SYM[::-1] * 2, np.uint8)[:n]
    a, b, c = workloads.bits(41, n), workloads.bits(42, n), workloads.bits(43, n)
    ca = sk.encrypt_bits(a, nonce=41_000_000)
    cb = sk.encrypt_bits(b, nonce=41_100_000)
    cc = sk.encrypt_bits(c, nonce=41_200_000)
    x0, x1 = oracle_compound(K, np.full(n, F.XOR, np.uint8), np.full(n, F.AND, np.uint8), ca, cb)
    try:
        F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, shape)
        log(f"compound on compound outputs, shape {shape}")
        g0, g1 = run_compound(ctx, o0, o1, x0, x1)
        g2, g3 = run_compound(ctx, o1, o0, x1, cc)
    finally:
        F.fhe_ctx_set_launch_config(ctx, 1, WIDEST, (1, 8, 1))
    w0, w1 = oracle_compound(K, o0, o1, x0, x1)
    np.testing.assert_array_equal(g0, w0)
    np.testing.assert_array_equal(g1, w1)
    w2, w3 = oracle_compound(K, o1, o0, x1, cc)
    np.testing.assert_array_equal(g2, w2)
    np.testing.assert_array_equal(g3, w3)
    xa, ya = a ^ b, a & b
    np.testing.assert_array_equal(sk.decrypt_bits(g0), [truth(o, p, q) for o, p, q in zip(o0, xa, ya)])
    np.testing.assert_array_equal(sk.decrypt_bits(g3), [truth(o, p, q) for o, p, q in zip(o0, ya, c)])


@pytest.mark.parametrize("width,count", [(1, 2), (2, 3), (5, 2), (16, 2)])
def test_add_compound_bit_exact(env, width, count):
    """The ripple-carry adder with compound (XOR, AND) nodes."""
    sk, ctx, K = env
    import torch
    a = workloads.uniform_uints(140 + width, count, width)
    b = workloads.uniform_uints(150 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=42_000_000)
    cb = sk.encrypt_uint(b, width, nonce=42_100_000)
    dA, dB = F.to_device(ca), F.to_device(cb)
    dR = torch.empty_like(dA)
    log(f"add_compound width={width} count={count}")
    F.fhe_add_compound(ctx, dA, dB, dR, count, width)
    torch.cuda.synchronize()
    got = F.to_host(dR)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a + b) % (1 << width))
    np.testing.assert_array_equal(got, K.add_compound(ca, cb, width))


def test_add_compound_1024_pairs_sampled(env):
    """The add16 workload (1024 pairs) through compound gates: every sum
    decrypts, pairs 0-3 bit-exact end to end, 64 sampled rotations of every
    level (both outputs of compound gates) bit-exact teacher-forced."""
    sk, ctx, K = env
    import torch
    wl = workloads.AddWorkload()
    a, b = wl.operands()
    ca = sk.encrypt_uint(a, wl.width, nonce=0)
    cb = sk.encrypt_uint(b, wl.width, nonce=1 << 40)
    dA, dB = F.to_device(ca), F.to_device(cb)
    dR = torch.empty_like(dA)
    log("add_compound x 1024 pairs")
    F.fhe_add_compound(ctx, dA, dB, dR, wl.count, wl.width)
    torch.cuda.synchronize()
    got = F.to_host(dR)
    np.testing.assert_array_equal(sk.decrypt_uint(got, wl.width), (a + b) % (1 << wl.width))
    np.testing.assert_array_equal(got[:4], K.add_compound(ca[:4], cb[:4], wl.width))
    check_sampled_levels(ctx, K, "add_compound", wl.width, dA, dB, dR, count=wl.count, seed=8, log=log)


def test_invalid_codes_give_zero_and_are_reported(env):
    """Codes outside a call's set: the gate's output is the all-zero sample,
    the other gates are unaffected, and the context reports FHE_EINVAL once
    (through fhe_ctx_check, or from the next batched call)."""
    import torch
    sk, ctx, K = env
    ops = np.array([F.NAND, 12, 255, F.XOR, F.MAJ], np.uint8)
    a, b = workloads.bits(44, 5), workloads.bits(45, 5)
    c0 = sk.encrypt_bits(a, nonce=43_000_000)
    c1 = sk.encrypt_bits(b, nonce=43_100_000)
    d_ops = torch.from_numpy(ops.copy()).cuda()
    d0, d1 = F.to_device(c0), F.to_device(c1)
    out = torch.full_like(d0, 7)
    log("invalid gate codes")
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d0, d1, out, 5)
    torch.cuda.synchronize()
    got = F.to_host(out)
    assert not got[[1, 2, 4]].any()
    np.testing.assert_array_equal(got[[0, 3]], K.bootstrap(ops[[0, 3]], c0[[0, 3]], c1[[0, 3]]))
    with pytest.raises(F.FheError) as e:
        F.fhe_ctx_check(ctx)
    assert e.value.code == F.FHE_EINVAL
    F.fhe_ctx_check(ctx)  # reported once
    # compound batch with a code that is not symmetric: zeros, then the next
    # batched call refuses
    g0, g1 = run_compound(ctx, np.array([F.AND, F.ANDNY], np.uint8), np.array([F.XOR, F.OR], np.uint8),
                          c0[:2], c1[:2])
    assert not g0[1].any() and not g1[1].any()
    w0, w1 = oracle_compound(K, np.array([F.AND]), np.array([F.XOR]), c0[:1], c1[:1])
    np.testing.assert_array_equal(g0[:1], w0)
    np.testing.assert_array_equal(g1[:1], w1)
    ok_ops = torch.from_numpy(np.array([F.AND], np.uint8)).cuda()
    with pytest.raises(F.FheError) as e:
        F.fhe_bootstrap_gate_batch(ctx, ok_ops, d0[:1], d1[:1], out[:1], 1)
    assert e.value.code == F.FHE_EINVAL
    F.fhe_bootstrap_gate_batch(ctx, ok_ops, d0[:1], d1[:1], out[:1], 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(F.to_host(out[:1]), K.bootstrap([F.AND], c0[:1], c1[:1]))


def test_two_streams_equal_one_stream(env):
    """Batches and a circuit issued back to back on two streams (same
    priority) share the context's scratch buffer; the context orders them, so
    every word equals the single-stream result."""
    import torch
    sk, ctx, K = env
    n = 3000
    ops = workloads.gate_ops(46, n)
    c0 = sk.encrypt_bits(workloads.bits(47, n), nonce=44_000_000)
    c1 = sk.encrypt_bits(workloads.bits(48, n), nonce=44_100_000)
    c2 = sk.encrypt_bits(workloads.bits(49, n), nonce=44_200_000)
    d_ops = torch.from_numpy(ops.copy()).cuda()
    d0, d1, d2 = F.to_device(c0), F.to_device(c1), F.to_device(c2)
    wl = workloads.AddWorkload(count=64)
    a, b = wl.operands()
    dA = F.to_device(sk.encrypt_uint(a, 16, nonce=44_300_000))
    dB = F.to_device(sk.encrypt_uint(b, 16, nonce=44_400_000))
    ref_x, ref_y, ref_r = torch.empty_like(d0), torch.empty_like(d0), torch.empty_like(dA)
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d0, d1, ref_x, n)
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d1, d2, ref_y, n)
    F.fhe_add(ctx, dA, dB, ref_r, 64, 16)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    x, y, r = torch.empty_like(d0), torch.empty_like(d0), torch.empty_like(dA)
    log("two streams: batch, batch, circuit")
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d0, d1, x, n, s1)
    F.fhe_bootstrap_gate_batch(ctx, d_ops, d1, d2, y, n, s2)
    F.fhe_add(ctx, dA, dB, r, 64, 16, s1)
    torch.cuda.synchronize()
    assert torch.equal(x, ref_x) and torch.equal(y, ref_y) and torch.equal(r, ref_r)
    np.testing.assert_array_equal(sk.decrypt_uint(F.to_host(r), 16), (a + b) % (1 << 16))
    pick = np.array([0, n // 2, n - 1])
    np.testing.assert_array_equal(F.to_host(y)[pick], K.bootstrap(ops[pick], c1[pick], c2[pick]))
