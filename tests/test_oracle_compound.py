"""Pins of the oracle's compound gate (Sec. V-A-3: two gates on the same two
inputs), computed from one blind rotation: truth tables of both outputs,
the exact phase of every combination under a zero key with noiseless keys
(a closed form of the rotation amount), the key-switch closed form, and the
output noise against the rotation's variance scaled by the combination
weights."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle

M32 = 1 << 32
SYM = [oracle.AND, oracle.NAND, oracle.OR, oracle.NOR, oracle.XOR, oracle.XNOR]
TRUTH = {oracle.AND: lambda a, b: a & b, oracle.NAND: lambda a, b: 1 - (a & b),
         oracle.OR: lambda a, b: a | b, oracle.NOR: lambda a, b: 1 - (a | b),
         oracle.XOR: lambda a, b: a ^ b, oracle.XNOR: lambda a, b: 1 - (a ^ b)}


def value(op, k):
    """+1 / -1: the gate's output with k of its two inputs true."""
    return 1 if TRUTH[op](1 if k >= 1 else 0, 1 if k == 2 else 0) else -1


def test_truth_tables_of_both_outputs(okeys):
    """Every symmetric code in both output positions, on all four input pairs."""
    pairs = [(oracle.AND, oracle.XOR), (oracle.XOR, oracle.AND), (oracle.OR, oracle.NAND),
             (oracle.NOR, oracle.XNOR), (oracle.XNOR, oracle.OR), (oracle.NAND, oracle.NOR)]
    a = np.array([0, 0, 1, 1] * len(pairs), np.uint8)
    b = np.array([0, 1, 0, 1] * len(pairs), np.uint8)
    ops = np.repeat(np.array(pairs, np.uint8), 4, axis=0)
    out = okeys.bootstrap_compound(ops, okeys.encrypt_bits(a, nonce=70_000), okeys.encrypt_bits(b, nonce=71_000))
    dec = okeys.decrypt_bits(out.reshape(-1, okeys.width)).reshape(-1, 2)
    for k in range(len(a)):
        for o in range(2):
            assert dec[k, o] == TRUTH[int(ops[k, o])](int(a[k]), int(b[k])), (k, o)
    with pytest.raises(ValueError):
        okeys.bootstrap_compound(np.array([[oracle.AND, oracle.ANDNY]], np.uint8), out[:1, 0], out[:1, 1])


def test_zero_key_closed_form(okeys):
    """LWE key s = 0, noiseless keys: every CMux adds an exact encryption of
    0, so the accumulator's phase is exactly X^(-bbar) (1/16)(1 + ... + X^(N-1))
    with bbar the switched body of c1 + c2.  Each code's combination then has
    phase exactly (g1 - g2) U(bbar + 3N/4) + (g1 - g0) U(bbar + N/4) +
    (g0 + g2) / 16, U(p) = +1/16 for p mod 2N < N and -1/16 otherwise, at every
    bbar including the switching points; and the key-switched output has
    body (its phase under s = 0) b' - sum_i S_i round16(a'_i)."""
    P = oracle.default_params(lwe_stdev=0.0, bk_stdev=0.0)
    K0 = oracle.Keys(5, params=P, lwe_key=np.zeros(P.n, np.int32))
    N = P.N
    S = K0.tlwe_key.astype(np.int64)
    g = np.random.default_rng(41)

    def U(p):
        return (1 << 28) if p % (2 * N) < N else M32 - (1 << 28)

    bbars = [0, 1, 255, 256, 257, 511, 512, 767, 768, 1023, 1024, 1279, 1280, 1536, 1791, 1792, 2047]
    c1 = g.integers(0, M32, (len(bbars), P.n + 1), dtype=np.uint64).astype(np.uint32)
    c1[:, -1] = (np.array(bbars, np.uint64) << np.uint64(21)).astype(np.uint32)
    c2 = np.zeros_like(c1)
    tv = np.full(N, 1 << 28, np.uint32)
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 8) as ex:
        accs = list(ex.map(lambda k: K0.blind_rotate(c1[k] + c2[k], tv), range(len(bbars))))
    for k, bb in enumerate(bbars):
        for op in SYM:
            big = oracle.compound_combine(op, accs[k], P).astype(np.int64)
            ph = (big[N] - big[:N] @ S) % M32
            g0, g1, g2 = value(op, 0), value(op, 1), value(op, 2)
            want = ((g1 - g2) * U(bb + 3 * N // 4) + (g1 - g0) * U(bb + N // 4) + (g0 + g2) * (1 << 28)) % M32
            assert ph == want, (bb, op)
    ops = np.array([[oracle.AND, oracle.XOR]] * len(bbars), np.uint8)
    out = K0.bootstrap_compound(ops, c1, c2)
    for k in (0, 4, 9, 16):
        for o, op in enumerate((oracle.AND, oracle.XOR)):
            big = oracle.compound_combine(op, accs[k], P).astype(np.int64)
            r16 = ((big[:N] + (1 << 15)) % M32) >> 16 << 16
            assert out[k, o, -1] == (big[N] - r16 @ S) % M32


def test_output_noise_scales_with_the_weights(okeys):
    """96 compounds (AND, XOR) on fresh inputs: the AND output (weights -2, 0)
    carries 4 and the XOR output (2, 2) 8 times the per-coefficient
    rotation variance (9.22e-6, average case; coefficients uncorrelated) plus
    the key-switching term 3.66e-6: 4.05e-5 and 7.74e-5.  Sample of 96 per
    output: band +-45%; a doubled weight would read 4x."""
    count = 96
    g = np.random.default_rng(42)
    a = g.integers(0, 2, count, dtype=np.uint8)
    b = g.integers(0, 2, count, dtype=np.uint8)
    ops = np.array([[oracle.AND, oracle.XOR]] * count, np.uint8)
    out = okeys.bootstrap_compound(ops, okeys.encrypt_bits(a, nonce=72_000), okeys.encrypt_bits(b, nonce=73_000))
    ph = okeys.phase(out.reshape(-1, okeys.width)).astype(np.int64).reshape(count, 2)
    mu = oracle.MU
    for o, (op, est) in enumerate(((oracle.AND, 4.05e-5), (oracle.XOR, 7.74e-5))):
        want = np.array([TRUTH[op](int(x), int(y)) for x, y in zip(a, b)])
        err = (ph[:, o] - np.where(want == 1, mu, -mu)) / M32
        var = float(np.mean(err ** 2))
        assert abs(var / est - 1) < 0.45, (op, var)


def test_compound_adder_decrypts_to_sum(okeys):
    """The ripple-carry adder of eqs. (1)-(2) built from compound nodes."""
    w = 4
    a = np.array([9, 15, 6], np.uint64)
    b = np.array([8, 3, 9], np.uint64)
    R = okeys.add_compound(okeys.encrypt_uint(a, w, nonce=74_000), okeys.encrypt_uint(b, w, nonce=75_000), w)
    np.testing.assert_array_equal(okeys.decrypt_uint(R, w), (a + b) % (1 << w))
