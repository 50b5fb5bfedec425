"""Pins of the oracle's whole bootstrap: truth tables, special-case keys whose
output phase has a closed form, measured noise against the variance bound,
and circuits that must decrypt to plaintext arithmetic."""
import os

import numpy as np
import pytest

import oracle
import workloads

M32 = 1 << 32
MU = oracle.MU

TRUTH = {
    oracle.AND: lambda a, b: a & b, oracle.NAND: lambda a, b: 1 - (a & b),
    oracle.OR: lambda a, b: a | b, oracle.NOR: lambda a, b: 1 - (a | b),
    oracle.XOR: lambda a, b: a ^ b, oracle.XNOR: lambda a, b: 1 - (a ^ b),
    oracle.ANDNY: lambda a, b: (1 - a) & b, oracle.ANDYN: lambda a, b: a & (1 - b),
    oracle.ORNY: lambda a, b: (1 - a) | b, oracle.ORYN: lambda a, b: a | (1 - b),
}


def signed(x):
    x = int(x) % M32
    return x - M32 if x >= M32 // 2 else x


def test_truth_tables_all_gates(okeys):
    a_bits, b_bits = workloads.truth_table_inputs()
    ops, A, B, want = [], [], [], []
    for op in range(10):
        for a, b in zip(a_bits, b_bits):
            ops.append(op)
            A.append(a)
            B.append(b)
            want.append(TRUTH[op](int(a), int(b)))
    ca = okeys.encrypt_bits(A, nonce=10_000)
    cb = okeys.encrypt_bits(B, nonce=20_000)
    out = okeys.bootstrap(ops, ca, cb)
    assert list(okeys.decrypt_bits(out)) == want
    # output phase is +-mu up to the bootstrap noise (sigma ~ 3.6e-3 << 1/16)
    ph = okeys.phase(out).astype(np.int64)
    err = np.abs(ph - np.where(np.array(want) == 1, MU, -MU)) / M32
    assert err.max() < 1 / 32


def test_zero_key_noiseless_closed_form():
    """LWE key s = 0 and noiseless keys: every BK_i is a noiseless TGSW(0), so
    the accumulator phase stays exactly X^(-bbar) v and the extracted phase is
    +mu iff bbar < N, else -mu, with no error at all.  After key switching with
    noiseless KSK under s = 0 the output body is exactly
    b' - sum_i S_i round16(a'_i)."""
    P = oracle.default_params(lwe_stdev=0.0, bk_stdev=0.0)
    K = oracle.Keys(seed=3, params=P, lwe_key=np.zeros(P.n, np.int32))
    g = np.random.default_rng(5)
    for trial in range(3):
        lwe = g.integers(0, M32, P.n + 1, dtype=np.uint64).astype(np.uint32)
        acc = K.blind_rotate(lwe)
        big = K.sample_extract(acc)
        S = K.tlwe_key.astype(np.int64)
        ph = (int(big[-1]) - int((big[:-1].astype(np.int64) * S).sum())) % M32
        bbar = oracle.modswitch(int(lwe[-1]), P)
        assert ph == (MU if bbar < P.N else M32 - MU)
        out = K.key_switch(big)
        rounded = (((big[:-1].astype(np.int64) + (1 << 15)) >> 16) << 16) % M32
        want = (int(big[-1]) - int((S * rounded).sum())) % M32
        assert int(out[-1]) == want


def test_single_key_bit_rotation_direction():
    """s = e_i0 with noiseless keys: only CMux i0 rotates, so the extracted
    phase is +mu iff (bbar - abar_i0) mod 2N < N (up to the gadget rounding
    error, at most 2^11 (1 + N) << mu)."""
    P = oracle.default_params(lwe_stdev=0.0, bk_stdev=0.0)
    i0 = 137
    key = np.zeros(P.n, np.int32)
    key[i0] = 1
    K = oracle.Keys(seed=4, params=P, lwe_key=key)
    g = np.random.default_rng(9)
    S = K.tlwe_key.astype(np.int64)
    for trial in range(3):
        lwe = g.integers(0, M32, P.n + 1, dtype=np.uint64).astype(np.uint32)
        acc = K.blind_rotate(lwe)
        big = K.sample_extract(acc)
        ph = signed(int(big[-1]) - int((big[:-1].astype(np.int64) * S).sum()))
        bbar = oracle.modswitch(int(lwe[-1]), P)
        abar = oracle.modswitch(int(lwe[i0]), P)
        sign = 1 if (bbar - abar) % (2 * P.N) < P.N else -1
        assert abs(ph - sign * MU) <= (1 << 11) * (1 + P.N)


def test_cmux_with_trivial_key_rotates_exactly():
    """A CMux whose key row set is the gadget matrix itself (a noiseless
    trivial TGSW(1)) replaces acc by X^abar acc up to the decomposition error
    of at most 2^11 per coefficient."""
    P = oracle.default_params()
    N = P.N
    bk = np.zeros((4, 2, N), np.uint32)
    for j in range(2):
        for p in range(2):
            bk[2 * j + p, j, 0] = 1 << (32 - 10 * (p + 1))
    g = np.random.default_rng(12)
    acc = g.integers(0, M32, 2 * N, dtype=np.uint64).astype(np.uint32)
    for abar in (0, 1, 777, 1024, 2047):
        out = oracle.cmux(bk, abar, acc, P)
        want = np.concatenate([oracle.rotate(acc[:N], abar), oracle.rotate(acc[N:], abar)])
        d = (out.astype(np.int64) - want.astype(np.int64)) % M32
        d = np.where(d >= M32 // 2, d - M32, d)
        assert np.abs(d).max() <= 1 << 11


def test_bootstrap_noise_within_bound(okeys):
    """Output noise of gate bootstraps against the worst-case bound 3.27e-5 and
    within 15% of the average-case estimate 1.29e-5, over 10,240 noise
    samples: 160 bootstraps of random gates on fresh inputs, each blind
    rotation read out at 64 coefficients m = 0, 16, ..., 1008 (extraction at m,
    then key switching).  The variance terms of the estimate hold for every
    coefficient of the rotated accumulator, and coefficient m carries the test
    vector entry at the rotation amount + m: +mu when (m + rho) mod 2N < N,
    with rho = bbar - sum abar_i s_i the exact rotation.  Different
    coefficients combine the same digits with different key-noise
    coefficients, so their errors are uncorrelated to first order.  The
    coefficient-0 samples are also the gates' own outputs (decrypting to the
    truth table)."""
    from concurrent.futures import ThreadPoolExecutor
    P = okeys.P
    count, coeffs = 160, np.arange(0, 1024, 16)
    g = np.random.default_rng(21)
    ops = g.integers(0, 10, count).astype(np.uint8)
    a = g.integers(0, 2, count, dtype=np.uint8)
    b = g.integers(0, 2, count, dtype=np.uint8)
    c1 = okeys.encrypt_bits(a, nonce=30_000)
    c2 = okeys.encrypt_bits(b, nonce=40_000)
    s = okeys.lwe_key.astype(np.int64)

    def one(k):
        comb = oracle.gate_combine(int(ops[k]), c1[k], c2[k], P)
        bar = np.array([oracle.modswitch(int(x), P) for x in comb], np.int64)
        rho = int(bar[-1] - bar[:-1] @ s) % (2 * P.N)
        acc = okeys.blind_rotate(comb)
        outs = np.stack([okeys.key_switch(okeys.sample_extract_at(acc, int(m))) for m in coeffs])
        want = np.where((coeffs + rho) % (2 * P.N) < P.N, MU, -MU)
        return outs, want

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 8) as ex:
        res = list(ex.map(one, range(count)))
    outs = np.stack([r[0] for r in res])
    want = np.stack([r[1] for r in res])
    ph = okeys.phase(outs.reshape(-1, P.n + 1)).astype(np.int64).reshape(count, coeffs.size)
    err = (ph - want) / M32
    var = float(np.mean(err ** 2))
    assert err.size == 10240
    assert var < 3.27e-5
    print(f"noise: mean square {var:.4e} over {err.size} samples")
    assert abs(var / 1.29e-5 - 1) < 0.15, var
    table = [a & b, 1 - (a & b), a | b, 1 - (a | b), a ^ b, 1 - (a ^ b), (1 - a) & b, a & (1 - b), (1 - a) | b,
             a | (1 - b)]
    truth = np.array([table[o][k] for k, o in enumerate(ops)])
    np.testing.assert_array_equal(okeys.decrypt_bits(outs[:, 0]), truth)
    np.testing.assert_array_equal(outs[:16, 0], okeys.bootstrap(ops[:16], c1[:16], c2[:16]))


def test_add_circuit_decrypts_to_sum(okeys):
    w = 4
    a = np.array([9, 15], np.uint64)
    b = np.array([8, 3], np.uint64)
    R = okeys.add(okeys.encrypt_uint(a, w, nonce=50_000), okeys.encrypt_uint(b, w, nonce=60_000), w)
    np.testing.assert_array_equal(okeys.decrypt_uint(R, w), (a + b) % (1 << w))


def test_mul_circuit_decrypts_to_low_product(okeys):
    w = 4
    a = np.array([13], np.uint64)
    b = np.array([11], np.uint64)
    R = okeys.mul(okeys.encrypt_uint(a, w, nonce=70_000), okeys.encrypt_uint(b, w, nonce=80_000), w)
    np.testing.assert_array_equal(okeys.decrypt_uint(R, w), (a * b) % (1 << w))


def test_mul_tree_circuit_decrypts_to_low_product(okeys):
    """Tree accumulation of the partial products (Sec. V-B-2): the product's
    low bits, with carries across every round and a wrap past 2^w."""
    w = 5
    a = np.array([29, 23], np.uint64)
    b = np.array([27, 22], np.uint64)
    R = okeys.mul_tree(okeys.encrypt_uint(a, w, nonce=72_000), okeys.encrypt_uint(b, w, nonce=82_000), w)
    np.testing.assert_array_equal(okeys.decrypt_uint(R, w), (a * b) % (1 << w))


def test_numberwise_add_decrypts_to_sum(okeys):
    w = 4
    a = np.array([9, 15], np.uint64)
    b = np.array([8, 1], np.uint64)
    R = okeys.add_numberwise(okeys.encrypt_uint(a, w, nonce=76_000), okeys.encrypt_uint(b, w, nonce=86_000), w)
    np.testing.assert_array_equal(okeys.decrypt_uint(R, w), (a + b) % (1 << w))


def test_karatsuba_circuit_decrypts_to_full_product(okeys):
    """Karatsuba's algorithm returns all 2w bits of the product (below 16 bits
    through its base product)."""
    w = 4
    a = np.array([13], np.uint64)
    b = np.array([11], np.uint64)
    R = okeys.karatsuba(okeys.encrypt_uint(a, w, nonce=74_000), okeys.encrypt_uint(b, w, nonce=84_000), w)
    assert R.shape[1] == 2 * w
    np.testing.assert_array_equal(okeys.decrypt_uint(R, 2 * w), a * b)


def test_matmul_cannon_decrypts_to_product(okeys):
    w, n = 2, 2
    A = np.array([[3, 2], [1, 3]], np.uint64)
    B = np.array([[2, 3], [3, 1]], np.uint64)
    C = okeys.matmul(okeys.encrypt_uint(A.reshape(-1), w, nonce=92_000),
                     okeys.encrypt_uint(B.reshape(-1), w, nonce=93_000), n, w)
    np.testing.assert_array_equal(okeys.decrypt_uint(C.reshape(n * n, w, -1), w).reshape(n, n), (A @ B) % (1 << w))


def test_matvec_circuit_decrypts_to_product(okeys):
    w, rows, cols = 2, 2, 2
    M = np.array([[3, 2], [1, 3]], np.uint64)
    x = np.array([3, 1], np.uint64)
    cm = okeys.encrypt_uint(M.reshape(-1), w, nonce=90_000)
    cx = okeys.encrypt_uint(x, w, nonce=95_000)
    y = okeys.matvec(cm, cx, rows, cols, w)
    np.testing.assert_array_equal(okeys.decrypt_uint(y, w), (M @ x) % (1 << w))


def test_circuit_gate_counts():
    """Gate counts of the circuit definitions: w-bit ripple-carry adder
    5w - 6, shift-and-add multiplier, and the 64x64 16-bit matvec."""
    assert oracle.circuit_gate_count("add", 16) == 74
    assert oracle.circuit_gate_count("add", 32) == 154
    for w in range(2, 40):
        assert oracle.circuit_gate_count("add", w) == 5 * w - 6
    ands = 32 * 33 // 2
    adders = 1 + sum(5 * m - 6 for m in range(2, 32))
    assert oracle.circuit_gate_count("mul", 32) == ands + adders == 2824
    assert oracle.circuit_gate_count("mul", 16) == 648
    assert oracle.circuit_gate_count("matvec", 16, 64, 64) == 4096 * 648 + 64 * 63 * 74


def test_mul_tree_gate_count_equals_shift_and_add():
    """Every partial product i >= 1 is the operand with more known-zero low
    bits in exactly one tree addition, which then spans bits i..w-1, as in the
    shift-and-add multiplier: the two circuits have the same gates."""
    add = lambda m: 1 if m == 1 else 5 * m - 6
    for w in range(1, 40):
        want = w * (w + 1) // 2 + sum(add(w - i) for i in range(1, w))
        assert oracle.circuit_gate_count("mul_tree", w) == want == oracle.circuit_gate_count("mul", w)


def test_three_input_gates_truth_tables(okeys):
    """MAJ and XOR3 decrypt to majority and parity for all eight inputs, fresh
    and on bootstrapped (noisier) inputs."""
    combos = [(i >> 2 & 1, i >> 1 & 1, i & 1) for i in range(8)]
    x = okeys.encrypt_bits([c[0] for c in combos], nonce=110_000)
    y = okeys.encrypt_bits([c[1] for c in combos], nonce=111_000)
    z = okeys.encrypt_bits([c[2] for c in combos], nonce=112_000)
    for op, f in [(oracle.MAJ, lambda a, b, c: int(a + b + c >= 2)), (oracle.XOR3, lambda a, b, c: (a + b + c) & 1)]:
        out = okeys.bootstrap3([op] * 8, x, y, z, threads=8)
        assert list(okeys.decrypt_bits(out)) == [f(*c) for c in combos]
    # inputs that are themselves gate outputs: z2 = AND(z, z) = z
    z2 = okeys.bootstrap([oracle.AND] * 8, z, z, threads=8)
    out = okeys.bootstrap3([oracle.XOR3] * 8, x, y, z2, threads=8)
    assert list(okeys.decrypt_bits(out)) == [(a + b + c) & 1 for a, b, c in combos]


def test_full_adder_circuit_decrypts_to_sum(okeys):
    w = 5
    a = np.array([29, 7], np.uint64)
    b = np.array([6, 25], np.uint64)
    R = okeys.add_fa(okeys.encrypt_uint(a, w, nonce=120_000), okeys.encrypt_uint(b, w, nonce=121_000), w)
    np.testing.assert_array_equal(okeys.decrypt_uint(R, w), (a + b) % (1 << w))


def lut_encrypt(K, phases, seed):
    """Noiseless LWE samples of the given torus phases (uint32) under K's key."""
    g = np.random.default_rng(seed)
    n = K.P.n
    a = g.integers(0, M32, (len(phases), n), dtype=np.uint64)
    b = ((a * K.lwe_key.astype(np.uint64)).sum(axis=1) + np.asarray(phases, np.uint64)) % M32
    return np.concatenate([a, b[:, None]], axis=1).astype(np.uint32)


def test_lut_zero_key_closed_form():
    """Programmable bootstrapping with s = 0 and noiseless keys: the extracted
    phase is exactly tv[bbar] for bbar < N and -tv[bbar - N] above."""
    P = oracle.default_params(lwe_stdev=0.0, bk_stdev=0.0)
    K = oracle.Keys(seed=3, params=P, lwe_key=np.zeros(P.n, np.int32))
    g = np.random.default_rng(6)
    tv = g.integers(0, M32, P.N, dtype=np.uint64).astype(np.uint32)
    for trial in range(4):
        lwe = g.integers(0, M32, P.n + 1, dtype=np.uint64).astype(np.uint32)
        big = K.sample_extract(K.blind_rotate(lwe, tv))
        S = K.tlwe_key.astype(np.int64)
        ph = (int(big[-1]) - int((big[:-1].astype(np.int64) * S).sum())) % M32
        bbar = oracle.modswitch(int(lwe[-1]), P)
        assert ph == (int(tv[bbar]) if bbar < P.N else (M32 - int(tv[bbar - P.N])) % M32)
    # the constant vector mu is the gate test vector
    lwe = g.integers(0, M32, P.n + 1, dtype=np.uint64).astype(np.uint32)
    np.testing.assert_array_equal(K.blind_rotate(lwe, np.full(P.N, MU, np.uint32)), K.blind_rotate(lwe))


def test_lut_two_bit_function(okeys):
    """A 2-bit lookup table with a padding bit: m in {0..3} at phase m/8 + 1/16
    (so the phase stays in [0, 1/2)); tv holds f(m)/8 + 1/16 on the quarter of
    [0, N) that m's phase switches to; the output decrypts to f(m)."""
    N = okeys.P.N
    f = [3, 0, 2, 1]
    tv = np.array([(f[j * 4 // N] << 29) + (1 << 28) for j in range(N)], np.uint32)
    ms = np.array([0, 1, 2, 3, 3, 2, 1, 0])
    ct = lut_encrypt(okeys, (ms << 29) + (1 << 28), seed=7)
    out = okeys.bootstrap_lut(tv, ct, threads=8)
    ph = okeys.phase(out).astype(np.int64) % M32
    assert list((ph >> 29) & 3) == [f[m] for m in ms]
