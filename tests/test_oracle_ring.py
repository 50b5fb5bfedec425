"""Pins of the oracle's ring arithmetic in Z/2^32[X]/(X^N+1) against facts that
do not depend on its code: brute-force polynomial products folded by X^N = -1,
monomial identities, and the rotation/product agreement."""
import numpy as np
import pytest

import oracle

M32 = 1 << 32


def brute_negacyclic(P, Q):
    """Full product in Python integers, then fold X^(N+m) -> -X^m."""
    N = len(P)
    full = [0] * (2 * N - 1)
    for i, p in enumerate(P):
        for j, q in enumerate(Q):
            full[i + j] += int(p) * int(q)
    out = [full[m] - (full[m + N] if m + N < len(full) else 0) for m in range(N)]
    return np.array([x % M32 for x in out], dtype=np.uint32)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 64])
def test_negacyclic_matches_brute_force(N):
    g = np.random.default_rng(N)
    for _ in range(20):
        P = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        Q = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        np.testing.assert_array_equal(oracle.negacyclic_mul(P, Q), brute_negacyclic(P, Q))


def test_negacyclic_extreme_words():
    N = 8
    P = np.full(N, 0xFFFFFFFF, np.uint32)
    Q = np.full(N, 0x80000000, np.uint32)
    np.testing.assert_array_equal(oracle.negacyclic_mul(P, Q), brute_negacyclic(P, Q))


def test_x_to_the_n_is_minus_one():
    N = 16
    g = np.random.default_rng(7)
    P = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
    np.testing.assert_array_equal(oracle.rotate(P, N), (-P.astype(np.int64)) % M32)
    np.testing.assert_array_equal(oracle.rotate(P, 2 * N), P)
    one = np.zeros(N, np.uint32)
    one[0] = 1
    np.testing.assert_array_equal(oracle.negacyclic_mul(P, one), P)


def test_rotation_composes_and_equals_monomial_product():
    N = 32
    g = np.random.default_rng(11)
    P = g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
    for a in [0, 1, 5, N - 1, N, N + 3, 2 * N - 1]:
        mono = np.zeros(N, np.uint32)
        if a < N:
            mono[a] = 1
        else:
            mono[a - N] = M32 - 1
        np.testing.assert_array_equal(oracle.rotate(P, a), oracle.negacyclic_mul(mono, P))
        for b in [0, 2, N - 2, N + 7]:
            np.testing.assert_array_equal(oracle.rotate(oracle.rotate(P, a), b),
                                          oracle.rotate(P, (a + b) % (2 * N)))


def test_product_is_bilinear_and_commutative_at_full_size():
    N = 1024
    g = np.random.default_rng(3)
    P, Q, R = (g.integers(0, M32, N, dtype=np.uint64).astype(np.uint32) for _ in range(3))
    pq = oracle.negacyclic_mul(P, Q)
    np.testing.assert_array_equal(pq, oracle.negacyclic_mul(Q, P))
    lhs = oracle.negacyclic_mul(P, (Q.astype(np.uint64) + R) .astype(np.uint32))
    rhs = (pq.astype(np.uint64) + oracle.negacyclic_mul(P, R)).astype(np.uint32)
    np.testing.assert_array_equal(lhs, rhs)
    # one coefficient by brute force at full size
    m = 517
    want = sum(int(P[j]) * int(Q[m - j]) for j in range(m + 1)) - \
        sum(int(P[j]) * int(Q[N + m - j]) for j in range(m + 1, N))
    assert int(pq[m]) == want % M32
