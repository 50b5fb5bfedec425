"""The oracle's circuits evaluated on plaintext bits, each gate by its truth
table: sums, low products (shift-and-add and tree accumulation, Sec. III-B-1
and V-B-2), full products by Karatsuba's algorithm (Sec. III-B-2,
Algorithm 1) and matrix-vector products equal integer arithmetic,
exhaustively for narrow operands and on random operands up to 64 bits
(Karatsuba recurses from 16 bits on)."""
import numpy as np
import pytest

import oracle


def bits(v, w):
    return [(int(v) >> i) & 1 for i in range(w)]


def value(b):
    return sum(int(x) << i for i, x in enumerate(b))


WANT = {"add": lambda a, b, w: (a + b) % (1 << w),
        "add_numberwise": lambda a, b, w: (a + b) % (1 << w),
        "add_fa": lambda a, b, w: (a + b) % (1 << w),
        "add_compound": lambda a, b, w: (a + b) % (1 << w),
        "mul": lambda a, b, w: (a * b) % (1 << w),
        "mul_tree": lambda a, b, w: (a * b) % (1 << w),
        "karatsuba": lambda a, b, w: a * b}


@pytest.mark.parametrize("kind", ["add", "add_numberwise", "add_fa", "add_compound", "mul", "mul_tree", "karatsuba"])
def test_exhaustive_narrow(kind):
    for w in range(2 if kind == "karatsuba" else 1, 6):
        for a in range(1 << w):
            for b in range(1 << w):
                out = oracle.circuit_eval_plain(kind, w, bits(a, w) + bits(b, w))
                assert value(out) == WANT[kind](a, b, w), (kind, w, a, b)


@pytest.mark.parametrize("w", [15, 16, 17, 24, 32, 33, 64])
def test_random_wide_products(w):
    rng = np.random.default_rng(w)
    for _ in range(60):
        a = int(rng.integers(0, 1 << 62)) % (1 << w) | (1 << (w - 1))  # top bit set: longest carries
        b = int(rng.integers(0, 1 << 62)) % (1 << w)
        ab = bits(a, w) + bits(b, w)
        assert value(oracle.circuit_eval_plain("karatsuba", w, ab)) == a * b
        assert value(oracle.circuit_eval_plain("mul_tree", w, ab)) == (a * b) % (1 << w)
        assert value(oracle.circuit_eval_plain("mul", w, ab)) == (a * b) % (1 << w)
        assert value(oracle.circuit_eval_plain("add", w, ab)) == (a + b) % (1 << w)
        assert value(oracle.circuit_eval_plain("add_numberwise", w, ab)) == (a + b) % (1 << w)
        assert value(oracle.circuit_eval_plain("add_fa", w, ab)) == (a + b) % (1 << w)
        assert value(oracle.circuit_eval_plain("add_compound", w, ab)) == (a + b) % (1 << w)
    top = (1 << w) - 1  # all ones: every carry chain at its longest
    assert value(oracle.circuit_eval_plain("karatsuba", w, bits(top, w) * 2)) == top * top
    one = bits(1, w)  # 2^w - 1 + 1: a carry through every round of the number-wise adder
    assert value(oracle.circuit_eval_plain("add_numberwise", w, bits(top, w) + one)) == 0


def test_matvec_random():
    rng = np.random.default_rng(7)
    for rows, cols, w in [(2, 3, 4), (3, 5, 6), (1, 7, 8)]:
        M = rng.integers(0, 1 << w, (rows, cols))
        x = rng.integers(0, 1 << w, cols)
        inp = sum((bits(v, w) for v in M.reshape(-1)), []) + sum((bits(v, w) for v in x), [])
        out = oracle.circuit_eval_plain("matvec", w, inp, rows, cols)
        got = [value(out[r * w:(r + 1) * w]) for r in range(rows)]
        assert got == list((M.astype(object) @ x.astype(object)) % (1 << w))


def test_karatsuba_gate_counts():
    """Below 16 bits the base product (w^2 ANDs and the tree's adders); from 16
    bits on, three half-size products plus adders and one subtractor (the
    totals also follow from an independent count of that construction)."""
    for w in range(2, 16):
        assert oracle.circuit_gate_count("karatsuba", w) >= w * w
    assert oracle.circuit_gate_count("karatsuba", 16) == 1457
    assert oracle.circuit_gate_count("karatsuba", 32) == 5271


def test_numberwise_add_gate_count():
    """Round k of the number-wise adder has w - k XORs and w - k - 1 ANDs."""
    for w in range(1, 40):
        assert oracle.circuit_gate_count("add_numberwise", w) == sum(2 * (w - k) - 1 for k in range(w)) == w * w


def test_matmul_cannon_random():
    """Cannon's algorithm (Sec. V-B-3) gives the matrix product mod 2^w."""
    rng = np.random.default_rng(11)
    for n, w in [(1, 5), (2, 4), (3, 6), (4, 16), (5, 3)]:
        A = rng.integers(0, 1 << w, (n, n))
        B = rng.integers(0, 1 << w, (n, n))
        inp = sum((bits(v, w) for v in A.reshape(-1)), []) + sum((bits(v, w) for v in B.reshape(-1)), [])
        out = oracle.circuit_eval_plain("matmul", w, inp, n)
        got = np.array([value(out[q * w:(q + 1) * w]) for q in range(n * n)], dtype=object).reshape(n, n)
        np.testing.assert_array_equal(got, (A.astype(object) @ B.astype(object)) % (1 << w))


def test_matmul_cannon_gate_count():
    """n^2 cells, each n tree products and n - 1 ripple additions."""
    for n, w in [(1, 4), (2, 16), (4, 16), (3, 7)]:
        want = n * n * (n * oracle.circuit_gate_count("mul_tree", w) + (n - 1) * oracle.circuit_gate_count("add", w))
        assert oracle.circuit_gate_count("matmul", w, n) == want


def test_full_adder_gate_count():
    """A half adder, w - 2 full adders (two gates each) and the top sum."""
    assert oracle.circuit_gate_count("add_fa", 1) == 1
    for w in range(2, 40):
        assert oracle.circuit_gate_count("add_fa", w) == 2 * w - 1


def test_compound_adder_gate_count():
    """Compound (XOR, AND) nodes at bit 0 and twice per middle bit, one OR per
    middle bit, two XORs at the top bit: 3w - 3 bootstraps for w >= 2."""
    assert oracle.circuit_gate_count("add_compound", 1) == 1
    for w in range(2, 40):
        assert oracle.circuit_gate_count("add_compound", w) == 3 * w - 3
