"""The paper's CPU parallel framework (Sec. IV), the second host baseline:
its gate bootstraps (AVX2 two-prime NTT products) give the oracle's words
bit for bit, and its addition (numbers across threads, bits in carry order)
and multiplication (partial-product ANDs across threads, accumulation in
order) give the oracle's circuit words and decrypt to plaintext arithmetic."""
import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads


@pytest.fixture(scope="module")
def env():
    from paper_2005_01945_amd import cpupar
    sk, ck = F.fhe_keygen(0)
    bk, ksk = ck.export()
    return sk, cpupar.CpuParallel(bk, ksk), oracle.Keys(0)


def test_gates_bit_exact(env):
    sk, cp, K = env
    ops = np.arange(10, dtype=np.uint8).repeat(2)
    a, b = workloads.bits(31, 20), workloads.bits(32, 20)
    c0 = sk.encrypt_bits(a, nonce=60_000_000)
    c1 = sk.encrypt_bits(b, nonce=60_100_000)
    got = cp.bootstrap(ops, c0, c1)
    np.testing.assert_array_equal(got, K.bootstrap(ops, c0, c1))
    # gates on gate outputs (key-switched, noisier samples), one thread
    got2 = cp.bootstrap(ops[:4], got[:4], got[4:8], threads=1)
    np.testing.assert_array_equal(got2, K.bootstrap(ops[:4], got[:4], got[4:8]))
    with pytest.raises(ValueError):
        cp.bootstrap([10], c0[:1], c1[:1])


@pytest.mark.parametrize("width,count", [(1, 2), (4, 3)])
def test_add_bit_exact(env, width, count):
    sk, cp, K = env
    a = workloads.uniform_uints(33 + width, count, width)
    b = workloads.uniform_uints(34 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=61_000_000)
    cb = sk.encrypt_uint(b, width, nonce=61_100_000)
    got = cp.add(ca, cb, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a + b) % (1 << width))
    np.testing.assert_array_equal(got, K.add(ca, cb, width))


def test_mul_bit_exact(env):
    sk, cp, K = env
    width, count = 4, 2
    a = workloads.uniform_uints(35, count, width)
    b = workloads.uniform_uints(36, count, width)
    ca = sk.encrypt_uint(a, width, nonce=62_000_000)
    cb = sk.encrypt_uint(b, width, nonce=62_100_000)
    got = cp.mul(ca, cb, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a * b) % (1 << width))
    np.testing.assert_array_equal(got, K.mul(ca, cb, width))
