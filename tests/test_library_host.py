"""Host-side tests of the C-ABI library: it loads without a GPU, exports every
symbol include/fhe.h declares, and its host logic (keygen, encryption, key
files, argument checks, circuit shapes) agrees with the oracle.  No compute
call reaches the GPU here."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fhe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fhe_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    syms = declared_symbols()
    assert len(syms) >= 25
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    # the binding wraps all of them
    assert set(syms) <= set(F.exported_symbols())


@pytest.fixture(scope="module")
def lib_keys():
    return F.fhe_keygen(0)


def test_keygen_bytes_equal_oracle(lib_keys, okeys):
    sk, ck = lib_keys
    lwe, tlwe = sk.export()
    np.testing.assert_array_equal(lwe, okeys.lwe_key)
    np.testing.assert_array_equal(tlwe, okeys.tlwe_key)
    bk, ksk = ck.export()
    np.testing.assert_array_equal(bk, okeys.bk)
    np.testing.assert_array_equal(ksk, okeys.ksk)


def test_special_keys_equal_oracle():
    P = F.fhe_default_params()
    P.lwe_stdev = 0.0
    P.bk_stdev = 0.0
    key = np.zeros(500, np.int32)
    key[137] = 1
    sk, ck = F.fhe_keygen(4, P, lwe_key=key)
    OP = oracle.default_params(lwe_stdev=0.0, bk_stdev=0.0)
    K = oracle.Keys(4, OP, lwe_key=key)
    bk, ksk = ck.export()
    np.testing.assert_array_equal(bk, K.bk)
    np.testing.assert_array_equal(ksk, K.ksk)


def test_encryption_equals_oracle_and_decrypts(lib_keys, okeys):
    sk, _ = lib_keys
    bits = workloads.bits(3, 257)
    ct = sk.encrypt_bits(bits, nonce=123)
    np.testing.assert_array_equal(ct, okeys.encrypt_bits(bits, nonce=123))
    np.testing.assert_array_equal(sk.decrypt_bits(ct), bits)
    np.testing.assert_array_equal(sk.phase(ct), okeys.phase(ct))
    v = workloads.uniform_uints(4, 9, 16)
    cu = sk.encrypt_uint(v, 16, nonce=999)
    np.testing.assert_array_equal(cu, okeys.encrypt_uint(v, 16, nonce=999))
    np.testing.assert_array_equal(sk.decrypt_uint(cu, 16), v)
    v64 = workloads.uniform_uints(5, 3, 64)
    np.testing.assert_array_equal(sk.decrypt_uint(sk.encrypt_uint(v64, 64, nonce=7), 64), v64)


def test_key_file_round_trip(tmp_path, lib_keys):
    sk, ck = lib_keys
    path = str(tmp_path / "keys.bin")
    F.fhe_key_save(sk, ck, path)
    sk2, ck2 = F.fhe_key_load(path)
    for a, b in zip(sk.export(), sk2.export()):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(ck.export(), ck2.export()):
        np.testing.assert_array_equal(a, b)
    F.fhe_key_save(None, ck, path)
    sk3, ck3 = F.fhe_key_load(path)
    assert sk3 is None and ck3 is not None
    with open(path, "r+b") as f:
        f.truncate(1000)
    with pytest.raises(F.FheError) as e:
        F.fhe_key_load(path)
    assert e.value.code == F.FHE_EIO


def test_argument_errors():
    P = F.fhe_default_params()
    P.N = 2048
    with pytest.raises(F.FheError) as e:
        F.fhe_keygen(0, P)
    assert e.value.code == F.FHE_EINVAL
    sk, _ = F.fhe_keygen(0)
    with pytest.raises(F.FheError) as e:
        sk.encrypt_bits([0, 2])
    assert e.value.code == F.FHE_EINVAL
    with pytest.raises(F.FheError) as e:
        sk.encrypt_uint([1], 65)
    assert e.value.code == F.FHE_EINVAL
    L = F.lib()
    assert L.fhe_bootstrap_gate_batch(None, None, None, None, None, 4, None) == F.FHE_EINVAL
    assert L.fhe_add(None, None, None, None, 1, 8, None) == F.FHE_EINVAL
    assert L.fhe_bootstrap_gate3_batch(None, None, None, None, None, None, 4, None) == F.FHE_EINVAL
    assert b"null context" in L.fhe_last_error()
    assert L.fhe_debug_cmux(0, 0, None, 0, None) == F.FHE_EINVAL
    assert L.fhe_debug_cmux(0, 2, None, 0, None) == F.FHE_EINVAL
    assert L.fhe_debug_plan(None, 0, 16, 0, 0, 1, None, 0, None, 0, None, None) == F.FHE_EINVAL
    assert L.fhe_debug_read_wires(None, 0, 16, 0, 0, 1, None, None, None, None, 0, None) == F.FHE_EINVAL


def test_level_schedules_fill_launch_rounds():
    """The balanced schedules of the paper-sized workloads: every gate once,
    and whole launch rounds of 2,048 gates (eight per compute unit) nearly
    full (the bound is the gate count over the round size)."""
    for kind, w, count, rows, cols, most in [("add", 16, 1024, 0, 0, 37), ("mul", 32, 256, 0, 0, 356),
                                            ("matvec", 16, 1, 64, 64, 1445)]:
        widths = F.fhe_circuit_schedule(kind, w, count, 256, rows, cols)
        assert sum(widths) == F.fhe_circuit_shape(kind, w, rows, cols)[0] * count
        assert len(widths) == F.fhe_circuit_shape(kind, w, rows, cols)[1]
        rounds = sum((x + 2047) // 2048 for x in widths if 2 * x > 2048)
        assert rounds <= most, (kind, rounds)


def test_circuit_shapes_match_oracle_gate_counts():
    for w in (1, 2, 5, 16, 32):
        assert F.fhe_circuit_shape("add", w)[0] == oracle.circuit_gate_count("add", w)
        assert F.fhe_circuit_shape("mul", w)[0] == oracle.circuit_gate_count("mul", w)
        assert F.fhe_circuit_shape("mul_tree", w)[0] == oracle.circuit_gate_count("mul_tree", w)
    for w in (2, 5, 15, 16, 17, 24, 32, 33, 64):
        assert F.fhe_circuit_shape("karatsuba", w)[0] == oracle.circuit_gate_count("karatsuba", w)
        assert F.fhe_circuit_shape("add_numberwise", w)[0] == oracle.circuit_gate_count("add_numberwise", w)
    assert F.fhe_circuit_shape("add_numberwise", 16) == (256, 16, 31)
    for n, w in [(1, 3), (2, 16), (3, 5), (4, 16)]:
        assert F.fhe_circuit_shape("matmul", w, n)[0] == oracle.circuit_gate_count("matmul", w, n)
    for w in (1, 2, 5, 16, 32):
        assert F.fhe_circuit_shape("add_fa", w)[0] == oracle.circuit_gate_count("add_fa", w)
    assert F.fhe_circuit_shape("add_fa", 16) == (31, 16, 2)
    for w in (1, 2, 3, 16, 32):  # a compound node counts once
        assert F.fhe_circuit_shape("add_compound", w)[0] == oracle.circuit_gate_count("add_compound", w) == \
            (1 if w == 1 else 3 * w - 3)
    assert F.fhe_circuit_shape("add_compound", 16)[1] == F.fhe_circuit_shape("add", 16)[1]
    assert F.fhe_circuit_shape("matvec", 16, 64, 64)[0] == oracle.circuit_gate_count("matvec", 16, 64, 64)
    assert F.fhe_circuit_shape("matvec", 3, 5, 7)[0] == oracle.circuit_gate_count("matvec", 3, 5, 7)
    # gates, ASAP depth, widest level of the paper-sized circuits
    assert F.fhe_circuit_shape("add", 16) == (74, 30, 31)
    assert F.fhe_circuit_shape("mul", 32) == (2824, 120, 528)
    # tree accumulation: five rounds of additions whose ripple carries overlap
    assert F.fhe_circuit_shape("mul_tree", 32) == (2824, 62, 528)
    assert [F.fhe_circuit_shape("mul_tree", w)[1] for w in (8, 16)] == [14, 30]
    assert F.fhe_circuit_shape("karatsuba", 32)[:2] == (5271, 116)
    assert F.fhe_circuit_shape("karatsuba", 16)[:2] == (1457, 58)
    assert F.fhe_circuit_shape("matvec", 16, 64, 64) == (2952576, 68, 557056)


def test_level_schedule_balancing():
    """add16 x 1024 on 256 compute units: ASAP puts 31,744 gates at level 1
    and alternates 2,048 / 1,024 after; balancing moves operand XOR/ANDs with
    slack into the narrow levels so that every level after the first holds one
    round of 2,048 gates (37 rounds instead of 45.5).  Same gates, same
    depth."""
    sched = F.fhe_circuit_schedule("add", 16, 1024)
    assert len(sched) == 30 and sum(sched) == 74 * 1024
    assert sched == [16384] + [2048] * 29
    # one instance: every level is narrow either way, nothing moves
    assert F.fhe_circuit_schedule("add", 16, 1) == [31] + [2, 1] * 14 + [1]
    for kind, w, n in [("mul", 32, 256), ("mul_tree", 32, 256), ("add_fa", 16, 1024), ("karatsuba", 32, 64)]:
        sched = F.fhe_circuit_schedule(kind, w, n)
        gates, depth, _ = F.fhe_circuit_shape(kind, w)
        assert len(sched) == depth and sum(sched) == gates * n
