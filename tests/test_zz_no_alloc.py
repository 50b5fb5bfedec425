"""The allocation-free gate batch (fixed scratch array of the library)
through the C ABI: word for word the result of fhe_bootstrap_gate_batch on
two calls in a row, the second smaller than the first, and sizes beyond the
array refused."""
import numpy as np
import pytest

import paper_2005_01945_amd as F
import workloads

pytestmark = pytest.mark.gpu
MAX_GATES = 4096


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    sk, ck = F.fhe_keygen(0)
    return sk, F.Context(ck, 0)


def test_noalloc_equals_batch_twice_then_smaller(env):
    import torch
    sk, ctx = env
    for n, seed in ((MAX_GATES, 60), (1537, 61), (5, 62)):
        ops = workloads.gate_ops(seed, n)
        c0 = sk.encrypt_bits(workloads.bits(seed + 100, n), nonce=50_000_000 + 10_000 * seed)
        c1 = sk.encrypt_bits(workloads.bits(seed + 200, n), nonce=51_000_000 + 10_000 * seed)
        d_ops = torch.from_numpy(ops.copy()).cuda()
        d0, d1 = F.to_device(c0), F.to_device(c1)
        ref, got = torch.empty_like(d0), torch.full_like(d0, 3)
        log(f"no-alloc batch of {n} gates against the allocating batch")
        F.fhe_bootstrap_gate_batch(ctx, d_ops, d0, d1, ref, n)
        torch.cuda.synchronize()
        F.fhe_bootstrap_gate_batch_noalloc(ctx, d_ops, d0, d1, got, n)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    with pytest.raises(F.FheError) as e:
        F.fhe_bootstrap_gate_batch_noalloc(ctx, d_ops, d0, d1, got, MAX_GATES + 1)
    assert e.value.code == F.FHE_EINVAL
