"""GPU parity of the integer circuits (level-scheduled batched gates) against
the oracle: bit-exact end to end at sizes the oracle finishes in seconds, and
at the paper-sized workloads bit-exact on sampled outputs plus decryption
equal to plaintext arithmetic on every output."""
import numpy as np
import pytest

import oracle
import paper_2005_01945_amd as F
import workloads
from sampled import check_sampled_levels, evaluate_cone, pure_cone

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    sk, ck = F.fhe_keygen(0)
    return sk, F.Context(ck, 0), oracle.Keys(0)


def gpu_binary(ctx, fn, ca, cb, count, width, keep=None):
    """Runs fn on device copies of ca, cb; with keep = [] the device buffers
    (A, B, R) are appended to it for later wire reads."""
    import torch
    dA, dB = F.to_device(ca), F.to_device(cb)
    dR = torch.empty_like(dA)
    fn(ctx, dA, dB, dR, count, width)
    torch.cuda.synchronize()
    if keep is not None:
        keep.extend([dA, dB, dR])
    return F.to_host(dR)


@pytest.mark.parametrize("width,count", [(1, 2), (4, 3), (7, 5)])
def test_add_bit_exact(env, width, count):
    sk, ctx, K = env
    a = workloads.uniform_uints(10 + width, count, width)
    b = workloads.uniform_uints(20 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=100_000)
    cb = sk.encrypt_uint(b, width, nonce=200_000)
    log(f"add width={width} count={count}")
    got = gpu_binary(ctx, F.fhe_add, ca, cb, count, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a + b) % (1 << width))
    np.testing.assert_array_equal(got, K.add(ca, cb, width))


@pytest.mark.parametrize("width,count", [(1, 2), (4, 3), (16, 2)])
def test_add_numberwise_bit_exact(env, width, count):
    """Number-wise addition (GPU_n, Sec. V-B-1)."""
    sk, ctx, K = env
    a = workloads.uniform_uints(110 + width, count, width)
    b = workloads.uniform_uints(120 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=1_700_000)
    cb = sk.encrypt_uint(b, width, nonce=1_800_000)
    log(f"add_numberwise width={width} count={count}")
    got = gpu_binary(ctx, F.fhe_add_numberwise, ca, cb, count, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a + b) % (1 << width))
    np.testing.assert_array_equal(got, K.add_numberwise(ca, cb, width))


@pytest.mark.parametrize("width,count", [(1, 2), (4, 3), (16, 2)])
def test_add_fa_bit_exact(env, width, count):
    """Full-adder gates (MAJ, XOR3): one level per bit."""
    sk, ctx, K = env
    a = workloads.uniform_uints(130 + width, count, width)
    b = workloads.uniform_uints(140 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=2_300_000)
    cb = sk.encrypt_uint(b, width, nonce=2_400_000)
    log(f"add_fa width={width} count={count}")
    got = gpu_binary(ctx, F.fhe_add_fa, ca, cb, count, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a + b) % (1 << width))
    np.testing.assert_array_equal(got, K.add_fa(ca, cb, width))


@pytest.mark.parametrize("width,count", [(1, 1), (3, 2), (5, 2)])
def test_mul_bit_exact(env, width, count):
    sk, ctx, K = env
    a = workloads.uniform_uints(30 + width, count, width)
    b = workloads.uniform_uints(40 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=300_000)
    cb = sk.encrypt_uint(b, width, nonce=400_000)
    log(f"mul width={width} count={count}")
    got = gpu_binary(ctx, F.fhe_mul, ca, cb, count, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a * b) % (1 << width))
    np.testing.assert_array_equal(got, K.mul(ca, cb, width))


@pytest.mark.parametrize("rows,cols,width", [(2, 3, 3), (1, 1, 2)])
def test_matvec_bit_exact(env, rows, cols, width):
    import torch
    sk, ctx, K = env
    M = workloads.uniform_range(50 + rows, (rows, cols), 0, 1 << width)
    x = workloads.uniform_range(60 + cols, (cols,), 0, 1 << width)
    cm = sk.encrypt_uint(M.reshape(-1), width, nonce=500_000)
    cx = sk.encrypt_uint(x, width, nonce=600_000)
    dM, dx = F.to_device(cm), F.to_device(cx)
    dy = torch.empty((rows, width, F.WORDS), dtype=torch.int32, device="cuda")
    log(f"matvec {rows}x{cols} width={width}")
    F.fhe_matvec(ctx, dM, dx, dy, rows, cols, width)
    torch.cuda.synchronize()
    got = F.to_host(dy)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (M @ x) % (1 << width))
    np.testing.assert_array_equal(got, K.matvec(cm, cx, rows, cols, width))


def test_add16_full_size(env):
    """1024 pairs of uniform uint16 in one level-scheduled run (the benchmark's
    launch configuration and balanced schedule): every sum decrypts correctly,
    pairs 0-7 and the last pair are bit-exact end to end (666 gates), 64
    sampled gates of every level are bit-exact teacher-forced."""
    sk, ctx, K = env
    wl = workloads.AddWorkload()
    a, b = wl.operands()
    ca = sk.encrypt_uint(a, wl.width, nonce=0)
    cb = sk.encrypt_uint(b, wl.width, nonce=1 << 40)
    log("add16 x 1024 pairs")
    dev = []
    got = gpu_binary(ctx, F.fhe_add, ca, cb, wl.count, wl.width, keep=dev)
    np.testing.assert_array_equal(sk.decrypt_uint(got, wl.width), (a + b) % (1 << wl.width))
    pick = list(range(8)) + [wl.count - 1]
    log("oracle: pairs 0-7 and 1023 end to end")
    np.testing.assert_array_equal(got[pick], K.add(ca[pick], cb[pick], wl.width))
    # 64 gates of every level (first, last and random between), teacher-forced
    check_sampled_levels(ctx, K, "add", wl.width, *dev, count=wl.count, seed=2, log=log)


@pytest.mark.parametrize("width,count", [(1, 1), (5, 2), (8, 3)])
def test_mul_tree_bit_exact(env, width, count):
    """Tree accumulation of the partial products (Sec. V-B-2)."""
    sk, ctx, K = env
    a = workloads.uniform_uints(50 + width, count, width)
    b = workloads.uniform_uints(60 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=500_000)
    cb = sk.encrypt_uint(b, width, nonce=600_000)
    log(f"mul_tree width={width} count={count}")
    got = gpu_binary(ctx, F.fhe_mul_tree, ca, cb, count, width)
    np.testing.assert_array_equal(sk.decrypt_uint(got, width), (a * b) % (1 << width))
    np.testing.assert_array_equal(got, K.mul_tree(ca, cb, width))


def test_mul_tree32_decrypts_and_mul_tree16_bit_exact(env):
    """64 pairs of uniform uint32 through the 62-level tree multiplier decrypt
    to the low product; a 16-bit tree product is bit-exact end to end."""
    sk, ctx, K = env
    a = workloads.uniform_uints(80, 64, 32)
    b = workloads.uniform_uints(81, 64, 32)
    ca = sk.encrypt_uint(a, 32, nonce=900_000)
    cb = sk.encrypt_uint(b, 32, nonce=1_000_000)
    log("mul_tree32 x 64 pairs")
    got = gpu_binary(ctx, F.fhe_mul_tree, ca, cb, 64, 32)
    want = (a.astype(object) * b.astype(object)) % (1 << 32)
    np.testing.assert_array_equal(sk.decrypt_uint(got, 32).astype(object), want)
    a16 = workloads.uniform_uints(82, 1, 16)
    b16 = workloads.uniform_uints(83, 1, 16)
    c16a = sk.encrypt_uint(a16, 16, nonce=1_100_000)
    c16b = sk.encrypt_uint(b16, 16, nonce=1_200_000)
    log("mul_tree16 x 1 pair")
    got16 = gpu_binary(ctx, F.fhe_mul_tree, c16a, c16b, 1, 16)
    log("oracle: mul_tree16 (648 gates)")
    np.testing.assert_array_equal(got16, K.mul_tree(c16a, c16b, 16))


@pytest.mark.parametrize("width,count", [(4, 3), (16, 1)])
def test_karatsuba_bit_exact(env, width, count):
    """Full products by Karatsuba's algorithm (Sec. III-B-2): through the base
    product at 4 bits, one level of the recursion at 16 bits (1,457 gates)."""
    import torch
    sk, ctx, K = env
    a = workloads.uniform_uints(90 + width, count, width)
    b = workloads.uniform_uints(95 + width, count, width)
    ca = sk.encrypt_uint(a, width, nonce=1_300_000)
    cb = sk.encrypt_uint(b, width, nonce=1_400_000)
    dA, dB = F.to_device(ca), F.to_device(cb)
    dR = torch.empty((count, 2 * width, F.WORDS), dtype=torch.int32, device="cuda")
    log(f"karatsuba width={width} count={count}")
    F.fhe_mul_karatsuba(ctx, dA, dB, dR, count, width)
    torch.cuda.synchronize()
    got = F.to_host(dR)
    np.testing.assert_array_equal(sk.decrypt_uint(got, 2 * width).astype(object),
                                  a.astype(object) * b.astype(object))
    log(f"oracle: karatsuba width={width}")
    np.testing.assert_array_equal(got, K.karatsuba(ca, cb, width))


def test_karatsuba32_full_products_decrypt(env):
    """32 pairs of uniform uint32: all 64 bits of every product."""
    import torch
    sk, ctx, K = env
    a = workloads.uniform_uints(96, 32, 32)
    b = workloads.uniform_uints(97, 32, 32)
    dA = F.to_device(sk.encrypt_uint(a, 32, nonce=1_500_000))
    dB = F.to_device(sk.encrypt_uint(b, 32, nonce=1_600_000))
    dR = torch.empty((32, 64, F.WORDS), dtype=torch.int32, device="cuda")
    log("karatsuba32 x 32 pairs")
    F.fhe_mul_karatsuba(ctx, dA, dB, dR, 32, 32)
    torch.cuda.synchronize()
    got = sk.decrypt_uint(F.to_host(dR), 64).astype(object)
    np.testing.assert_array_equal(got, a.astype(object) * b.astype(object))


@pytest.mark.parametrize("n,width", [(2, 3), (3, 2)])
def test_matmul_cannon_bit_exact(env, n, width):
    """Cannon's algorithm (Sec. V-B-3) against the oracle."""
    import torch
    sk, ctx, K = env
    rng = np.random.default_rng(100 + n)
    A = rng.integers(0, 1 << width, (n, n)).astype(np.uint64)
    B = rng.integers(0, 1 << width, (n, n)).astype(np.uint64)
    cA = sk.encrypt_uint(A.reshape(-1), width, nonce=1_900_000)
    cB = sk.encrypt_uint(B.reshape(-1), width, nonce=2_000_000)
    dA, dB = F.to_device(cA), F.to_device(cB)
    dC = torch.empty_like(dA)
    log(f"matmul n={n} width={width}")
    F.fhe_matmul(ctx, dA, dB, dC, n, width)
    torch.cuda.synchronize()
    got = F.to_host(dC)
    np.testing.assert_array_equal(sk.decrypt_uint(got.reshape(n * n, width, -1), width).reshape(n, n),
                                  (A @ B) % (1 << width))
    log(f"oracle: matmul n={n} width={width}")
    np.testing.assert_array_equal(got.reshape(n, n, width, -1), K.matmul(cA, cB, n, width))


def test_matmul16_4x4_decrypts(env):
    """The 4 x 4 16-bit product (45,024 gates)."""
    import torch
    sk, ctx, K = env
    rng = np.random.default_rng(104)
    A = rng.integers(0, 1 << 16, (4, 4)).astype(np.uint64)
    B = rng.integers(0, 1 << 16, (4, 4)).astype(np.uint64)
    dA = F.to_device(sk.encrypt_uint(A.reshape(-1), 16, nonce=2_100_000))
    dB = F.to_device(sk.encrypt_uint(B.reshape(-1), 16, nonce=2_200_000))
    dC = torch.empty_like(dA)
    log("matmul 4x4 16-bit")
    F.fhe_matmul(ctx, dA, dB, dC, 4, 16)
    torch.cuda.synchronize()
    got = sk.decrypt_uint(F.to_host(dC).reshape(16, 16, -1), 16).reshape(4, 4).astype(object)
    np.testing.assert_array_equal(got, (A.astype(object) @ B.astype(object)) % (1 << 16))


def test_mul32_full_size(env):
    """256 pairs of uniform uint32 (722,944 gates, 120 levels): every low-32-bit
    product decrypts correctly, pair 0 is bit-exact end to end (2,824 gates),
    64 sampled gates of every level are bit-exact teacher-forced."""
    sk, ctx, K = env
    wl = workloads.MulWorkload()
    a, b = wl.operands()
    ca = sk.encrypt_uint(a, wl.width, nonce=0)
    cb = sk.encrypt_uint(b, wl.width, nonce=1 << 40)
    log("mul32 x 256 pairs")
    dev = []
    got = gpu_binary(ctx, F.fhe_mul, ca, cb, wl.count, wl.width, keep=dev)
    want = (a.astype(object) * b.astype(object)) % (1 << 32)
    np.testing.assert_array_equal(sk.decrypt_uint(got, 32).astype(object), want)
    log("oracle: mul32 pair 0 end to end (2,824 gates)")
    np.testing.assert_array_equal(got[0], K.mul(ca[:1], cb[:1], wl.width)[0])
    check_sampled_levels(ctx, K, "mul", wl.width, *dev, count=wl.count, seed=3, log=log)


def test_mul8_in_wide_batch_bit_exact(env):
    """A 256-pair batch of 8-bit products; pair 0 bit-exact against the oracle."""
    sk, ctx, K = env
    a = workloads.uniform_uints(70, 256, 8)
    b = workloads.uniform_uints(71, 256, 8)
    ca = sk.encrypt_uint(a, 8, nonce=700_000)
    cb = sk.encrypt_uint(b, 8, nonce=800_000)
    log("mul8 x 256 pairs")
    got = gpu_binary(ctx, F.fhe_mul, ca, cb, 256, 8)
    np.testing.assert_array_equal(sk.decrypt_uint(got, 8), (a * b) % 256)
    log("oracle: mul8 pair 0")
    np.testing.assert_array_equal(got[0], K.mul(ca[:1], cb[:1], 8)[0])


def test_matvec8_serving_size_decrypts(env):
    """The 8x8 8-bit product of the serving mix (10,608 gates)."""
    import torch
    sk, ctx, K = env
    M = workloads.uniform_range(80, (8, 8), 0, 256)
    x = workloads.uniform_range(81, (8,), 0, 256)
    cm = sk.encrypt_uint(M.reshape(-1), 8, nonce=900_000)
    cx = sk.encrypt_uint(x, 8, nonce=990_000)
    dy = torch.empty((8, 8, F.WORDS), dtype=torch.int32, device="cuda")
    log("matvec 8x8 8-bit")
    F.fhe_matvec(ctx, F.to_device(cm), F.to_device(cx), dy, 8, 8, 8)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sk.decrypt_uint(F.to_host(dy), 8), (M @ x) % 256)


def test_matvec64_full_size(env):
    """The 64x64 16-bit matrix-vector product with entries in [0, 256)
    (2,952,576 gates in 68 levels, all 4096 products batched per level):
    every output decrypts to M x mod 2^16 (row sums exceed 2^16, so the
    wraparound is exercised), 64 sampled gates of every level are bit-exact
    teacher-forced, and product (0, 0) is bit-exact end to end (648 gates)."""
    import torch
    sk, ctx, K = env
    wl = workloads.MatvecWorkload()
    M, x = wl.operands()
    assert int((M @ x).max()) >= 1 << 16
    cm = sk.encrypt_uint(M.reshape(-1), wl.width, nonce=0)
    cx = sk.encrypt_uint(x, wl.width, nonce=1 << 40)
    dy = torch.empty((wl.rows, wl.width, F.WORDS), dtype=torch.int32, device="cuda")
    log("matvec 64x64 16-bit (2.95 M gates)")
    dM, dx = F.to_device(cm), F.to_device(cx)
    F.fhe_matvec(ctx, dM, dx, dy, wl.rows, wl.cols, wl.width)
    torch.cuda.synchronize()
    got = F.to_host(dy)
    np.testing.assert_array_equal(sk.decrypt_uint(got, wl.width), (M @ x) % (1 << wl.width))
    w, shape = wl.width, dict(rows=wl.rows, cols=wl.cols)
    check_sampled_levels(ctx, K, "matvec", w, dM, dx, dy, seed=4, log=log, **shape)

    # Product (0, 0) end to end: the gates that read only M[0][0] and x[0]
    # (and each other) are that product's multiplier; the oracle evaluates
    # them from the two input integers and every one of their words must
    # equal the GPU's, and the oracle's own 16-bit multiplier (its own
    # wiring) must produce the cone's 16 output words.
    gates, off = F.fhe_debug_plan(ctx, "matvec", w, 1, **shape)
    cmf, cxf = cm.reshape(-1, F.WORDS), cx.reshape(-1, F.WORDS)
    inputs = {int(k): cmf[k] for k in range(w)}  # region A (M), samples 0..w-1 = M[0][0]
    inputs.update({(1 << 30) | k: cxf[k] for k in range(w)})  # region B (x), x[0]
    cone = pure_cone(gates, inputs.keys())
    assert len(cone) == F.fhe_circuit_shape("mul", w)[0] == 648
    log(f"oracle: product (0,0), {len(cone)} gates end to end")
    val = evaluate_cone(K, gates, off, cone, inputs)
    outs = gates[cone, 3]
    gpu = F.fhe_debug_read_wires(ctx, "matvec", w, dM, dx, dy, outs, 1, **shape)
    np.testing.assert_array_equal(gpu, np.stack([val[int(o)] for o in outs]))
    inner = set(int(v) for v in gates[cone][:, 1:3].reshape(-1))
    last = [i for i, o in enumerate(outs) if int(o) not in inner]  # no gate of the cone reads them
    own = K.mul(cmf[:w].reshape(1, w, -1), cxf[:w].reshape(1, w, -1), w)[0]
    assert len(last) == w
    assert {r.tobytes() for r in own} == {gpu[i].tobytes() for i in last}


def test_custom_circuit_bit_exact(env):
    """A caller-defined random DAG (two- and three-input gates, outputs taken
    from several depths) over 5 instances, against the oracle evaluating the
    same gates one by one; invalid circuits are refused."""
    import torch
    sk, ctx, K = env
    rng = np.random.default_rng(150)
    n_in, n_gates, count = 6, 60, 5
    gates = []
    for k in range(n_gates):
        lim = n_in + k
        op = int(rng.integers(0, 12))
        a, b, c = (int(rng.integers(max(0, lim - 12), lim)) for _ in range(3))
        gates.append((op, a, b, c) if op >= 10 else (op, a, b))
    outputs = [n_in + k for k in (5, 23, 40, 59, 58)]
    circ = F.Circuit(ctx, gates, n_in, outputs)
    bits = rng.integers(0, 2, (count, n_in))
    cin = sk.encrypt_bits(bits.reshape(-1).tolist(), nonce=2_500_000).reshape(count, n_in, -1)
    d_in = F.to_device(cin)
    d_out = torch.empty((count, len(outputs), F.WORDS), dtype=torch.int32, device="cuda")
    log("custom circuit: 60 gates x 5 instances")
    circ.run(d_in, d_out, count)
    torch.cuda.synchronize()
    got = F.to_host(d_out)
    # the oracle: wire by wire, all instances of one gate in one call
    wires = [cin[:, i, :] for i in range(n_in)]
    for g in gates:
        if g[0] >= 10:
            wires.append(K.bootstrap3([g[0]] * count, wires[g[1]], wires[g[2]], wires[g[3]], threads=8))
        else:
            wires.append(K.bootstrap([g[0]] * count, wires[g[1]], wires[g[2]], threads=8))
    want = np.stack([wires[o] for o in outputs], axis=1)
    np.testing.assert_array_equal(got, want)
    # plaintext check of the outputs through decryption
    vals = [bits[:, i] for i in range(n_in)]
    tt = [lambda x, y: x & y, lambda x, y: 1 - (x & y), lambda x, y: x | y, lambda x, y: 1 - (x | y),
          lambda x, y: x ^ y, lambda x, y: 1 - (x ^ y), lambda x, y: (1 - x) & y, lambda x, y: x & (1 - y),
          lambda x, y: (1 - x) | y, lambda x, y: x | (1 - y)]
    for g in gates:
        if g[0] == F.MAJ:
            vals.append((vals[g[1]] + vals[g[2]] + vals[g[3]] >= 2).astype(int))
        elif g[0] == F.XOR3:
            vals.append((vals[g[1]] + vals[g[2]] + vals[g[3]]) & 1)
        else:
            vals.append(tt[g[0]](vals[g[1]], vals[g[2]]))
    dec = sk.decrypt_bits(got.reshape(-1, F.WORDS)).reshape(count, len(outputs))
    np.testing.assert_array_equal(dec, np.stack([vals[o] for o in outputs], axis=1))
    circ.close()
    for bad_gates, bad_out in [([(0, 0, 7)], [6]), ([(12, 0, 1)], [6]), ([(0, 0, 1)], [0]), ([(0, 0, 1)], [6, 6]),
                               ([(10, 0, 1, 6)], [6])]:
        with pytest.raises(F.FheError):
            F.Circuit(ctx, bad_gates, n_in, bad_out)
