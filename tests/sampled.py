"""Teacher-forced parity of full-size circuits: gates sampled from every level
of a plan are recomputed by the oracle from the very input samples the GPU
gave them, and the oracle's output must equal the GPU's word for word.

A gate's output is a function of its inputs and the keys only, so checking
each sampled gate on the GPU's own inputs checks it at the launch width and
position where the full-size run computed it, without the oracle having to
replay the whole circuit."""
import numpy as np

import paper_2005_01945_amd as F

NO_WIRE = 0xFFFFFFFF
COMPOUND = 0x10000  # op field of a compound gate: COMPOUND | code0 | code1 << 8


def sample_positions(level_off, per_level, seed):
    """Indices into the plan's gate list: per level the first and the last
    gate plus random others, per_level in all (every gate of narrower levels)."""
    rng = np.random.default_rng(seed)
    picks = []
    for L in range(len(level_off) - 1):
        lo, hi = int(level_off[L]), int(level_off[L + 1])
        n = hi - lo
        if n <= per_level:
            picks.append(np.arange(lo, hi))
            continue
        mid = rng.choice(np.arange(1, n - 1), per_level - 2, replace=False)
        picks.append(lo + np.sort(np.concatenate([[0, n - 1], mid])))
    return np.concatenate(picks).astype(np.int64)


def check_sampled_levels(ctx, K, kind, width, A, B, R, count=1, rows=0, cols=0, per_level=64, seed=0, log=print):
    """Recomputes per_level sampled gates of every level with the oracle and
    compares.  Returns (levels, gates checked)."""
    gates, off = F.fhe_debug_plan(ctx, kind, width, count, rows, cols)
    idx = sample_positions(off, per_level, seed)
    g = gates[idx]
    comp = (g[:, 0] & COMPOUND) != 0
    three = (g[:, 4] != NO_WIRE) & ~comp
    two = ~three & ~comp
    m = len(idx)
    # in0, in1, out of every sampled gate, then the third input (three-input
    # gates) or the second output (compound gates) where there is one
    extra = g[:, 4] != NO_WIRE
    wires = np.concatenate([g[:, 1], g[:, 2], g[:, 3], g[extra, 4]])
    words = F.fhe_debug_read_wires(ctx, kind, width, A, B, R, wires, count, rows, cols)
    in0, in1, out = words[:m], words[m:2 * m], words[2 * m:3 * m]
    fourth = np.zeros_like(out)
    fourth[extra] = words[3 * m:]
    log(f"oracle: {m} sampled gates over {len(off) - 1} levels of {kind} (width {width})")
    want = np.empty_like(out)
    if two.any():
        want[two] = K.bootstrap(g[two, 0].astype(np.uint8), in0[two], in1[two])
    if three.any():
        want[three] = K.bootstrap3(g[three, 0].astype(np.uint8), in0[three], in1[three], fourth[three])
    bad = np.nonzero((want[~comp] != out[~comp]).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} sampled gates differ, first at plan position {idx[~comp][bad[0]]}"
    if comp.any():
        codes = np.stack([g[comp, 0] & 0xFF, (g[comp, 0] >> 8) & 0xFF], axis=1).reshape(-1).astype(np.uint8)
        pair = K.bootstrap_compound(codes, in0[comp], in1[comp])
        np.testing.assert_array_equal(out[comp], pair[:, 0])
        np.testing.assert_array_equal(fourth[comp], pair[:, 1])
    return len(off) - 1, m


def pure_cone(gates, inputs):
    """The gates (positions in launch order) whose inputs all come from the
    wire set `inputs` or from earlier gates of the cone."""
    have = set(int(w) for w in inputs)
    cone = []
    for k, (op, a, b, o, c) in enumerate(gates):
        if int(a) in have and int(b) in have and (int(c) == NO_WIRE or int(c) in have):
            have.add(int(o))
            cone.append(k)
    return np.array(cone, np.int64)


def evaluate_cone(K, gates, level_off, cone, input_words):
    """The oracle evaluates the cone's gates level by level from the input
    samples (dict wire -> words); returns dict wire -> words of every wire."""
    val = dict(input_words)
    level_of = np.searchsorted(level_off, cone, side="right") - 1
    for L in np.unique(level_of):
        ks = cone[level_of == L]
        g = gates[ks]
        assert (g[:, 4] == NO_WIRE).all(), "only two-input gates are expected here"
        out = K.bootstrap(g[:, 0].astype(np.uint8), np.stack([val[int(w)] for w in g[:, 1]]),
                          np.stack([val[int(w)] for w in g[:, 2]]))
        for w, words in zip(g[:, 3], out):
            val[int(w)] = words
    return val
