"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Only plaintext workloads live here (integers, bits, gate codes, job streams);
none of the method's arithmetic does.  Keys, masks and noise are drawn inside
the library and inside the oracle, each from its own implementation of the
same counter-based generator definition.

All draws use numpy's PCG64 generator seeded explicitly, so every input is
reproducible from (seed, shape).
"""
from dataclasses import dataclass
from typing import List

import numpy as np

NUM_GATES = 10
GATE_NAMES = ["AND", "NAND", "OR", "NOR", "XOR", "XNOR", "ANDNY", "ANDYN", "ORNY", "ORYN"]
NAND = 1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_uints(seed: int, count: int, width: int) -> np.ndarray:
    """`count` integers uniform in [0, 2^width) as uint64."""
    g = rng(seed)
    if width >= 64:
        return g.integers(0, 2**63, size=count, dtype=np.uint64) * np.uint64(2) + \
            g.integers(0, 2, size=count, dtype=np.uint64)
    return g.integers(0, 1 << width, size=count, dtype=np.uint64)


def uniform_range(seed: int, shape, lo: int, hi: int) -> np.ndarray:
    """Integers uniform in [lo, hi) as uint64 with the given shape."""
    return rng(seed).integers(lo, hi, size=shape, dtype=np.uint64)


def bits(seed: int, count: int) -> np.ndarray:
    return rng(seed).integers(0, 2, size=count, dtype=np.uint8)


def gate_ops(seed: int, count: int) -> np.ndarray:
    return rng(seed).integers(0, NUM_GATES, size=count, dtype=np.uint8)


def truth_table_inputs():
    """The four input pairs (0,0), (0,1), (1,0), (1,1)."""
    return np.array([0, 0, 1, 1], np.uint8), np.array([0, 1, 0, 1], np.uint8)


# --- the paper's workload shapes -------------------------------------------------

@dataclass
class AddWorkload:
    """Batched ripple-carry addition of `count` independent pairs of `width`-bit
    uniform integers."""
    count: int = 1024
    width: int = 16
    seed: int = 1

    def operands(self):
        a = uniform_uints(self.seed, self.count, self.width)
        b = uniform_uints(self.seed + 1000, self.count, self.width)
        return a, b


@dataclass
class MulWorkload:
    """Batched shift-and-add multiplication of `count` pairs (low `width` bits)."""
    count: int = 256
    width: int = 32
    seed: int = 2

    def operands(self):
        a = uniform_uints(self.seed, self.count, self.width)
        b = uniform_uints(self.seed + 1000, self.count, self.width)
        return a, b


@dataclass
class MatvecWorkload:
    """rows x cols matrix times a length-cols vector, entries uniform in
    [0, entry_max), encrypted as `width`-bit integers."""
    rows: int = 64
    cols: int = 64
    width: int = 16
    entry_max: int = 256
    seed: int = 4

    def operands(self):
        M = uniform_range(self.seed, (self.rows, self.cols), 0, self.entry_max)
        x = uniform_range(self.seed + 1000, (self.cols,), 0, self.entry_max)
        return M, x


# --- serving: Poisson stream of mixed jobs --------------------------------------

JOB_KINDS = ["gate", "add16", "add32", "mul32", "matvec8"]
JOB_MIX = [0.40, 0.20, 0.15, 0.15, 0.10]


@dataclass
class Job:
    kind: str
    arrival_s: float
    op: int = 0          # gate code for "gate" jobs
    a: np.ndarray = None  # plaintext operands (bits / integers / matrix)
    b: np.ndarray = None


def job_stream(seed: int, count: int, rate_per_s: float) -> List[Job]:
    """`count` jobs with exponential inter-arrival times (Poisson process of
    rate `rate_per_s`) and kinds drawn from JOB_MIX."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    kinds = g.choice(len(JOB_KINDS), size=count, p=JOB_MIX)
    jobs = []
    for k, (kind_i, at) in enumerate(zip(kinds, t)):
        kind = JOB_KINDS[kind_i]
        sub = rng(seed * 1_000_003 + k)
        if kind == "gate":
            jobs.append(Job(kind, float(at), op=int(sub.integers(0, NUM_GATES)),
                            a=sub.integers(0, 2, size=1, dtype=np.uint8),
                            b=sub.integers(0, 2, size=1, dtype=np.uint8)))
        elif kind in ("add16", "add32", "mul32"):
            w = int(kind[3:])
            jobs.append(Job(kind, float(at),
                            a=sub.integers(0, 1 << w, size=1, dtype=np.uint64),
                            b=sub.integers(0, 1 << w, size=1, dtype=np.uint64)))
        else:
            jobs.append(Job(kind, float(at),
                            a=sub.integers(0, 256, size=(8, 8), dtype=np.uint64),
                            b=sub.integers(0, 256, size=(8,), dtype=np.uint64)))
    return jobs
