"""Seeded synthetic inputs and workload definitions.

This module holds no arithmetic of the method: it only draws operands and
arrival patterns from seeds and names the workloads.  Both the library's
tests/benchmark and the CPU oracle take their inputs from here, so both see
identical float32 bits.

Streams: numpy's PCG64 seeded with SeedSequence([seed, tag]), one tag per
quantity, so that changing one draw never shifts another.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TAG_A, TAG_B, TAG_SCALE, TAG_ARRIVAL, TAG_SHAPE, TAG_CODE = 1, 2, 3, 4, 5, 6


def rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, tag])))


def uniform(seed, tag, shape, lo=-1.0, hi=1.0) -> np.ndarray:
    return rng(seed, tag).uniform(lo, hi, size=shape).astype(np.float32)


def normal(seed, tag, shape) -> np.ndarray:
    return rng(seed, tag).standard_normal(size=shape, dtype=np.float32)


def integers(seed, tag, shape, lo=-8, hi=8) -> np.ndarray:
    return rng(seed, tag).integers(lo, hi + 1, size=shape).astype(np.float32)


def row_scaled(A: np.ndarray, seed: int, lo=1e-3, hi=1e3) -> np.ndarray:
    """Rows of A times factors log-uniform in [lo, hi]."""
    f = np.exp(rng(seed, TAG_SCALE).uniform(np.log(lo), np.log(hi), size=(A.shape[0], 1)))
    return (A * f).astype(np.float32)


def erasure_arrival(seed: int, n: int, n_lost: int):
    """Uniformly chosen erased columns placed last; survivors in random order."""
    perm = rng(seed, TAG_ARRIVAL).permutation(n).astype(np.int32)
    return perm, n_lost


def shifted_exp_arrival(seed: int, n: int, shift=1.0, rate=1.0):
    """Worker completion times T_j = shift + Exp(rate); arrival = stable argsort."""
    t = shift + rng(seed, TAG_ARRIVAL).exponential(1.0 / rate, size=n)
    return np.argsort(t, kind="stable").astype(np.int32), t


# ---------------------------------------------------------------- workloads --

@dataclass
class CodeSpec:
    kind: str            # "search", "mojette", "table1", "table3", "identity"
    n: int
    k: int
    b: int
    sigma: int = 0
    seed: int = 0
    restarts: int = 1
    iters: int = 0
    qe: int = 0
    walk: int = 0        # search acceptance: 0 hill-climb, 1 plateau walk


# Array codes at the workloads' parameters (the paper prints no construction
# for them; they come from the deterministic search).
# (6,4,2): the plateau walk reaches one failing column pair, the fewest the
# Bush bound allows at b = 2 (the hill-climb stops at two).
CODE_642 = CodeSpec("search", n=6, k=4, b=2, sigma=3, seed=0, restarts=8, iters=6000, walk=1)
CODE_1284 = CodeSpec("search", n=12, k=8, b=4, sigma=4, seed=0, restarts=1, iters=40000)
CODE_1282 = CodeSpec("search", n=12, k=8, b=2, sigma=4, seed=0, restarts=1, iters=40000)
CODE_MOJ = CodeSpec("mojette", n=24, k=16, b=8, qe=0)
# Construction B (q_i = 2^qe, odd p_i): sigma = ceil(k / 2^qe) = 4 at k = 8.
CODE_MOJ_B = CodeSpec("mojette", n=12, k=8, b=4, qe=1)


@dataclass
class Workload:
    name: str
    M: int
    K: int
    N: int
    code: CodeSpec
    prec: str
    dist: str            # "uniform", "normal", "rowscaled"
    arrival: str         # "erasure:<n_lost>" or "shiftexp"
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "fp32_small": Workload("fp32_small", 512, 512, 512, CODE_642, "f32", "uniform", "erasure:2"),
    "fp32_scale": Workload("fp32_scale", 8192, 8192, 4096, CODE_1284, "f32", "normal", "shiftexp"),
    "bf16_small": Workload("bf16_small", 512, 512, 512, CODE_642, "bf16x3", "rowscaled",
                           "erasure:2"),
    "fp8_mojette": Workload("fp8_mojette", 16384, 16384, 8192, CODE_MOJ, "fp8", "normal",
                            "erasure:8"),
    # Mojette Construction B at the headline's shape, FP32, a third of the
    # columns erased
    "mojette_b": Workload("mojette_b", 8192, 8192, 4096, CODE_MOJ_B, "f32", "normal",
                          "erasure:4"),
    # the two-dimensional form: A in 4 row blocks, B in 4 column blocks, the
    # (12,8,2) code over the 4 x 4 grid of block products
    "fp32_2d": Workload("fp32_2d", 8192, 8192, 8192, CODE_1282, "f32", "normal", "shiftexp",
                        extra={"two_d": True}),
}


def operands(w: Workload, seed: int = 0):
    """(A, B) float32 for a workload."""
    if w.dist == "uniform":
        A = uniform(seed, TAG_A, (w.M, w.K))
        B = uniform(seed, TAG_B, (w.K, w.N))
    elif w.dist == "normal":
        A = normal(seed, TAG_A, (w.M, w.K))
        B = normal(seed, TAG_B, (w.K, w.N))
    elif w.dist == "rowscaled":
        A = row_scaled(uniform(seed, TAG_A, (w.M, w.K)), seed)
        B = uniform(seed, TAG_B, (w.K, w.N))
    else:
        raise ValueError(w.dist)
    return A, B


def arrival_of(w: Workload, seed: int = 0):
    """(arrival permutation, n_lost, mode name)."""
    if w.arrival.startswith("erasure:"):
        lost = int(w.arrival.split(":")[1])
        perm, lost = erasure_arrival(seed, w.code.n, lost)
        return perm, lost, "erasure"
    if w.arrival == "shiftexp":
        perm, _ = shifted_exp_arrival(seed, w.code.n)
        return perm, 0, "straggler"
    raise ValueError(w.arrival)


def batch_shapes(seed: int, count: int = 256, lo: int = 256, hi: int = 4096, mult: int = 128):
    """count (M, K, N, k) tuples: each dim log-uniform in [lo, hi] rounded to a
    multiple of mult (clamped to [lo, hi]); k drawn from {4, 8}."""
    g = rng(seed, TAG_SHAPE)
    out = []
    for _ in range(count):
        dims = []
        for _ in range(3):
            x = float(np.exp(g.uniform(np.log(lo), np.log(hi))))
            x = int(round(x / mult)) * mult
            dims.append(min(max(x, lo), hi))
        k = 4 if g.integers(0, 2) == 0 else 8
        out.append((dims[0], dims[1], dims[2], k))
    return out
