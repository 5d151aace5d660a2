"""Latency model of the coded product: the paper's total computation time

    T = T_e + min over decodable sets S of max_{i in S} T_i + T_d

(Sec. II, Eq. (eqnTtotal) without the transmission terms, which is the T the
paper itself studies), fed with times measured on the GPU.

Mapping onto one GPU.  Node column j is a virtual worker whose b processors
each compute one coded product.  As in the paper's analysis (Sec. IV-A), a
processor's task time is its unit work times an exponential variable of rate
mu; the unit work here is the measured GPU time of one coded product (the
encode is fused into the product, so every symbol costs about the same).  A
column has finished when its b processors have, and the cluster term is the
time at which the arrived columns first peel: the arrival order is the
columns sorted by finishing time and the prefix comes from the library's
planner (bpx_plan_create, STRAGGLER mode), exactly as for a real run.  T_e is
the encode time the master spends (zero when it is fused into the products;
the FP8 encode+quantise pass otherwise); T_d is the peel of the sample's plan
at the measured peel bandwidth.

This is analysis, not the product path: it uses only host calls of the
library (plans), no device memory.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def peel_bytes(plan, M: int, N: int):
    """Algorithmic (read, write) bytes of a plan's peel: a block whose
    releaser's product went to a workspace slot is read there and written to
    C; a block released into C in place is read only if a later release
    subtracts it."""
    sch = plan.schedule()
    Mb = plan.info()["Mb"]
    grid, Nb = plan.grid()           # block s: rows of block row s // grid
    rows = lambda s: max(0, min(Mb, M - (s // grid) * Mb))
    dest = dict(zip(sch["computed"].tolist(), sch["dest"].tolist()))
    used = set(sch["sub_data"].tolist())
    rd = wr = 0
    for s, g in enumerate(sch["releaser"].tolist()):
        d = dest[g]
        if d >= 0 or s in used:
            rd += rows(s) * Nb * 4
        if d >= 0:
            wr += rows(s) * Nb * 4
    return rd, wr


@dataclass
class LatencySample:
    t_encode: float
    t_cluster: float
    t_decode: float
    prefix_m: int

    @property
    def total(self):
        return self.t_encode + self.t_cluster + self.t_decode


def sample(bpx, code, M, K, N, t_unit, peel_bytes_per_s, t_encode=0.0, mu=1.0, samples=1000,
           seed=0, prec=None, two_d=False):
    """Monte Carlo of T over `samples` draws of the processors' task times.
    t_unit: seconds per coded product; peel_bytes_per_s: measured peel
    bandwidth (None or 0: T_d = 0).  Returns the list of LatencySample."""
    inf = code.info()
    n, b = inf["n"], inf["b"]
    rng = np.random.default_rng([seed, 1904])
    prec = bpx.PREC_F32 if prec is None else prec
    cache = {}
    out = []
    for _ in range(samples):
        x = rng.exponential(1.0 / mu, size=(n, b))
        t_col = t_unit * x.max(axis=1)
        order = np.argsort(t_col, kind="stable").astype(np.int32)
        plan = bpx.Plan(code, order, 0, bpx.MODE_STRAGGLER, M, K, N, prec, two_d=two_d)
        m = plan.info()["prefix_m"]
        if not plan.decodable:
            raise ValueError("the code does not decode from all of its columns")
        t_cluster = float(t_col[order[m - 1]])
        key = tuple(order[:m].tolist())
        if key not in cache:
            rd, wr = peel_bytes(plan, M, N)
            cache[key] = (rd + wr) / peel_bytes_per_s if peel_bytes_per_s else 0.0
        out.append(LatencySample(t_encode, t_cluster, cache[key], m))
    return out


def summary(samples):
    """Means of the terms (same units as the inputs) and of the prefix."""
    return {"E_T": float(np.mean([s.total for s in samples])),
            "encode": float(np.mean([s.t_encode for s in samples])),
            "cluster": float(np.mean([s.t_cluster for s in samples])),
            "decode": float(np.mean([s.t_decode for s in samples])),
            "mean_prefix_m": float(np.mean([s.prefix_m for s in samples])),
            "samples": len(samples)}
