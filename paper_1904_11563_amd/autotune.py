"""Tile-shape autotuner for the grouped BF16 / BF16x3 coded GEMM.

Products are grouped into shape buckets (log2 of ceil(x/128), clamped to
[0, 7], for x = Mb, N, K: the buckets of the library's table).  Tiles are
tuned where they are used, inside one grouped launch of the whole batch:
starting from the library's default shape for every product, each bucket
(largest total work first) tries every compiled shape for its products
while the others keep theirs, and keeps the shape that gives the shortest
grouped GEMM phase.  A change must beat the default, timed again in the
same round, by more than 1 % and by no more than 1.5 times the bucket's
share of the work (a bucket cannot save more than its own time; larger
"gains" are noise).  Timing products
one at a time misleads here: a small product alone cannot fill the GPU with
large tiles, but inside the batch every CU is busy anyway.

The table is saved as JSON next to this file and installed with
bpx_set_tile_table by load().

Run on the GPU:  python -m paper_1904_11563_amd.autotune [--prec bf16x3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tuning", "tiles.json")
N_ENTRIES = 8 * 8 * 8 * 5


def bucket(x: int) -> int:
    v = (x + 127) // 128
    b = 0
    while v > 1 and b < 7:
        v >>= 1
        b += 1
    return b


def index(prec: int, Mb: int, N: int, K: int) -> int:
    return ((prec * 8 + bucket(Mb)) * 8 + bucket(N)) * 8 + bucket(K)


KERNEL_SOURCE = os.path.join(HERE, "csrc", "gemm_bf16.hip")
# The library's BF16 / BF16x3 shape where the table has no entry (the flat
# 128 x 256 tiling, tile 4 of bpx_tile_count): an entry naming it would be
# no override at all.
DEFAULT_TILE = 4


def kernel_source_hash() -> str:
    """Hash of the source holding the tuned kernels: a table measured on
    other kernels is stale."""
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load(path: str = TABLE_PATH) -> str:
    """Install the saved table in the library if it was measured on the
    current kernels.  Returns what the grouped launch will use: "none" (no
    table), "stale" (measured on other kernels; not installed), "default
    won every bucket" (a current table with no override), or
    "autotuned (n overrides)"."""
    from . import bpx
    if not os.path.exists(path):
        return "none"
    with open(path) as f:
        d = json.load(f)
    if d.get("meta", {}).get("gemm_source") != kernel_source_hash():
        return "stale"
    table = [-1] * N_ENTRIES
    for k, v in d["entries"].items():
        table[int(k)] = int(v)
    bpx.set_tile_table(table)
    n = len(d["entries"])
    return f"autotuned ({n} overrides)" if n else "default won every bucket"


def accept(ref_ms: float, best_ms: float, share: float) -> bool:
    """Keep a bucket's best candidate over the default (timed in the same
    round, ref_ms) only if it wins by more than 1 % and by no more than 1.5
    times the bucket's share of the work: a bucket cannot save more than its
    own time, so a larger "gain" is run-to-run noise (1-2 % on this phase)."""
    gain = ref_ms - best_ms
    return gain > 0.01 * ref_ms and gain <= 1.5 * share * ref_ms


def _gemm_phase_ms(bpx, torch, plans, As, Bs, Cs, ws, reps):
    """Shortest of `reps` timings of the grouped GEMM phase (group built with
    the table currently installed)."""
    group = bpx.Group(plans, As, Bs, Cs, ws)
    group.launch_phase(0)                      # B split, once
    for _ in range(2):
        group.launch_phase(1)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        group.launch_phase(1)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del group
    return best


def tune_grouped(prec_name: str, shapes, codes_by_k, reps: int = 5, seed: int = 0, log=print):
    """shapes: (M, K, N, k) tuples of one batch.  Returns {index: tile}."""
    import torch

    from . import bpx, inputs
    prec = bpx.PREC_NAMES[prec_name]
    dev = torch.device("cuda:0")
    plans, As, Bs, Cs, keys, work = [], [], [], [], [], {}
    for i, (M, K, N, k) in enumerate(shapes):
        code = codes_by_k[k]
        n = code.info()["n"]
        arrival, _ = inputs.erasure_arrival(seed * 1000 + i, n, n - k)
        plan = bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, prec)
        inf = plan.info()
        key = index(prec, inf["Mb"], N, K)
        plans.append(plan)
        keys.append(key)
        work[key] = work.get(key, 0.0) + 2.0 * inf["Mb"] * inf["n_computed"] * K * N
        As.append(torch.randn(M, K, device=dev))
        Bs.append(torch.randn(K, N, device=dev))
        Cs.append(torch.empty(M, N, device=dev))
    ws = torch.empty(bpx.group_workspace_bytes(plans), dtype=torch.uint8, device=dev)
    n_tiles = bpx.tile_count(prec)
    table = [-1] * N_ENTRIES
    bpx.set_tile_table(table)
    best = _gemm_phase_ms(bpx, torch, plans, As, Bs, Cs, ws, reps)
    log(f"default shapes: grouped GEMM {best:.3f} ms")
    chosen = {}
    total = sum(work.values())
    for key in sorted(work, key=lambda x: -work[x]):
        cur = table[key]
        # the bucket's current choice is timed again in the same round as
        # the candidates, so that a slow drift of the clock is no win
        bpx.set_tile_table(table)
        ref = _gemm_phase_ms(bpx, torch, plans, As, Bs, Cs, ws, reps)
        times = {}
        for t in range(n_tiles):
            if t == DEFAULT_TILE:
                continue  # the default is what the reference run used
            table[key] = t
            bpx.set_tile_table(table)
            times[t] = _gemm_phase_ms(bpx, torch, plans, As, Bs, Cs, ws, reps)
        t_best = min(times, key=times.get)
        if accept(ref, times[t_best], work[key] / total):
            table[key] = t_best
            best = times[t_best]
        else:
            table[key] = cur
            best = ref
        chosen[key] = table[key]
        log(f"bucket {key} ({work[key] / 1e9:.1f} GFLOP, {100 * work[key] / total:.1f} %): "
            f"default={ref:.3f} " +
            " ".join(f"t{t}={x:.3f}" for t, x in times.items()) +
            f" -> {'t%d' % table[key] if table[key] >= 0 else 'default'} (total {best:.3f} ms)")
    bpx.set_tile_table(table)
    return {k: v for k, v in chosen.items() if v >= 0}, best


def save(entries: dict, meta: dict, path: str = TABLE_PATH):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"meta": meta, "entries": {str(k): int(v) for k, v in entries.items()}}, f,
                  indent=1, sort_keys=True)


def main():
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1904_11563_amd import bpx, inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--prec", default="bf16x3")
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    t0 = time.time()
    c4 = bpx.Code.search(*[getattr(inputs.CODE_642, f) for f in
                           ("n", "k", "b", "sigma", "seed", "restarts", "iters", "walk")])
    c8 = bpx.Code.search(*[getattr(inputs.CODE_1282, f) for f in
                           ("n", "k", "b", "sigma", "seed", "restarts", "iters", "walk")])
    shapes = inputs.batch_shapes(0, args.count)
    entries, ms = tune_grouped(args.prec, shapes, {4: c4, 8: c8}, reps=args.reps)
    save(entries, {"prec": args.prec, "workload": "batch", "count": args.count,
                   "criterion": "grouped GEMM phase of the whole batch",
                   "grouped_gemm_ms": round(ms, 4), "seconds": round(time.time() - t0, 1),
                   "gemm_source": kernel_source_hash()})
    print(f"saved {len(entries)} bucket overrides to {TABLE_PATH}", flush=True)


if __name__ == "__main__":
    main()
