"""Tile-shape autotuner for the coded GEMM kernels.

For a precision and a set of product shapes, the shapes are grouped into
buckets (log2 of ceil(x/128), clamped to [0, 7], for x = Mb, N, K, the same
buckets the library's table uses); for each bucket one representative coded
product is timed with every compiled tile shape (bpx_force_tile) and the
fastest shape is recorded.  The table is saved as JSON next to this file and
installed with bpx_set_tile_table by load().

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


def load(path: str = TABLE_PATH) -> bool:
    """Install the saved table in the library; False if there is none."""
    from . import bpx
    if not os.path.exists(path):
        return False
    with open(path) as f:
        d = json.load(f)
    table = [-1] * N_ENTRIES
    for k, v in d["entries"].items():
        table[int(k)] = int(v)
    bpx.set_tile_table(table)
    return True


def _time_gemm(bpx, torch, plan, A, B, C, ws, reps):
    for _ in range(2):
        bpx.coded_gemm(plan, A, B, C, ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bpx.coded_gemm(plan, A, B, C, ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(prec_name: str, shapes, codes_by_k, reps: int = 5, seed: int = 0, log=print):
    """shapes: iterable of (M, K, N, k).  Returns {index: best tile}."""
    import torch

    from . import bpx, inputs
    prec = bpx.PREC_NAMES[prec_name]
    reps_by_bucket = {}
    for (M, K, N, k) in shapes:
        kb = k * codes_by_k[k].info()["b"]
        Mb = -(-M // kb)
        key = index(prec, Mb, N, K)
        reps_by_bucket.setdefault(key, []).append((M, K, N, k))
    out = {}
    n_tiles = bpx.tile_count(prec)
    for key, group in sorted(reps_by_bucket.items()):
        group.sort(key=lambda s: s[0] * s[1] * s[2])
        M, K, N, k = group[len(group) // 2]            # median-volume representative
        code = codes_by_k[k]
        n = code.info()["n"]
        arrival, _ = inputs.erasure_arrival(seed, n, n - k)
        plan = bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, prec)
        A = torch.randn(M, K, device="cuda")
        B = torch.randn(K, N, device="cuda")
        C = torch.empty(M, N, device="cuda")
        ws = bpx.alloc_workspace(plan)
        times = []
        for t in range(n_tiles):
            bpx.force_tile(t)
            times.append(_time_gemm(bpx, torch, plan, A, B, C, ws, reps))
        bpx.force_tile(-1)
        best = min(range(n_tiles), key=lambda t: times[t])
        out[key] = best
        log(f"bucket {key}: rep {M}x{K}x{N} k={k}: " +
            " ".join(f"t{t}={x:.3f}ms" for t, x in enumerate(times)) + f" -> t{best}")
    return out


def save(entries: dict, meta: dict, path: str = TABLE_PATH):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    old = {}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f).get("entries", {})
    old.update({str(k): int(v) for k, v in entries.items()})
    with open(path, "w") as f:
        json.dump({"meta": meta, "entries": old}, f, indent=1, sort_keys=True)


def main():
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1904_11563_amd import bpx, inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--prec", default="bf16x3")
    ap.add_argument("--workload", default="batch", choices=["batch"])
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    t0 = time.time()
    c4 = bpx.Code.search(*[getattr(inputs.CODE_642, f) for f in
                           ("n", "k", "b", "sigma", "seed", "restarts", "iters")])
    c8 = bpx.Code.search(*[getattr(inputs.CODE_1282, f) for f in
                           ("n", "k", "b", "sigma", "seed", "restarts", "iters")])
    shapes = inputs.batch_shapes(0, args.count)
    entries = tune(args.prec, shapes, {4: c4, 8: c8}, reps=args.reps)
    save(entries, {"prec": args.prec, "workload": args.workload, "count": args.count,
                   "seconds": round(time.time() - t0, 1)})
    print(f"saved {len(entries)} buckets to {TABLE_PATH}", flush=True)


if __name__ == "__main__":
    main()
