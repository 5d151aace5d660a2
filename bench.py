"""Benchmark: useful TFLOP/s of the coded product (encode + coded GEMM + peel).

One step = one full coded product C = A.B on the workload: the encode fused
into the coded GEMM launch, then the peel launch, with A, B and the plan
already resident on the GPU.  Useful FLOPs are 2*M*N*K whatever the
redundancy.  The uncoded product on the same operands is timed beside it
(the same GEMM kernel with the identity code, and torch.matmul), the
coded GEMM launch is timed on its own for the roofline, and the float64
oracle is timed on the host for a bounded sample of the same workload.

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0, "fp8": 5000.0, "fp8x2": 5000.0}
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fp32_scale")
    ap.add_argument("--mode", default="straggler", choices=["straggler", "full", "min"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-ref", action="store_true", help="skip the uncoded references")
    ap.add_argument("--cpu-cols", type=int, default=256,
                    help="columns of B in the CPU oracle sample")
    return ap.parse_args()


def gemm_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1904_11563_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith("gemm") and f.endswith(".hip"):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload, prec):
    """HBM bytes per coded-GEMM launch from the committed rocprofv3 counter
    summary, or None when it is missing or the GEMM sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d[f"{workload}:{prec}"]
        if e.get("gemm_source") != gemm_source_hash():
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def cpu_baseline(A, B, ocode, ref_plan, cols):
    """The float64 oracle on the first `cols` columns of B (same A, same code
    and schedule): useful GFLOP/s on the host cores."""
    import numpy as np

    from oracle import pipeline
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    Bs = np.ascontiguousarray(B[:, :cols])
    t0 = time.perf_counter()
    C = pipeline.coded_matmul_ref(A, Bs, ocode, ref_plan)
    dt = time.perf_counter() - t0
    M, K = A.shape
    useful = 2.0 * M * K * cols
    return {"value": useful / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"float64 oracle coded pipeline (encode, {len(ref_plan.computed)} coded "
                      f"products, peel) on A {M}x{K} and the first {cols} of B's columns; "
                      f"{dt:.1f} s", "seconds": dt}, C


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_11563_amd import bpx, inputs

    w = inputs.WORKLOADS[args.workload]
    prec = bpx.PREC_NAMES[w.prec]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    spec = w.code
    t0 = time.perf_counter()
    if spec.kind == "search":
        code = bpx.Code.search(spec.n, spec.k, spec.b, spec.sigma, spec.seed, spec.restarts,
                               spec.iters)
    else:
        code = bpx.Code.mojette(spec.k, spec.b, spec.n, spec.qe)
    code_s = time.perf_counter() - t0
    arrival, lost, mode_name = inputs.arrival_of(w, seed=args.seed)
    mode = {"straggler": bpx.MODE_STRAGGLER if mode_name == "straggler" else bpx.MODE_ERASURE,
            "full": bpx.MODE_FULL, "min": bpx.MODE_MIN}[args.mode]
    t0 = time.perf_counter()
    plan = bpx.Plan(code, arrival, lost, mode, w.M, w.K, w.N, prec)
    plan_us = (time.perf_counter() - t0) * 1e6
    info = plan.info()
    if not info["decodable"]:
        print(json.dumps({"error": "arrival pattern not decodable", "plan": info}), flush=True)
        sys.exit(1)
    plan.upload()

    A, B = inputs.operands(w, seed=args.seed)
    Ad = torch.from_numpy(A).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    Cd = torch.empty((w.M, w.N), dtype=torch.float32, device=dev)
    ws = bpx.alloc_workspace(plan, dev)
    stream = torch.cuda.current_stream()

    def step():
        bpx.coded_matmul(plan, Ad, Bd, Cd, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        bpx.coded_gemm(plan, Ad, Bd, Cd, ws)
        e1.record(stream)
        bpx.peel_decode(plan, ws, Cd)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    gemm_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    peel_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    step_ms = float(np.mean([a.elapsed_time(c) for a, _, c in ev]))
    ms_per_step = wall * 1e3 / args.steps

    useful = 2.0 * w.M * w.N * w.K
    value = useful / (ms_per_step * 1e-3) / 1e12

    # correctness on sampled rows against float64
    Mb = info["Mb"]
    kb = spec.k * spec.b
    rows = np.unique(np.concatenate([np.arange(s * Mb, min((s + 1) * Mb, w.M),
                                               max(1, Mb // 4)) for s in range(kb)]))
    C = Cd.cpu().numpy()
    R = A[rows].astype(np.float64) @ B.astype(np.float64)
    rel_err = float(np.linalg.norm(C[rows] - R) / np.linalg.norm(R))

    # uncoded references on the same operands
    refs = {}
    if not args.no_ref:
        ident = bpx.Code.identity(spec.k, spec.b)
        uplan = bpx.Plan(ident, list(range(spec.k)), 0, bpx.MODE_STRAGGLER, w.M, w.K, w.N, prec)
        uplan.upload()
        Cu = torch.empty_like(Cd)
        for _ in range(3):
            bpx.coded_matmul(uplan, Ad, Bd, Cu, None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            bpx.coded_matmul(uplan, Ad, Bd, Cu, None)
        torch.cuda.synchronize()
        refs["uncoded_own_tflops"] = useful / ((time.perf_counter() - t1) / args.steps) / 1e12
        if w.prec == "f32":
            torch.backends.cuda.matmul.allow_tf32 = False
            for _ in range(3):
                torch.matmul(Ad, Bd, out=Cu)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                torch.matmul(Ad, Bd, out=Cu)
            torch.cuda.synchronize()
            refs["uncoded_torch_tflops"] = useful / ((time.perf_counter() - t1) / args.steps) / 1e12
        best = max(refs.values())
        refs["frac_of_uncoded"] = value / best

    # roofline of the dominant kernel (the coded GEMM)
    n_comp = info["n_computed"]
    gemm_flops = 2.0 * Mb * w.K * w.N * n_comp
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[w.prec]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": load_traffic(w.name, w.prec),
                "kernel": "coded_gemm", "flops_per_launch": gemm_flops,
                "launch_ms": gemm_ms}

    out = {
        "metric": "useful TFLOP/s of coded A.B (encode+GEMM+peel) vs uncoded GEMM at stated rel err",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": w.prec, "data": "synthetic",
        "config": {"workload": w.name, "M": w.M, "K": w.K, "N": w.N,
                   "code": f"{spec.kind}(n={spec.n},k={spec.k},b={spec.b})",
                   "mode": args.mode if mode_name == "straggler" else "erasure",
                   "prefix_m": info["prefix_m"], "n_computed": n_comp,
                   "depth_max": info["depth_max"], "parallelism": "none (1 GPU)"},
        "rel_err": rel_err,
        "times_ms": {"step_events": step_ms, "coded_gemm": gemm_ms, "peel": peel_ms,
                     "plan_host_us": plan_us, "code_build_s": code_s},
        "roofline": roofline,
    }
    out.update(refs)
    if not args.no_cpu:
        from oracle import codes as ocodes
        from oracle.peeling import make_plan
        cinf = code.info()
        ocode = ocodes.Code("array", cinf["n"], cinf["k"], cinf["b"], code.columns())
        ref_plan = make_plan(ocode, list(arrival), lost,
                             {"straggler": 1 if mode_name == "straggler" else 0,
                              "full": 2, "min": 3}[args.mode])
        cb, _ = cpu_baseline(A, B, ocode, ref_plan, min(args.cpu_cols, w.N))
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
