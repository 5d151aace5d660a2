"""Benchmark: useful TFLOP/s of the coded product (encode + coded GEMM + peel).

Default workload (the headline): FP32, A 8192x8192, B 8192x4096 N(0,1), the
(12,8,4) array code, shifted-exponential worker times; the decode uses the
first arrived columns that peel, and every symbol of those columns is
computed.  One step = one whole coded product: the coded-GEMM launch (encode
fused into its A loads) and the peel launch, operands already resident on
the GPU.  Useful FLOPs are 2*M*N*K whatever the redundancy.

Beside it: the same kernels on the identity code (uncoded), torch.matmul on
the same operands, the dominant kernel's roofline from HIP events over the
timed region, and the float64 oracle on the host for a bounded sample.

Other workloads (--workload): fp32_small, bf16_small (split-BF16x3),
fp8_mojette (FP8x2, Mojette Construction A), mojette_b (FP32, Mojette
Construction B at the headline's shape), fp32_2d (FP32, the two-dimensional
form: A row blocks times B column blocks), batch (256 uneven products, one
grouped launch sequence captured in a HIP graph).

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

# MI355X dense peaks (TFLOP/s).  A split-BF16x3 product issues 3 BF16 MFMA
# passes and FP8x2 two FP8 passes per useful flop, so their effective peaks
# are the BF16 / FP8 peak divided by 3 / 2.
PEAK = {"f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0 / 3, "fp8": 5000.0, "fp8x2": 2500.0}
METRIC = "useful TFLOP/s of coded A.B (encode+GEMM+peel) vs uncoded GEMM at stated rel err"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fp32_scale",
                    choices=["fp32_scale", "fp32_small", "bf16_small", "fp8_mojette", "mojette_b",
                             "fp32_2d", "batch"])
    ap.add_argument("--prec", default=None, help="override the workload's precision")
    ap.add_argument("--mode", default="arrival", choices=["arrival", "full", "min"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-ref", action="store_true", help="skip the uncoded references")
    ap.add_argument("--tile", type=int, default=-1,
                    help="force one GEMM tile shape (bpx_force_tile) instead of the defaults")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="rough budget of the CPU oracle sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    return ap.parse_args()


GEMM_SOURCE = {"f32": "gemm_f32.hip", "bf16": "gemm_bf16.hip", "bf16x3": "gemm_bf16.hip",
               "fp8": "gemm_fp8.hip", "fp8x2": "gemm_fp8.hip"}


def source_hash(name):
    """Hash of one kernel source file under the package's csrc/."""
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_1904_11563_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload, prec, source):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if missing, taken on another kernel
    source, or taken on another form of the step (source = the file that
    holds the kernel the roofline names)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        e = json.load(open(path))[f"{workload}:{prec}"]
        if e.get("gemm_source_file") != source or e.get("gemm_source") != source_hash(source):
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def timed(torch, fn, steps, stream=None):
    """Mean milliseconds of fn over `steps` calls (events on the stream)."""
    s = stream or torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def capture(torch, fn):
    """A HIP graph holding the launches of fn (captured on a side stream)."""
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                     # warm, not captured
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return graph


def graph_ms(torch, fn, steps, warmup=3):
    """Mean wall milliseconds per replay of fn captured in a HIP graph,
    bracketed by device synchronisation."""
    g = capture(torch, fn)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def build_code(bpx, spec):
    if spec.kind == "search":
        return bpx.Code.search(spec.n, spec.k, spec.b, spec.sigma, spec.seed, spec.restarts,
                               spec.iters, walk=spec.walk)
    return bpx.Code.mojette(spec.k, spec.b, spec.n, spec.qe)


def oracle_code(code):
    from oracle import codes as ocodes
    inf = code.info()
    return ocodes.Code("array", inf["n"], inf["k"], inf["b"], code.columns())


def header(args, value, ms, prec, config):
    return {"metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
            "data": "synthetic", "config": config}


# ----------------------------------------------------------- single product --

def run_single(args):
    import numpy as np
    import torch

    from paper_1904_11563_amd import autotune, bpx, inputs

    autotune.load()
    if args.tile >= 0:
        bpx.force_tile(args.tile)
    w = inputs.WORKLOADS[args.workload]
    prec_name = args.prec or ("fp8x2" if w.prec == "fp8" else w.prec)
    prec = bpx.PREC_NAMES[prec_name]
    dev = torch.device("cuda:0")
    spec = w.code
    t0 = time.perf_counter()
    code = build_code(bpx, spec)
    code_s = time.perf_counter() - t0
    arrival, lost, mode_name = inputs.arrival_of(w, seed=args.seed)
    if args.mode == "full":
        mode = bpx.MODE_FULL
    elif args.mode == "min":
        mode = bpx.MODE_MIN
    else:
        mode = bpx.MODE_STRAGGLER if mode_name == "straggler" else bpx.MODE_ERASURE
    t0 = time.perf_counter()
    two_d = bool(w.extra.get("two_d"))
    plan = bpx.Plan(code, arrival, lost, mode, w.M, w.K, w.N, prec, two_d=two_d)
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

    fused = plan.fused()
    for _ in range(args.warmup):
        bpx.coded_matmul(plan, Ad, Bd, Cd, ws)
    torch.cuda.synchronize()

    # timed region: K whole steps, each one replay of a HIP graph holding the
    # step's launches (coded GEMM + peel, or the one fused launch)
    step_graph = capture(torch, lambda: bpx.coded_matmul(plan, Ad, Bd, Cd, ws))
    for _ in range(args.warmup):
        step_graph.replay()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step_graph.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = wall * 1e3 / args.steps

    # per-launch durations: events on the launch stream around each launch
    # (the fused form: around all K launches back to back, so that a launch
    # shorter than its own event overhead is not inflated by it)
    if fused:
        gemm_ms = timed(torch, lambda: bpx.coded_matmul(plan, Ad, Bd, Cd, ws), args.steps,
                        stream)
        peel_ms = 0.0
    else:
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
              for _ in range(args.steps)]
        for e0, e1, e2 in ev:
            e0.record(stream)
            bpx.coded_gemm(plan, Ad, Bd, Cd, ws)
            e1.record(stream)
            bpx.peel_decode(plan, ws, Cd)
            e2.record(stream)
        torch.cuda.synchronize()
        gemm_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
        peel_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))

    # cost of one graph replay itself: a graph of one one-element kernel,
    # replayed back to back as the step is
    x1 = torch.zeros(1, device=dev)
    replay_floor_ms = graph_ms(torch, lambda: x1.add_(1.0), args.steps, warmup=args.warmup)

    useful = 2.0 * w.M * w.N * w.K
    value = useful / (ms * 1e-3) / 1e12

    # error on sampled rows (up to four per data block, about 256 in all)
    # against float64
    Mb = info["Mb"]
    kb = spec.k * spec.b
    per = max(1, min(4, 256 // kb))
    rows = np.unique(np.concatenate([np.arange(s * Mb, min((s + 1) * Mb, w.M),
                                               max(1, Mb // per))[:per] for s in range(kb)]))
    C = Cd.cpu().numpy()
    R = A[rows].astype(np.float64) @ B.astype(np.float64)
    rel_err = float(np.linalg.norm(C[rows] - R) / np.linalg.norm(R))
    worst = worst_errors(C[rows], R, rows, Mb)

    refs = {}
    if not args.no_ref:
        ref_prec = bpx.PREC_BF16 if prec_name.startswith("fp8") else prec
        ident = bpx.Code.identity(spec.k, spec.b)
        uplan = bpx.Plan(ident, list(range(spec.k)), 0, bpx.MODE_STRAGGLER, w.M, w.K, w.N,
                         prec=ref_prec, two_d=two_d)
        uplan.upload()
        uws = bpx.alloc_workspace(uplan, dev)
        Cu = torch.empty_like(Cd)
        for _ in range(3):
            bpx.coded_matmul(uplan, Ad, Bd, Cu, uws)
        refs["uncoded_own_tflops"] = useful / (graph_ms(
            torch, lambda: bpx.coded_matmul(uplan, Ad, Bd, Cu, uws), args.steps) * 1e-3) / 1e12
        refs["uncoded_own_prec"] = [k for k, v in bpx.PREC_NAMES.items() if v == ref_prec][0]
        if prec_name == "f32":
            torch.backends.cuda.matmul.allow_tf32 = False
            X, Y = Ad, Bd
            tprec = "f32"
        else:
            X, Y = Ad.to(torch.bfloat16), Bd.to(torch.bfloat16)
            tprec = "bf16"
        Ct = torch.empty((w.M, w.N), dtype=X.dtype, device=dev)
        for _ in range(3):
            torch.matmul(X, Y, out=Ct)
        refs["uncoded_torch_tflops"] = useful / (graph_ms(
            torch, lambda: torch.matmul(X, Y, out=Ct), args.steps) * 1e-3) / 1e12
        refs["uncoded_torch_prec"] = tprec
        refs["frac_of_uncoded_best"] = value / max(refs["uncoded_own_tflops"],
                                                   refs["uncoded_torch_tflops"])
        refs["frac_of_uncoded_own"] = value / refs["uncoded_own_tflops"]

    hbm = hbm_kernels(torch, bpx, plan, code, Ad, Bd, Cd, ws, w, info, args.steps, two_d)

    n_comp = info["n_computed"]
    gemm_flops = 2.0 * Mb * w.K * w.N * n_comp
    if two_d:   # Mb x Nb products; a gray symbol takes one pass per member
        grid, Nb = plan.grid()
        col_ptr, sym_ptr, sym_data = code.csr()
        passes = 0
        for g in plan.schedule()["computed"].tolist():
            mem = [int(x) for x in sym_data[sym_ptr[g]:sym_ptr[g + 1]]]
            rs, cs = {x // grid for x in mem}, {x % grid for x in mem}
            passes += 1 if (len(rs) == 1 or len(cs) == 1) else len(mem)
        gemm_flops = 2.0 * Mb * w.K * Nb * passes
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12
    if two_d:
        full = Mb % 256 == 0 and Nb % 256 == 0 and w.K % 32 == 0 and grid * Mb == w.M
        f32_kernel = ("coded_gemm_2d_wide_kernel (256x256 tiles of block products, symbols "
                      "dealt by decreasing passes)" if full else
                      "coded_gemm_2d_kernel (64x128 tiles of block products)")
    elif fused:
        f32_kernel = ("fused_f32_kernel (coded products of 16-row tiles of every block and "
                      "the peel in LDS, one launch)")
    elif Mb % 256 == 0 and w.N % 256 == 0 and w.K % 32 == 0 and w.M % Mb == 0:
        f32_kernel = ("coded_gemm_f32_wide_kernel<4,2> (full rounds of 256x256 tiles; a short "
                      "last round split along K + splitk_reduce_kernel, or as "
                      "coded_gemm_f32_kernel<64,128,32,2> sub-tiles), one call")
    else:
        f32_kernel = "coded_gemm_f32_kernel<64,128,32,2>"
    bf16_kernel = ("fused_bf16_kernel (coded products and peel, one launch)" if fused else
                   "split_b + coded_gemm_bf16_flat_kernel, one call")
    kernel = {"f32": f32_kernel, "bf16": bf16_kernel, "bf16x3": bf16_kernel,
              "fp8": "quant_b + quant_a + coded_gemm_fp8_wide_kernel, one call",
              "fp8x2": "quant_b + quant_a + coded_gemm_fp8_wide_kernel, one call"}[prec_name]
    source = "gemm2d.hip" if two_d else "fused.hip" if fused else GEMM_SOURCE[prec_name]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec_name],
                "unit": "TFLOP/s", "frac": achieved / PEAK[prec_name],
                "traffic": load_traffic(w.name, prec_name, source), "kernel": kernel,
                "flops_per_launch": gemm_flops, "launch_ms": gemm_ms}
    cfg = {"workload": w.name, "M": w.M, "K": w.K, "N": w.N,
           "code": f"{spec.kind}(n={spec.n},k={spec.k},b={spec.b})",
           "mode": args.mode if args.mode != "arrival" else mode_name,
           "prefix_m": info["prefix_m"], "n_computed": n_comp, "kb": kb,
           "depth_max": info["depth_max"], "parallelism": "none (1 GPU)"}
    out = header(args, value, ms, prec_name, cfg)
    out.update({"rel_err": rel_err, "rel_err_sample": f"{len(rows)} rows x all columns",
                "rel_err_worst": worst,
                # the plan (arrival prefix + schedule, host) is made once per
                # arrival pattern, outside the timed region; with it per step:
                "ms_per_step_incl_plan": ms + plan_us * 1e-3,
                "value_incl_plan": useful / ((ms + plan_us * 1e-3) * 1e-3) / 1e12,
                "timing": "HIP graph replay of each step (and of each reference)",
                "times_ms": {("fused_call" if fused else "coded_gemm_call"): gemm_ms,
                             "peel": peel_ms, "plan_host_us": plan_us, "code_build_s": code_s,
                             "graph_replay_floor": replay_floor_ms},
                "roofline": roofline, "hbm": hbm})
    out.update(refs)
    out["latency_model"] = latency_model(bpx, code, w, prec, gemm_ms, n_comp, hbm, refs, spec)
    if two_d:
        cfg["form"] = "two-dimensional (A row blocks x B column blocks)"
        cfg["grid"] = plan.grid()[0]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_single(A, B, code, arrival, lost, mode, w, args.cpu_seconds,
                                         two_d)
    return out


def worst_errors(C, R, rows, Mb):
    """Worst relative error over the sampled rows and over the data blocks'
    sampled rows (the Frobenius error of the whole sample hides rows whose
    error grew along a release chain or through cancellation)."""
    import numpy as np
    num = np.sum((C.astype(np.float64) - R) ** 2, axis=1)
    den = np.maximum(np.sum(R ** 2, axis=1), 1e-300)
    per_row = np.sqrt(num / den)
    blocks = np.asarray(rows) // Mb
    best_b, best_e = -1, -1.0
    for b in np.unique(blocks):
        m = blocks == b
        e = float(np.sqrt(num[m].sum() / den[m].sum()))
        if e > best_e:
            best_b, best_e = int(b), e
    return {"row": float(per_row.max()), "row_at": int(rows[int(per_row.argmax())]),
            "block": best_e, "block_at": best_b}


def latency_model(bpx, code, w, prec, gemm_ms, n_comp, hbm, refs, spec, samples=500):
    """The paper's T = T_e + min_S max_{i in S} T_i + T_d with exponential
    task times (rate 1 per unit of work), the unit being the measured GPU
    time of one coded product and the peel at its measured bandwidth; the
    uncoded case runs the identity code at the uncoded product's time."""
    from paper_1904_11563_amd import latency
    gbps = hbm["peel"]["GBps"]
    res = {"unit": "us", "mu": 1.0, "model": "column done when its b products are; "
           "prefix from the library planner; encode fused into the products"}
    two_d = bool(w.extra.get("two_d"))
    lm = latency.summary(latency.sample(bpx, code, w.M, w.K, w.N, gemm_ms * 1e-3 / n_comp,
                                        gbps * 1e9 if gbps else None, samples=samples, prec=prec,
                                        two_d=two_d))
    res["coded"] = {k: (v * 1e6 if k in ("E_T", "encode", "cluster", "decode") else v)
                    for k, v in lm.items()}
    if refs.get("uncoded_own_tflops"):
        kb = spec.k * spec.b
        t_u = 2.0 * w.M * w.K * w.N / (refs["uncoded_own_tflops"] * 1e12) / kb
        ident = bpx.Code.identity(spec.k, spec.b)
        lu = latency.summary(latency.sample(bpx, ident, w.M, w.K, w.N, t_u, None,
                                            samples=samples, prec=prec, two_d=two_d))
        res["uncoded"] = {k: (v * 1e6 if k in ("E_T", "encode", "cluster", "decode") else v)
                          for k, v in lu.items()}
    return res


def hbm_kernels(torch, bpx, plan, code, Ad, Bd, Cd, ws, w, info, steps, two_d=False):
    """Achieved HBM GB/s of the two streaming kernels: the standalone encode
    (bpx_encode) and the peel, each as algorithmic bytes / event time.  (A
    plan that takes the fused form runs neither in its step; they are
    measured on the same plan for reference.)"""
    sch = plan.schedule()
    col_ptr, sym_ptr, sym_data = code.csr()
    Mb, K, N, M = info["Mb"], w.K, w.N, w.M
    from paper_1904_11563_amd.latency import peel_bytes
    rd, wr = peel_bytes(plan, M, N)
    bpx.coded_gemm(plan, Ad, Bd, Cd, ws)   # the peel below reads these products
    peel_ms = timed(torch, lambda: bpx.peel_decode(plan, ws, Cd), steps)
    res = {"peak_GBps": 8000.0}
    legs = [("peel", rd + wr, peel_ms)]
    if not two_d:   # the stand-alone encode exists for row-block plans
        rows = lambda s: max(0, min(Mb, M - s * Mb))
        comp = sch["computed"].tolist()
        enc_read = sum(rows(int(s)) * K * 4 for g in comp
                       for s in sym_data[sym_ptr[g]:sym_ptr[g + 1]])
        enc_write = len(comp) * Mb * K * 4
        _, enc_bytes = plan.workspace_bytes()
        out_enc = torch.empty(enc_bytes // 4, dtype=torch.float32, device=Ad.device)
        bpx.encode(plan, Ad, out_enc)
        enc_ms = timed(torch, lambda: bpx.encode(plan, Ad, out_enc), steps)
        del out_enc
        legs.insert(0, ("encode", enc_read + enc_write, enc_ms))
    for name, b, t in legs:
        res[name] = {"bytes": b, "ms": t, "GBps": b / (t * 1e-3) / 1e9 if t > 0 else None,
                     "frac": (b / (t * 1e-3) / 1e9) / 8000.0 if t > 0 else None}
    return res


def cpu_single(A, B, code, arrival, lost, mode, w, budget, two_d=False):
    """The float64 oracle's coded pipeline on A and the first columns of B,
    the column count scaled so the run takes about `budget` seconds."""
    import numpy as np

    from oracle import pipeline, pipeline2d
    from oracle.peeling import make_plan
    oc = oracle_code(code)
    ref_plan = make_plan(oc, list(arrival), lost, mode)
    ref = pipeline2d.coded_matmul_ref if two_d else pipeline.coded_matmul_ref
    def timed_run(c):
        t0 = time.perf_counter()
        ref(A, np.ascontiguousarray(B[:, :c]), oc, ref_plan)
        return time.perf_counter() - t0

    # time = fixed (the encode of A, independent of the columns) + per column;
    # two small runs fit both, then the sample is as many columns as fit the
    # budget, or the whole product repeated until the budget is used
    c1, c2 = min(64, w.N), min(256, w.N)
    t1, t2 = timed_run(c1), timed_run(c2)
    per_col = max((t2 - t1) / max(c2 - c1, 1), 1e-9)
    fixed = max(t1 - c1 * per_col, 0.0)
    cols = int((budget - fixed) / per_col)
    cols = max(c1, min(w.N, cols - cols % 64))
    reps, dt = 0, 0.0
    while reps == 0 or (cols == w.N and dt < budget and reps < 100):
        dt += timed_run(cols)
        reps += 1
    useful = 2.0 * w.M * w.K * cols * reps
    what = (f"the whole product, {reps} runs" if cols == w.N else
            f"all of A ({w.M}x{w.K}) and the first {cols} of B's {w.N} columns")
    return {"value": useful / dt / 1e12, "unit": "TFLOP/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"float64 oracle coded pipeline (encode, {len(ref_plan.computed)} coded "
                      f"products, peel) on {what}, {dt:.1f} s"}


# -------------------------------------------------------------------- batch --

def run_batch(args):
    import numpy as np
    import torch

    from paper_1904_11563_amd import autotune, bpx, inputs, latency

    tuned = autotune.load()
    if args.tile >= 0:
        bpx.force_tile(args.tile)
    prec_name = args.prec or "bf16x3"
    prec = bpx.PREC_NAMES[prec_name]
    dev = torch.device("cuda:0")
    codes = {4: build_code(bpx, inputs.CODE_642), 8: build_code(bpx, inputs.CODE_1282)}
    shapes = inputs.batch_shapes(args.seed, 256)
    plans, uplans, As, Bs, Cs, Cus = [], [], [], [], [], []
    meta = []
    for i, (M, K, N, k) in enumerate(shapes):
        code = codes[k]
        n = code.info()["n"]
        arrival, _ = inputs.erasure_arrival(args.seed * 1000 + i, n, n - k)
        plans.append(bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, prec))
        uplans.append(bpx.Plan(bpx.Code.identity(k, 2), list(range(k)), 0,
                               bpx.MODE_STRAGGLER, M, K, N, prec))
        g = torch.Generator(device="cpu").manual_seed(args.seed * 1000 + i)
        As.append(torch.randn(M, K, generator=g).to(dev))
        Bs.append(torch.randn(K, N, generator=g).to(dev))
        Cs.append(torch.empty(M, N, device=dev))
        Cus.append(torch.empty(M, N, device=dev))
        meta.append(plans[-1].info())
    ws = torch.empty(bpx.group_workspace_bytes(plans), dtype=torch.uint8, device=dev)
    uws = torch.empty(max(bpx.group_workspace_bytes(uplans), 256), dtype=torch.uint8, device=dev)
    group = bpx.Group(plans, As, Bs, Cs, ws)
    ugroup = bpx.Group(uplans, As, Bs, Cus, uws)

    useful = sum(2.0 * M * K * N for (M, K, N, _) in shapes)

    graph = capture(torch, group.launch)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    value = useful / (ms * 1e-3) / 1e12

    # phase durations (eager, events on the launch stream)
    phase_ms = [timed(torch, lambda p=p: group.launch_phase(p), max(3, args.steps // 3))
                for p in range(3)]
    comp_flops = 0.0
    split_bytes = peel_rd = peel_wr = 0
    planes = 2 if prec_name == "bf16x3" else 1
    for (M, K, N, k), inf, pl in zip(shapes, meta, plans):
        comp_flops += 2.0 * inf["Mb"] * K * N * inf["n_computed"]
        split_bytes += K * N * 4 + N * (-(-K // 32) * 32) * 2 * planes
        r, wb = latency.peel_bytes(pl, M, N)
        peel_rd += r
        peel_wr += wb
    hbm = {"peak_GBps": 8000.0}
    for name, b, t in (("split_b", split_bytes, phase_ms[0]),
                       ("peel", peel_rd + peel_wr, phase_ms[2])):
        hbm[name] = {"bytes": b, "ms": t, "GBps": b / (t * 1e-3) / 1e9,
                     "frac": b / (t * 1e-3) / 1e9 / 8000.0}
    achieved = comp_flops / (phase_ms[1] * 1e-3) / 1e12

    refs = {}
    if not args.no_ref:
        ugraph = capture(torch, ugroup.launch)
        for _ in range(3):
            ugraph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ugraph.replay()
        torch.cuda.synchronize()
        refs["uncoded_own_tflops"] = useful / ((time.perf_counter() - t0) / args.steps) / 1e12
        refs["uncoded_own_prec"] = prec_name
        refs["frac_of_uncoded_own"] = value / refs["uncoded_own_tflops"]

    # error: 8 sampled rows of every product against float64
    num = den = 0.0
    worst = {"product": 0.0, "product_at": -1, "row": 0.0, "row_at": [-1, -1]}
    for i, (M, K, N, k) in enumerate(shapes):
        rows = np.linspace(0, M - 1, 8).astype(int)
        A = As[i][rows].double().cpu().numpy()
        R = A @ Bs[i].double().cpu().numpy()
        Cr = Cs[i][rows].double().cpu().numpy()
        pn, pd = float(np.sum((Cr - R) ** 2)), float(np.sum(R ** 2))
        num += pn
        den += pd
        if np.sqrt(pn / pd) > worst["product"]:
            worst["product"], worst["product_at"] = float(np.sqrt(pn / pd)), i
        rw = np.sqrt(np.sum((Cr - R) ** 2, axis=1) / np.sum(R ** 2, axis=1))
        if rw.max() > worst["row"]:
            worst["row"], worst["row_at"] = float(rw.max()), [i, int(rows[int(rw.argmax())])]
    rel_err = float(np.sqrt(num / den))

    cfg = {"workload": "batch", "products": len(shapes),
           "shapes": "M,K,N log-uniform in [256,4096], multiples of 128",
           "codes": "(6,4,2) for k=4, (12,8,2) for k=8 (searched)", "mode": "arrival",
           "mean_prefix_overhead": float(np.mean([m["n_computed"] * 1.0 /
                                                  (2 * s[3]) for m, s in zip(meta, shapes)])),
           "tile_table": (f"forced {args.tile}" if args.tile >= 0 else
                          f"autotuner table: {tuned}"), "graph": "hipGraph replay",
           "parallelism": "none (1 GPU)"}
    out = header(args, value, ms, prec_name, cfg)
    out.update({"rel_err": rel_err, "rel_err_sample": "8 rows x all columns of every product",
                "rel_err_worst": worst,
                "times_ms": {"split_b": phase_ms[0], "grouped_gemm": phase_ms[1],
                             "peel": phase_ms[2]},
                "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec_name],
                             "unit": "TFLOP/s", "frac": achieved / PEAK[prec_name],
                             "traffic": load_traffic("batch", prec_name, "gemm_bf16.hip"),
                             "kernel": "gemm_bf16_flat_grouped_kernel (GEMM phase)",
                             "flops_per_launch": comp_flops, "launch_ms": phase_ms[1]},
                "hbm": hbm})
    out.update(refs)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_batch(shapes, plans, codes, As, Bs, args)
    return out


def cpu_batch(shapes, plans, codes, As, Bs, args):
    """The oracle on the smallest products of the batch until about
    cpu-seconds of work."""
    from oracle import pipeline
    from oracle.peeling import make_plan
    from paper_1904_11563_amd import inputs
    order = sorted(range(len(shapes)), key=lambda i: shapes[i][0] * shapes[i][1] * shapes[i][2])
    done, flops, t_total = 0, 0.0, 0.0
    for i in order:
        M, K, N, k = shapes[i]
        code = codes[k]
        n = code.info()["n"]
        arrival, _ = inputs.erasure_arrival(args.seed * 1000 + i, n, n - k)
        oc = oracle_code(code)
        rp = make_plan(oc, list(arrival), 0, 1)
        A = As[i].cpu().numpy()
        B = Bs[i].cpu().numpy()
        t0 = time.perf_counter()
        pipeline.coded_matmul_ref(A, B, oc, rp)
        t_total += time.perf_counter() - t0
        flops += 2.0 * M * K * N
        done += 1
        if t_total > args.cpu_seconds:
            break
    return {"value": flops / t_total / 1e12, "unit": "TFLOP/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"float64 oracle coded pipeline on the {done} smallest of the 256 "
                      f"products, {t_total:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read, 1 GiB written per launch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "launches": 3}), flush=True)
        return
    out = run_batch(args) if args.workload == "batch" else run_single(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
