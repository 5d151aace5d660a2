"""GPU parity of the fused form (the peel in the GEMM epilogue, one launch):
integer operands decode to A.B exactly on every erasure pattern, float
results equal the two-launch path (coded GEMM + streaming peel) bit for bit,
and a captured HIP graph replays it exactly."""
import itertools
import sys
from contextlib import contextmanager

import numpy as np
import pytest

from oracle import codes as ocodes
from oracle import pipeline
from oracle.peeling import make_plan
from paper_1904_11563_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1904_11563_amd import bpx  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@contextmanager
def fused_mode(mode):
    bpx.set_fused_peel(mode)
    try:
        yield
    finally:
        bpx.set_fused_peel(1)


def _code642():
    s = inputs.CODE_642
    return bpx.Code.search(s.n, s.k, s.b, s.sigma, s.seed, s.restarts, s.iters, walk=s.walk)


def _code1284():
    s = inputs.CODE_1284
    return bpx.Code.search(s.n, s.k, s.b, s.sigma, s.seed, s.restarts, s.iters, walk=s.walk)


def _oracle(code):
    inf = code.info()
    return ocodes.Code("array", inf["n"], inf["k"], inf["b"], code.columns())


def _run(plan, A, B, mode):
    """Decoded C (numpy) of one product with the given fused-peel mode; C is
    prefilled with NaN so that every row must be written."""
    M, N = A.shape[0], B.shape[1]
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    Cd = torch.full((M, N), float("nan"), device="cuda")
    ws = bpx.alloc_workspace(plan)
    with fused_mode(mode):
        bpx.coded_matmul(plan, Ad, Bd, Cd, ws)
    torch.cuda.synchronize()
    return Cd.cpu().numpy()


@pytest.mark.parametrize("prec", [bpx.PREC_F32, bpx.PREC_BF16, bpx.PREC_BF16X3])
def test_fused_every_erasure_pair_integer_exact(prec):
    # Integer operands in [-8, 8]: every FP32 / BF16 operation is exact, so
    # the fused decode must equal A.B on every decodable pair of erased
    # columns, ragged in every dimension (K a multiple of 4 only).
    code = _code642()
    oc = _oracle(code)
    M, K, N = 517, 260, 300
    A = inputs.integers(1, inputs.TAG_A, (M, K))
    B = inputs.integers(1, inputs.TAG_B, (K, N))
    R = A.astype(np.float64) @ B.astype(np.float64)
    n_ok = 0
    for lost in itertools.combinations(range(6), 2):
        order = [j for j in range(6) if j not in lost] + list(lost)
        plan = bpx.Plan(code, order, 2, bpx.MODE_ERASURE, M, K, N, prec)
        if not plan.decodable:
            assert not make_plan(oc, order, 2, 0).decodable
            continue
        _say("fused erasure pattern", lost, "prec", prec)
        C = _run(plan, A, B, 2)
        assert np.array_equal(C.astype(np.float64), R), (lost, prec)
        n_ok += 1
    assert n_ok >= 10


@pytest.mark.parametrize("prec", [bpx.PREC_F32, bpx.PREC_BF16, bpx.PREC_BF16X3])
def test_fused_equals_two_launch_float(prec):
    # Same products, same k order, same member order, same peel program
    # arithmetic: the fused result equals the two-launch result bit for bit.
    # Cases: the 512^3 workload's code and arrival, Table III's depth-9
    # chain (FP64 accumulation past depth 4), the (12,8,4) code in FULL
    # mode (non-releasers computed and dropped), ragged shapes.
    cases = []
    arrival, lost = inputs.erasure_arrival(0, 6, 2)
    cases.append((_code642(), list(arrival), lost, bpx.MODE_ERASURE, 512, 512, 512))
    cases.append((bpx.Code.table3(), [0, 1, 2, 3, 4], 2, bpx.MODE_ERASURE, 9 * 40 - 3, 256, 136))
    cases.append((_code1284(), list(range(12)), 0, bpx.MODE_FULL, 32 * 20 + 5, 196, 260))
    for ci, (code, order, nl, mode, M, K, N) in enumerate(cases):
        plan = bpx.Plan(code, order, nl, mode, M, K, N, prec)
        assert plan.decodable
        A = inputs.normal(30 + ci, inputs.TAG_A, (M, K))
        B = inputs.normal(30 + ci, inputs.TAG_B, (K, N))
        C2 = _run(plan, A, B, 0)
        Cf = _run(plan, A, B, 2)
        _say("fused vs two-launch case", ci, "prec", prec, "depth", plan.info()["depth_max"],
             "max |diff|", float(np.nanmax(np.abs(Cf - C2))))
        assert not np.isnan(Cf).any()
        assert np.array_equal(Cf, C2), (ci, prec)


def test_fused_small_workloads_meet_targets():
    # The 512^3 FP32 workload and the row-scaled BF16x3 workload through the
    # default mode (which takes the fused form at this size).
    for name, tol in (("fp32_small", 1e-5), ("bf16_small", 1e-5)):
        w = inputs.WORKLOADS[name]
        A, B = inputs.operands(w, seed=0)
        arrival, lost, _ = inputs.arrival_of(w, seed=0)
        prec = bpx.PREC_NAMES[w.prec]
        plan = bpx.Plan(_code642(), arrival, lost, bpx.MODE_ERASURE, w.M, w.K, w.N, prec)
        C = _run(plan, A, B, 1)
        e = pipeline.rel_frobenius(C, pipeline.uncoded(A, B))
        _say(name, "fused relF", e)
        assert e <= tol


def test_fused_graph_replay_matches_eager():
    # The fused launch captured in a HIP graph, replayed three times with
    # eager work in between; every replay equals the eager result.
    code = _code642()
    arrival, lost = inputs.erasure_arrival(0, 6, 2)
    M = K = N = 512
    plan = bpx.Plan(code, list(arrival), lost, bpx.MODE_ERASURE, M, K, N)
    plan.upload()
    A = torch.from_numpy(inputs.normal(5, inputs.TAG_A, (M, K))).cuda()
    B = torch.from_numpy(inputs.normal(5, inputs.TAG_B, (K, N))).cuda()
    ws = bpx.alloc_workspace(plan)
    C_eager = torch.empty((M, N), device="cuda")
    with fused_mode(2):
        bpx.coded_matmul(plan, A, B, C_eager, ws)
        torch.cuda.synchronize()
        C = torch.full((M, N), float("nan"), device="cuda")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                bpx.coded_matmul(plan, A, B, C, ws)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
    for rep in range(3):
        C.fill_(float("nan"))
        torch.matmul(A, B)                      # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, C_eager), rep
