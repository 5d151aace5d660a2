"""GPU parity: the HIP path through the C ABI against the oracle.

Integer-valued operands in [-8, 8] make every FP32 operation of the HIP
path exact (all partial sums stay far below 2^24), so for them the decoded
product must equal A.B bit for bit.  Float operands are held to the FP32
bound: relative Frobenius error <= 1e-5 against the float64 oracle.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle import codes as ocodes
from oracle import pipeline
from oracle.peeling import make_plan
from paper_1904_11563_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1904_11563_amd import bpx  # noqa: E402  (fails loudly if the library is missing)

TOL_F32 = 1e-5


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def lib_code(spec):
    if spec.kind == "search":
        return bpx.Code.search(spec.n, spec.k, spec.b, spec.sigma, spec.seed, spec.restarts,
                               spec.iters, walk=spec.walk)
    if spec.kind == "mojette":
        return bpx.Code.mojette(spec.k, spec.b, spec.n, spec.qe)
    raise ValueError(spec.kind)


def oracle_of(code):
    inf = code.info()
    return ocodes.Code("array", inf["n"], inf["k"], inf["b"], code.columns())


def padded(x):
    """Device copy of a 2-D array whose row stride is rounded up to 4 floats
    (the ABI's alignment rule), returned as the unpadded view."""
    r, c = x.shape
    ld = -(-c // 4) * 4
    t = torch.zeros((r, ld), dtype=torch.float32, device="cuda")
    t[:, :c] = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t[:, :c]


def run(plan, A, B, ldc_pad=0):
    M, N = A.shape[0], B.shape[1]
    Ad, Bd = padded(A), padded(B)
    ldc = -(-N // 4) * 4 + ldc_pad
    Cfull = torch.full((M, ldc), float("nan"), device="cuda")
    Cd = Cfull[:, :N]
    ws = bpx.alloc_workspace(plan)
    bpx.coded_matmul(plan, Ad, Bd, Cd, ws)
    return host(Cd)


def relf(X, R):
    return pipeline.rel_frobenius(X, R)


def worst_errors(C, R, rows, Mb):
    """Worst relative error of a sampled row and of a data block's sampled
    rows: the Frobenius norm of the whole sample hides rows or blocks whose
    error grew along a release chain or through cancellation."""
    num = np.sum((C.astype(np.float64) - R) ** 2, axis=1)
    den = np.sum(R ** 2, axis=1)
    per_row = np.sqrt(num / np.maximum(den, 1e-300))
    blocks = np.asarray(rows) // Mb
    per_block = {}
    for b in np.unique(blocks):
        m = blocks == b
        per_block[int(b)] = float(np.sqrt(num[m].sum() / max(den[m].sum(), 1e-300)))
    wb = max(per_block, key=per_block.get)
    return {"row": float(per_row.max()), "row_at": int(rows[int(per_row.argmax())]),
            "block": per_block[wb], "block_at": wb, "per_block": per_block}


CODE_642 = None


def code642():
    global CODE_642
    if CODE_642 is None:
        CODE_642 = lib_code(inputs.CODE_642)
    return CODE_642


# ------------------------------------------------------------- small, exact --

def test_every_erasure_pair_small_code_integer_exact():
    # the two-launch path (coded GEMM + streaming peel); the fused form has
    # its own tests
    bpx.set_fused_peel(0)
    try:
        _every_erasure_pair_small_code_integer_exact()
    finally:
        bpx.set_fused_peel(1)


def _every_erasure_pair_small_code_integer_exact():
    code = code642()
    oc = oracle_of(code)
    M, K, N = 517, 260, 300            # ragged in every dimension
    A = inputs.integers(1, inputs.TAG_A, (M, K))
    B = inputs.integers(1, inputs.TAG_B, (K, N))
    R = A.astype(np.float64) @ B.astype(np.float64)
    n_ok = n_bad = 0
    for lost in itertools.combinations(range(6), 2):
        order = [j for j in range(6) if j not in lost] + list(lost)
        _say("erasure pattern", lost)
        plan = bpx.Plan(code, order, 2, bpx.MODE_ERASURE, M, K, N)
        want = make_plan(oc, order, 2, 0)
        assert plan.decodable == want.decodable
        if not plan.decodable:
            n_bad += 1
            Cd = torch.full((M, N), float("nan"), device="cuda")
            ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
            with pytest.raises(bpx.BpxError) as e:
                bpx.coded_matmul(plan, dev(A), dev(B), Cd, ws)
            assert e.value.status == bpx.E_UNDECODABLE
            assert torch.isnan(Cd).all().item()       # nothing written
            continue
        n_ok += 1
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), R), lost
    assert n_ok > 0 and n_bad >= 1     # (6,4,2) cannot be column-MDS


def test_peel_register_and_lds_slots_integer_exact():
    # The single-product peel keeps a program's live slots in registers when
    # it needs at most 12 and in LDS otherwise.  The (12,8,4) code's
    # straggler plans (seeds 0-5: 10-12 slots, release depth up to 14, FP64
    # accumulation) and its FULL plan (13 slots), two-launch path, integer
    # operands (every FP32 and FP64 operation exact), M ragged with an empty
    # padding block: C must equal A.B.
    bpx.set_fused_peel(0)
    try:
        code = lib_code(inputs.CODE_1284)
        M, K, N = 32 * 20 + 5, 64, 260
        A = inputs.integers(9, inputs.TAG_A, (M, K))
        B = inputs.integers(9, inputs.TAG_B, (K, N))
        R = A.astype(np.float64) @ B.astype(np.float64)
        cases = []
        for seed in range(6):
            arrival, lost, _ = inputs.arrival_of(inputs.WORKLOADS["fp32_scale"], seed=seed)
            cases.append((list(arrival), lost, bpx.MODE_STRAGGLER))
        cases.append((list(range(12)), 0, bpx.MODE_FULL))
        seen = set()
        for order, lost, mode in cases:
            plan = bpx.Plan(code, order, lost, mode, M, K, N)
            assert plan.decodable
            slots = plan.peel_program()["n_slots"]
            seen.add(slots)
            _say("peel slots", slots, "mode", mode, "depth", plan.info()["depth_max"])
            C = run(plan, A, B)
            assert np.array_equal(C.astype(np.float64), R), (slots, mode)
        assert 12 in seen and 13 in seen     # both sides of the register limit
    finally:
        bpx.set_fused_peel(1)


def test_small_workload_float_tolerance():
    w = inputs.WORKLOADS["fp32_small"]
    A, B = inputs.operands(w, seed=0)
    arrival, lost, _ = inputs.arrival_of(w, seed=0)
    code = code642()
    plan = bpx.Plan(code, arrival, lost, bpx.MODE_STRAGGLER, w.M, w.K, w.N)
    C = run(plan, A, B)
    want = make_plan(oracle_of(code), list(arrival), lost, 1)
    C_ref = pipeline.coded_matmul_ref(A, B, oracle_of(code), want)
    R = pipeline.uncoded(A, B)
    assert relf(C_ref, R) < 1e-12
    e = relf(C, R)
    _say("fp32_small relF", e)
    assert e <= TOL_F32


def test_coded_gemm_products_and_aliases():
    code = code642()
    oc = oracle_of(code)
    M, K, N = 300, 132, 200
    A = inputs.integers(2, inputs.TAG_A, (M, K))
    B = inputs.integers(2, inputs.TAG_B, (K, N))
    order = [5, 3, 0, 1, 2, 4]
    plan = bpx.Plan(code, order, 0, bpx.MODE_FULL, M, K, N)
    sch = plan.schedule()
    want = make_plan(oc, order, 0, 2)
    Y_ref = pipeline.coded_products(pipeline.encode(A, oc, want.computed), B)
    Ad, Bd = dev(A), dev(B)
    Cd = torch.zeros((M, N), device="cuda")
    ws = bpx.alloc_workspace(plan)
    bpx.coded_gemm(plan, Ad, Bd, Cd, ws)
    Mb = plan.info()["Mb"]
    Y = host(ws).view(np.float32)
    C = host(Cd)
    for g, d in zip(sch["computed"].tolist(), sch["dest"].tolist()):
        if d >= 0:
            got = Y[d * Mb * N:(d + 1) * Mb * N].reshape(Mb, N)
            assert np.array_equal(got.astype(np.float64), Y_ref[g]), g
        else:
            s = -1 - d
            rows = min(Mb, M - s * Mb)
            assert np.array_equal(C[s * Mb:s * Mb + rows].astype(np.float64), Y_ref[g][:rows])


def test_encode_matches_oracle():
    code = code642()
    oc = oracle_of(code)
    M, K = 250, 96
    A = inputs.integers(3, inputs.TAG_A, (M, K))
    plan = bpx.Plan(code, [0, 1, 2, 3, 4, 5], 0, bpx.MODE_FULL, M, K, 8)
    _, enc_bytes = plan.workspace_bytes()
    out = torch.empty(enc_bytes // 4, dtype=torch.float32, device="cuda")
    bpx.encode(plan, dev(A), out)
    got = host(out)
    Mb = plan.info()["Mb"]
    want = pipeline.encode(A, oc, plan.schedule()["computed"].tolist())
    for i, g in enumerate(plan.schedule()["computed"].tolist()):
        assert np.array_equal(got[i * Mb * K:(i + 1) * Mb * K].reshape(Mb, K), want[g])
    # float operands: fp32 sum against the float64 sum
    Af = inputs.normal(3, inputs.TAG_A, (M, K))
    bpx.encode(plan, dev(Af), out)
    got = host(out)
    want = pipeline.encode(Af, oc, plan.schedule()["computed"].tolist())
    for i, g in enumerate(plan.schedule()["computed"].tolist()):
        blk = got[i * Mb * K:(i + 1) * Mb * K].reshape(Mb, K)
        assert np.abs(blk - want[g]).max() <= 4 * np.finfo(np.float32).eps * (np.abs(want[g]).max() + 1)


def test_table3_depth_nine_chain_fp64_path():
    code = bpx.Code.table3()
    M, K, N = 9 * 33 + 4, 64, 130
    order = [0, 1, 2, 3, 4]
    plan = bpx.Plan(code, order, 2, bpx.MODE_ERASURE, M, K, N)
    assert plan.info()["depth_max"] == 9
    A = inputs.integers(4, inputs.TAG_A, (M, K))
    B = inputs.integers(4, inputs.TAG_B, (K, N))
    C = run(plan, A, B)
    assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B)
    Af = inputs.normal(4, inputs.TAG_A, (M, K))
    Bf = inputs.normal(4, inputs.TAG_B, (K, N))
    C = run(plan, Af, Bf)
    assert relf(C, pipeline.uncoded(Af, Bf)) <= TOL_F32


@pytest.mark.parametrize("mode", [bpx.MODE_STRAGGLER, bpx.MODE_FULL, bpx.MODE_MIN])
def test_modes_table1(mode):
    code = bpx.Code.table1()
    M, K, N = 64, 36, 70
    A = inputs.integers(5, inputs.TAG_A, (M, K))
    B = inputs.integers(5, inputs.TAG_B, (K, N))
    for order in itertools.permutations(range(5)):
        plan = bpx.Plan(code, order, 0, mode, M, K, N)
        C = run(plan, A, B, ldc_pad=4)
        assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B), order


def test_mojette_codes_integer_exact():
    for (k, b, n, qe) in [(4, 3, 7, 0), (4, 3, 6, 1), (16, 8, 24, 0), (16, 16, 24, 0)]:
        code = bpx.Code.mojette(k, b, n, qe)
        kb = k * b
        M, K, N = kb * 5 + 3, 68, 90
        A = inputs.integers(6, inputs.TAG_A, (M, K))
        B = inputs.integers(6, inputs.TAG_B, (K, N))
        arrival = inputs.rng(k * 100 + b, 9).permutation(n).astype(np.int32)
        lost = n // 3
        _say("mojette", k, b, n, qe)
        plan = bpx.Plan(code, arrival, lost, bpx.MODE_ERASURE, M, K, N)
        if not plan.decodable:
            continue
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B), (k, b, n, qe)


def test_construction_b_codes_exact_and_full_size_sampled():
    """Mojette Construction B (q_i = 2^qe, odd p_i): integer operands decode
    exactly for several erasure patterns at q_e = 1 and 2, and the
    8192x8192 . 8192x4096 FP32 workload (k=8, b=4, n=12, q_e=1, 4 columns
    erased) meets the FP32 bound on sampled rows."""
    for qe in (1, 2):
        code = bpx.Code.mojette(8, 4, 12, qe)
        M, K, N = 32 * 9 + 5, 96, 100
        A = inputs.integers(40 + qe, inputs.TAG_A, (M, K))
        B = inputs.integers(40 + qe, inputs.TAG_B, (K, N))
        R = A.astype(np.float64) @ B.astype(np.float64)
        for seed in range(4):
            arrival, lost = inputs.erasure_arrival(seed, 12, 4)
            plan = bpx.Plan(code, arrival, lost, bpx.MODE_ERASURE, M, K, N)
            _say("construction B", qe, seed, plan.info())
            assert plan.decodable
            assert np.array_equal(run(plan, A, B).astype(np.float64), R), (qe, seed)
    w = inputs.WORKLOADS["mojette_b"]
    A, B = inputs.operands(w, seed=0)
    arrival, lost, _ = inputs.arrival_of(w, seed=0)
    plan = bpx.Plan(lib_code(w.code), arrival, lost, bpx.MODE_ERASURE, w.M, w.K, w.N)
    _say("mojette_b plan", plan.info())
    C = run(plan, A, B)
    rows = np.concatenate([np.arange(s * 256, s * 256 + 256, 37)[:4] for s in range(32)])
    e = relf(C[rows], A[rows].astype(np.float64) @ B.astype(np.float64))
    _say("mojette_b sampled relF", e)
    assert e <= TOL_F32


def test_two_dimensional_form_exact_and_products():
    """The two-dimensional form (A by rows, B by columns, symbols of block
    products): integer operands decode exactly for every erasure pattern of
    Tables I and III that peels (ragged M, K not a multiple of 32, Nb not a
    multiple of the tile), and every coded product, gray symbols included,
    equals the oracle's (sum of its members' block products)."""
    from oracle import pipeline2d
    for lib, oc, M, K, N in ((bpx.Code.table1(), ocodes.table1(), 37, 68, 200),
                             (bpx.Code.table3(), ocodes.table3(), 50, 100, 264)):
        A = inputs.integers(50, inputs.TAG_A, (M, K))
        B = inputs.integers(50, inputs.TAG_B, (K, N))
        R = A.astype(np.float64) @ B.astype(np.float64)
        n_ok = 0
        for lost in itertools.combinations(range(5), 2):
            order = [j for j in range(5) if j not in lost] + list(lost)
            plan = bpx.Plan(lib, order, 2, bpx.MODE_ERASURE, M, K, N, two_d=True)
            if not plan.decodable:
                continue
            _say("2-D", lib.info()["k"], lost)
            assert np.array_equal(run(plan, A, B).astype(np.float64), R), lost
            n_ok += 1
        assert n_ok >= 1
        # every symbol's product, FULL mode
        plan = bpx.Plan(lib, [0, 1, 2, 3, 4], 0, bpx.MODE_FULL, M, K, N, two_d=True)
        grid, Nb = plan.grid()
        Mb = plan.info()["Mb"]
        sch = plan.schedule()
        Cd = torch.zeros((M, N), device="cuda")
        ws = bpx.alloc_workspace(plan)
        bpx.coded_gemm(plan, dev(A), dev(B), Cd, ws)
        Y = host(ws).view(np.float32)
        C = host(Cd)
        want = pipeline2d.coded_products(A, B, oc, sch["computed"].tolist())
        sym = {g: d for g, _, d in oc.symbols()}
        for g, d in zip(sch["computed"].tolist(), sch["dest"].tolist()):
            if d >= 0:
                got = Y[d * Mb * Nb:(d + 1) * Mb * Nb].reshape(Mb, Nb).astype(np.float64)
                assert np.array_equal(got, want[g]), (g, pipeline2d.kind(sym[g], grid))
            else:
                r, c = divmod(-1 - d, grid)
                rows = min(Mb, M - r * Mb)
                got = C[r * Mb:r * Mb + rows, c * Nb:(c + 1) * Nb].astype(np.float64)
                assert np.array_equal(got, want[g][:rows]), g


def test_two_dimensional_wide_tiles_exact_and_products():
    """The two-dimensional form on full 256-multiple blocks, which run on the
    256 x 256 tiling: the (12,8,2) searched code over its 4 x 4 grid (gray
    symbols, symbols sharing an A block and symbols sharing a B block all
    present), one and four tiles per product.  Every coded product equals
    the oracle's exactly on integer operands, straggler arrivals decode to
    A.B exactly, and float operands stay within the FP32 bound."""
    from oracle import pipeline2d
    code = lib_code(inputs.CODE_1282)
    oc = oracle_of(code)
    sym = {g: d for g, _, d in oc.symbols()}
    for M, K, N in ((1024, 96, 1024), (2048, 96, 2048)):
        A = inputs.integers(52, inputs.TAG_A, (M, K))
        B = inputs.integers(52, inputs.TAG_B, (K, N))
        plan = bpx.Plan(code, list(range(12)), 0, bpx.MODE_FULL, M, K, N, two_d=True)
        grid, Nb = plan.grid()
        Mb = plan.info()["Mb"]
        assert Mb % 256 == 0 and Nb % 256 == 0 and grid * Mb == M and grid * Nb == N
        sch = plan.schedule()
        kinds = {pipeline2d.kind(sym[g], grid) for g in sch["computed"].tolist()}
        assert {"a", "b", "gray"} <= kinds
        _say("2-D wide products", M, K, N)
        Cd = torch.zeros((M, N), device="cuda")
        ws = bpx.alloc_workspace(plan)
        bpx.coded_gemm(plan, dev(A), dev(B), Cd, ws)
        Y = host(ws).view(np.float32)
        C = host(Cd)
        want = pipeline2d.coded_products(A, B, oc, sch["computed"].tolist())
        for g, d in zip(sch["computed"].tolist(), sch["dest"].tolist()):
            if d >= 0:
                got = Y[d * Mb * Nb:(d + 1) * Mb * Nb].reshape(Mb, Nb).astype(np.float64)
            else:
                r, c = divmod(-1 - d, grid)
                got = C[r * Mb:(r + 1) * Mb, c * Nb:(c + 1) * Nb].astype(np.float64)
            assert np.array_equal(got, want[g]), (g, pipeline2d.kind(sym[g], grid))
        R = A.astype(np.float64) @ B.astype(np.float64)
        Af = inputs.normal(53, inputs.TAG_A, (M, K))
        Bf = inputs.normal(53, inputs.TAG_B, (K, N))
        for seed in range(2):
            arrival, _ = inputs.shifted_exp_arrival(seed, 12)
            sp = bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, two_d=True)
            _say("2-D wide straggler", M, seed)
            assert np.array_equal(run(sp, A, B).astype(np.float64), R), seed
            Cw = run(sp, Af, Bf)
            assert relf(Cw, pipeline.uncoded(Af, Bf)) <= TOL_F32
            try:  # the 64 x 128 tiling sums every product in the same order
                bpx.force_tile(1)
                C1 = run(sp, Af, Bf)
            finally:
                bpx.force_tile(-1)
            assert np.array_equal(Cw, C1), seed


def test_two_dimensional_form_float_tolerance():
    """The (12,8,2) searched code in the two-dimensional form (4 x 4 block
    grid, gray symbols present) on float operands: relative Frobenius error
    against float64 within the FP32 bound, straggler arrivals."""
    from oracle import pipeline2d
    code = lib_code(inputs.CODE_1282)
    oc = oracle_of(code)
    assert pipeline2d.gray_ratio(oc) > 0
    M, K, N = 1000, 520, 1024
    A = inputs.normal(51, inputs.TAG_A, (M, K))
    B = inputs.normal(51, inputs.TAG_B, (K, N))
    R = pipeline.uncoded(A, B)
    for seed in range(3):
        arrival, _ = inputs.shifted_exp_arrival(seed, 12)
        plan = bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, two_d=True)
        e = relf(run(plan, A, B), R)
        _say("2-D float", seed, plan.info(), e)
        assert e <= TOL_F32


def test_identity_code_is_plain_gemm():
    code = bpx.Code.identity(4, 2)
    M, K, N = 203, 100, 77
    A = inputs.normal(7, inputs.TAG_A, (M, K))
    B = inputs.normal(7, inputs.TAG_B, (K, N))
    plan = bpx.Plan(code, list(range(4)), 0, bpx.MODE_STRAGGLER, M, K, N)
    assert plan.workspace_bytes()[0] == 0       # every product lands in C
    C = run(plan, A, B)
    assert relf(C, pipeline.uncoded(A, B)) <= TOL_F32


def test_padding_blocks_without_rows():
    # M = 5 with k*b = 4: Mb = 2 and block 3 has no rows at all.
    code = bpx.Code.table1()
    M, K, N = 5, 8, 6
    A = inputs.integers(8, inputs.TAG_A, (M, K))
    B = inputs.integers(8, inputs.TAG_B, (K, N))
    for order in itertools.permutations(range(5)):
        plan = bpx.Plan(code, order, 3, bpx.MODE_ERASURE, M, K, N)
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B)


@pytest.mark.parametrize("prec", [bpx.PREC_F32, bpx.PREC_BF16, bpx.PREC_BF16X3])
def test_smallest_products_exact(prec):
    """The degenerate end of the method: a single output row (M = 1, so one
    data block holds the row and every other block is empty), K = 4 (the
    smallest K the device path takes) and N = 1 and 5, through both forms,
    on every decodable two-column arrival of Table I and on the (6,4,2)
    code; integer operands, so each result is exact."""
    cases = [(bpx.Code.table1(), 5, 3), (code642(), 6, 2)]
    for code, n, lost in cases:
        for N in (1, 5):
            A = inputs.integers(40 + N, inputs.TAG_A, (1, 4))
            B = inputs.integers(40 + N, inputs.TAG_B, (4, N))
            R = A.astype(np.float64) @ B.astype(np.float64)
            n_ok = 0
            for kept in itertools.combinations(range(n), n - lost):
                order = list(kept) + [j for j in range(n) if j not in kept]
                plan = bpx.Plan(code, order, lost, bpx.MODE_ERASURE, 1, 4, N, prec)
                if not plan.decodable:
                    continue
                for mode in (0, 2):     # two-launch form, fused form
                    bpx.set_fused_peel(mode)
                    try:
                        _say("smallest product", n, N, kept, "prec", prec, "fused", mode)
                        C = run(plan, A, B)
                    finally:
                        bpx.set_fused_peel(1)
                    assert np.array_equal(C.astype(np.float64), R), (n, N, kept, mode)
                n_ok += 1
            assert n_ok >= 1


def test_argument_errors():
    code = bpx.Code.table1()
    plan = bpx.Plan(code, [0, 1, 2, 3, 4], 0, bpx.MODE_STRAGGLER, 16, 6, 8)
    A = torch.zeros((16, 6), device="cuda")
    B = torch.zeros((6, 8), device="cuda")
    C = torch.zeros((16, 8), device="cuda")
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(bpx.BpxError) as e:       # K not a multiple of 4
        bpx.coded_matmul(plan, A, B, C, ws)
    assert e.value.status == bpx.E_INVALID
    plan = bpx.Plan(code, [0, 1, 2, 3, 4], 0, bpx.MODE_FULL, 16, 8, 8)
    A = torch.zeros((16, 8), device="cuda")
    B = torch.zeros((8, 8), device="cuda")
    if plan.workspace_bytes()[0] > 0:
        with pytest.raises(bpx.BpxError):        # workspace too small
            bpx.coded_matmul(plan, A, B, C, torch.empty(4, dtype=torch.uint8, device="cuda"))
    flat = torch.zeros(16 * 8 + 1, device="cuda")
    Cmis = flat[1:].view(16, 8)
    with pytest.raises(bpx.BpxError):            # misaligned C
        bpx.coded_matmul(plan, A, B, Cmis, ws)
    # the binding checks every operand against the plan before the call
    with pytest.raises(ValueError):              # shape differs from the plan's
        bpx.coded_matmul(plan, A[:, :4].contiguous(), B[:4].contiguous(), C, ws)
    with pytest.raises(ValueError):              # wrong dtype
        bpx.coded_matmul(plan, A.double(), B, C, ws)
    with pytest.raises(ValueError):              # host tensor
        bpx.coded_matmul(plan, A.cpu(), B, C, ws)
    with pytest.raises(ValueError):              # transposed view: not unit column stride
        bpx.coded_matmul(plan, A, B.t().contiguous().t(), C, ws)
    g_plan = bpx.Plan(code, [0, 1, 2, 3, 4], 0, bpx.MODE_STRAGGLER, 16, 8, 8, bpx.PREC_BF16X3)
    gws = torch.empty(bpx.group_workspace_bytes([g_plan]), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):              # grouped operands must be dense
        bpx.Group([g_plan], [A], [B.t().contiguous().t()], [C], gws)
    with pytest.raises(ValueError):
        bpx.Group([g_plan], [A], [B], [C.double()], gws)


# ----------------------------------------------------------- full size, f32 --

def test_fp32_scale_full_size_sampled():
    """8192x8192 . 8192x4096, (12,8,4) searched code, shifted-exponential
    arrivals: the bench's configuration.  Checked on 256 sampled rows (8 per
    data block) against float64, plus the Frobenius bound on the sample."""
    w = inputs.WORKLOADS["fp32_scale"]
    A, B = inputs.operands(w, seed=0)
    arrival, lost, _ = inputs.arrival_of(w, seed=0)
    code = lib_code(w.code)
    plan = bpx.Plan(code, arrival, lost, bpx.MODE_STRAGGLER, w.M, w.K, w.N)
    _say("fp32_scale plan", plan.info())
    C = run(plan, A, B)
    rows = np.concatenate([np.arange(s * 256, s * 256 + 256, 37)[:8] for s in range(32)])
    R = A[rows].astype(np.float64) @ B.astype(np.float64)
    e = relf(C[rows], R)
    worst = worst_errors(C[rows], R, rows, 256)
    depth = plan.schedule()["depth"]
    _say("fp32_scale sampled relF", e, "worst row", worst["row"], "at", worst["row_at"],
         "worst block", worst["block"], "at", worst["block_at"],
         "depth", int(depth[worst["block_at"]]))
    assert e <= TOL_F32
    # every block within the FP32 target (N(0,1) rows have similar norms,
    # so no row cancels)
    assert worst["block"] <= TOL_F32 and worst["row"] <= 2 * TOL_F32
    assert np.isfinite(C).all()


def test_fp32_2d_full_size_sampled():
    """The two-dimensional workload at the bench's size and launch (8192^3,
    (12,8,2) code over the 4 x 4 block grid, shifted-exponential arrivals,
    256 x 256 tiles dealt by decreasing passes): 16 sampled rows (4 per row
    block) against float64 within the FP32 bound, everything finite."""
    w = inputs.WORKLOADS["fp32_2d"]
    A, B = inputs.operands(w, seed=0)
    arrival, lost, _ = inputs.arrival_of(w, seed=0)
    code = lib_code(w.code)
    plan = bpx.Plan(code, arrival, lost, bpx.MODE_STRAGGLER, w.M, w.K, w.N, two_d=True)
    _say("fp32_2d plan", plan.info())
    C = run(plan, A, B)
    Mb = plan.info()["Mb"]
    rows = np.concatenate([np.arange(r * Mb + 5, (r + 1) * Mb, Mb // 4)[:4] for r in range(4)])
    R = A[rows].astype(np.float64) @ B.astype(np.float64)
    e = relf(C[rows], R)
    _say("fp32_2d sampled relF", e)
    assert e <= TOL_F32
    assert np.isfinite(C).all()


def test_wide_tile_split_k_last_round():
    """The 256 x 256 FP32 tiling on a shape with one full round and a short
    last round (12 symbols x 24 column tiles = 288 tiles; K = 1024 gives the
    last 32 tiles four 8-slice pieces each, reduced in piece order): integer
    operands decode exactly, float operands agree with the 64 x 128 tiling to
    the FP32 summation-order level, and two runs are bit-identical."""
    code = code642()
    M, K, N = 2048, 1024, 6144
    plan = bpx.Plan(code, list(range(6)), 0, bpx.MODE_FULL, M, K, N)
    A = inputs.integers(8, inputs.TAG_A, (M, K))
    B = inputs.integers(8, inputs.TAG_B, (K, N))
    Af = inputs.normal(8, inputs.TAG_A, (M, K))
    Bf = inputs.normal(8, inputs.TAG_B, (K, N))
    try:
        bpx.force_tile(6)
        _say("wide split-K integer")
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))
        Cw = run(plan, Af, Bf)
        Cw2 = run(plan, Af, Bf)
        bpx.force_tile(1)
        C1 = run(plan, Af, Bf)
    finally:
        bpx.force_tile(-1)
    assert np.array_equal(Cw, Cw2)
    assert relf(Cw, C1) <= 1e-6
    assert relf(Cw, Af.astype(np.float64) @ Bf.astype(np.float64)) <= TOL_F32


def test_wide_tile_split_k_chunked_last_round():
    """A last round of more than half the CUs: 12 symbols x 37 column tiles
    = 444 tiles, so on a 256-CU MI355X one full round and 188 tiles split
    four ways (three rounds of quarter pieces), run in chunks of 64 tiles
    that fit the 256-tile partial buffer (the last chunk ragged), each chunk
    reduced in piece order.  Integer operands decode exactly, floats agree
    with the 64 x 128 tiling to the FP32 summation-order level, and two runs
    are bit-identical."""
    code = code642()
    M, K, N = 2048, 1024, 37 * 256
    plan = bpx.Plan(code, list(range(6)), 0, bpx.MODE_FULL, M, K, N)
    A = inputs.integers(9, inputs.TAG_A, (M, K))
    B = inputs.integers(9, inputs.TAG_B, (K, N))
    Af = inputs.normal(9, inputs.TAG_A, (M, K))
    Bf = inputs.normal(9, inputs.TAG_B, (K, N))
    try:
        bpx.force_tile(6)
        _say("wide chunked split-K integer")
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))
        Cw = run(plan, Af, Bf)
        Cw2 = run(plan, Af, Bf)
        bpx.force_tile(1)
        C1 = run(plan, Af, Bf)
    finally:
        bpx.force_tile(-1)
    assert np.array_equal(Cw, Cw2)
    assert relf(Cw, C1) <= 1e-6
    assert relf(Cw, Af.astype(np.float64) @ Bf.astype(np.float64)) <= TOL_F32


def test_wide_tile_exact_and_identical_to_small_tile():
    """The 256 x 256 FP32 tiles (three wave layouts) on a shape that fills
    more than one round of the CUs, whose last round (K = 96: too few
    slices to split) runs as 64 x 128 sub-tiles of the wide tiling: integer
    operands decode to A.B exactly, and float operands give bit-identical
    results to the 64 x 128 tile (both sum in the same order)."""
    code = code642()
    M, K, N = 2048, 96, 6144           # Mb = 256; 12 symbols x 24 column tiles
    arrival = list(range(6))
    plan = bpx.Plan(code, arrival, 0, bpx.MODE_FULL, M, K, N)
    assert plan.info()["Mb"] == 256 and plan.info()["n_computed"] == 12
    A = inputs.integers(7, inputs.TAG_A, (M, K))
    B = inputs.integers(7, inputs.TAG_B, (K, N))
    R = A.astype(np.float64) @ B.astype(np.float64)
    Af = inputs.normal(7, inputs.TAG_A, (M, K))
    Bf = inputs.normal(7, inputs.TAG_B, (K, N))
    try:
        for tile in (4, 5, 6):
            _say("wide tile", tile, "integer")
            bpx.force_tile(tile)
            C = run(plan, A, B)
            assert np.array_equal(C.astype(np.float64), R), tile
        bpx.force_tile(1)
        C1 = run(plan, Af, Bf)
        for tile in (4, 5, 6):
            _say("wide tile", tile, "float vs 64x128")
            bpx.force_tile(tile)
            Cw = run(plan, Af, Bf)
            assert np.array_equal(Cw, C1), tile
    finally:
        bpx.force_tile(-1)
    assert relf(C1, Af.astype(np.float64) @ Bf.astype(np.float64)) <= TOL_F32


# ------------------------------------------------------------ BF16 paths --

TOL_BF16X3 = 1e-5


@pytest.mark.parametrize("prec", [bpx.PREC_BF16, bpx.PREC_BF16X3])
def test_bf16_integer_operands_exact(prec):
    # integers in [-8, 8] and their coded sums are exact in bf16 (lo = 0),
    # products and FP32 accumulation are exact: the decode is bit exact.
    code = code642()
    M, K, N = 517, 260, 300
    A = inputs.integers(11, inputs.TAG_A, (M, K))
    B = inputs.integers(11, inputs.TAG_B, (K, N))
    R = A.astype(np.float64) @ B.astype(np.float64)
    for lost in [(0, 1), (2, 5), (3, 4)]:
        order = [j for j in range(6) if j not in lost] + list(lost)
        plan = bpx.Plan(code, order, 2, bpx.MODE_ERASURE, M, K, N, prec)
        if not plan.decodable:
            continue
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), R), (prec, lost)


@pytest.mark.parametrize("prec", [bpx.PREC_BF16, bpx.PREC_BF16X3])
def test_bf16_flat_tile_exact_and_identical_to_per_symbol_tile(prec):
    """The flat-row BF16 tiling (128x256 tiles over the stacked rows of all
    symbols, tiles crossing symbol boundaries) on a ragged shape: integer
    operands decode exactly; float operands give the same bits as the
    per-symbol 64x128 tiling (same k order and same MFMA order per
    output)."""
    code = code642()
    M, K, N = 517, 256, 300          # Mb = 65: tiles straddle symbols
    order = [5, 3, 0, 1, 2, 4]
    plan = bpx.Plan(code, order, 0, bpx.MODE_STRAGGLER, M, K, N, prec)
    A = inputs.integers(31, inputs.TAG_A, (M, K))
    B = inputs.integers(31, inputs.TAG_B, (K, N))
    Af = inputs.normal(31, inputs.TAG_A, (M, K))
    Bf = inputs.normal(31, inputs.TAG_B, (K, N))
    try:
        bpx.force_tile(4)
        C = run(plan, A, B)
        assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))
        Cf4 = run(plan, Af, Bf)
        bpx.force_tile(1)
        Cf1 = run(plan, Af, Bf)
    finally:
        bpx.force_tile(-1)
    assert np.array_equal(Cf4, Cf1)


@pytest.mark.parametrize("prec", [bpx.PREC_BF16, bpx.PREC_BF16X3])
def test_bf16_flat_tile_k_tails_and_degrees(prec):
    """The flat tiling's k loop for every stage count from 1 to 7 (its
    two-stage body and each tail after it) and for tiles whose largest
    symbol degree runs from 1 to 4: the (12,8,4) code in FULL mode (all 48
    symbols, degrees 1 to 4), Mb = 64, so a 128-row tile holds two symbols.
    Integer operands decode exactly; float operands give the per-symbol
    tiling's bits."""
    s = inputs.CODE_1284
    code = bpx.Code.search(s.n, s.k, s.b, s.sigma, s.seed, s.restarts, s.iters, walk=s.walk)
    M, N = 32 * 64 - 37, 260
    for nk in range(1, 8):
        K = 32 * nk
        plan = bpx.Plan(code, list(range(12)), 0, bpx.MODE_FULL, M, K, N, prec)
        assert plan.decodable
        A = inputs.integers(40 + nk, inputs.TAG_A, (M, K))
        B = inputs.integers(40 + nk, inputs.TAG_B, (K, N))
        Af = inputs.normal(40 + nk, inputs.TAG_A, (M, K))
        Bf = inputs.normal(40 + nk, inputs.TAG_B, (K, N))
        _say("flat k tail", "prec", prec, "K", K)
        try:
            bpx.force_tile(4)
            C = run(plan, A, B)
            assert np.array_equal(C.astype(np.float64),
                                  A.astype(np.float64) @ B.astype(np.float64)), K
            Cf4 = run(plan, Af, Bf)
            bpx.force_tile(1)
            Cf1 = run(plan, Af, Bf)
        finally:
            bpx.force_tile(-1)
        assert np.array_equal(Cf4, Cf1), K


def test_grouped_flat_tile_exact_and_identical_to_per_symbol_tile():
    """The grouped launch with every product on the flat-row tiling: integer
    operands bit exact, float operands bit-identical to the per-symbol
    tiling."""
    outs = {}
    for tile in (4, 1):
        for integer in (True, False):
            try:
                bpx.force_tile(tile)
                plans, As, Bs, Cs, ws, ops = _group_case(5, 16, integer, mult=32)
                g = bpx.Group(plans, As, Bs, Cs, ws)
            finally:
                bpx.force_tile(-1)
            g.launch()
            torch.cuda.synchronize()
            outs[tile, integer] = [host(c) for c in Cs]
            if integer:
                for (A, B), C in zip(ops, outs[tile, integer]):
                    assert np.array_equal(C.astype(np.float64),
                                          A.astype(np.float64) @ B.astype(np.float64))
            del g
    for a, b in zip(outs[4, False], outs[1, False]):
        assert np.array_equal(a, b)


def test_bf16x3_row_scaled_workload():
    """512^3, A rows scaled log-uniformly in [1e-3, 1e3], (6,4,2) code with two
    erased columns: split-BF16x3 must stay within 1e-5 of float64."""
    w = inputs.WORKLOADS["bf16_small"]
    A, B = inputs.operands(w, seed=0)
    arrival, lost, _ = inputs.arrival_of(w, seed=0)
    code = code642()
    R = pipeline.uncoded(A, B)
    errs = {}
    worst = {}
    rows = np.arange(w.M)
    for prec in (bpx.PREC_BF16X3, bpx.PREC_BF16):
        plan = bpx.Plan(code, arrival, lost, bpx.MODE_ERASURE, w.M, w.K, w.N, prec)
        C = run(plan, A, B)
        errs[prec] = relf(C, R)
        worst[prec] = worst_errors(C, R, rows, plan.info()["Mb"])
    _say("bf16_small relF", errs)
    for prec, wv in worst.items():
        _say("bf16_small prec", prec, "worst row", wv["row"], "at", wv["row_at"],
             "worst block", wv["block"], "at", wv["block_at"])
    assert errs[bpx.PREC_BF16X3] <= TOL_BF16X3
    assert errs[bpx.PREC_BF16] <= 1e-2          # one bf16 rounding per operand
    # Per row the error is not bounded by the target: a coded sum mixes rows
    # scaled up to 1e6 apart, and subtracting the large rows' share leaves
    # the small row with the large rows' rounding.  Each block is a mix of
    # all scales, so per block the error stays near the Frobenius one.
    assert worst[bpx.PREC_BF16X3]["block"] <= 4 * TOL_BF16X3


def test_bf16x3_deep_chain_float():
    """Table III's depth-9 chain: each release subtracts a decoded block, so
    the independent errors of the degree-2 coded products add in quadrature
    along the chain; block s at depth d carries about sqrt(2 d) times the
    error e of one split-BF16x3 product (e <= 1e-5 is the single-product
    bound).  Averaged over depths 1..9 that is sqrt(10) e."""
    code = bpx.Code.table3()
    M, K, N = 9 * 40, 256, 136
    plan = bpx.Plan(code, [0, 1, 2, 3, 4], 2, bpx.MODE_ERASURE, M, K, N, bpx.PREC_BF16X3)
    A = inputs.normal(12, inputs.TAG_A, (M, K))
    B = inputs.normal(12, inputs.TAG_B, (K, N))
    C = run(plan, A, B)
    e = relf(C, pipeline.uncoded(A, B))
    _say("bf16x3 depth-9 chain relF", e)
    assert e <= TOL_BF16X3 * np.sqrt(10)


# ------------------------------------------------------------- FP8 paths --

TOL_FP8 = 3e-2


def test_fp8_codes_and_scales_match_oracle():
    """The FP8 encode+quantise pass: every code byte and scale of the coded
    A tiles (and the FP8x2 residual codes) and of B equals the oracle's
    quantiser, which follows the OCP e4m3 definition in the same float32
    order (ragged M, K, N)."""
    from oracle import quant
    code = code642()
    oc = oracle_of(code)
    M, K, N = 300, 260, 200
    A = inputs.normal(21, inputs.TAG_A, (M, K))
    B = inputs.normal(21, inputs.TAG_B, (K, N))
    plan = bpx.Plan(code, [5, 3, 0, 1, 2, 4], 0, bpx.MODE_STRAGGLER, M, K, N, bpx.PREC_FP8X2)
    Ad, Bd = padded(A), padded(B)
    Cd = torch.zeros((M, -(-N // 4) * 4), device="cuda")[:, :N]
    ws = bpx.alloc_workspace(plan)
    bpx.coded_gemm(plan, Ad, Bd, Cd, ws)
    raw = host(ws)
    off = plan.workspace_layout()
    Mb = plan.info()["Mb"]
    r = lambda x: -(-x // 128) * 128
    Mbp, Kp, Np = r(Mb), r(K), r(N)
    comp = plan.schedule()["computed"].tolist()
    aq = raw[off[1]:off[1] + len(comp) * Mbp * Kp].reshape(len(comp), Mbp, Kp)
    aq2 = raw[off[2]:off[2] + len(comp) * Mbp * Kp].reshape(len(comp), Mbp, Kp)
    sa = raw[off[3]:off[3] + len(comp) * (Mbp // 128) * (Kp // 128) * 4].view(np.float32)
    sa = sa.reshape(len(comp), Mbp // 128, Kp // 128)
    bq = raw[off[4]:off[4] + Np * Kp].reshape(Np, Kp)
    sb = raw[off[5]:off[5] + (Kp // 128) * (Np // 128) * 4].view(np.float32).reshape(Kp // 128, Np // 128)
    sym = {g: d for g, _, d in oc.symbols()}
    for i, g in enumerate(comp):
        blk = np.zeros((Mbp, Kp), dtype=np.float32)
        blk[:Mb, :K] = quant.coded_block_fp32(A, Mb, sym[g], M)
        for rb in range(Mbp // 128):
            for kb in range(Kp // 128):
                tile = blk[rb * 128:(rb + 1) * 128, kb * 128:(kb + 1) * 128]
                s, c1, c2 = quant.quantize_block(tile, residual=True)
                assert sa[i, rb, kb] == s, (g, rb, kb)
                got1 = aq[i, rb * 128:(rb + 1) * 128, kb * 128:(kb + 1) * 128]
                got2 = aq2[i, rb * 128:(rb + 1) * 128, kb * 128:(kb + 1) * 128]
                assert np.array_equal(got1, c1), (g, rb, kb, np.argwhere(got1 != c1)[:3])
                assert np.array_equal(got2, c2), (g, rb, kb)
    Bp = np.zeros((Kp, Np), dtype=np.float32)
    Bp[:K, :N] = B
    for kb in range(Kp // 128):
        for nb in range(Np // 128):
            s, c = quant.quantize_block(Bp[kb * 128:(kb + 1) * 128, nb * 128:(nb + 1) * 128])
            assert sb[kb, nb] == s
            assert np.array_equal(bq[nb * 128:(nb + 1) * 128, kb * 128:(kb + 1) * 128], c.T)


@pytest.mark.parametrize("prec", [bpx.PREC_FP8, bpx.PREC_FP8X2])
def test_fp8_gemm_products_match_quantised_codes(prec):
    """Each coded product of the FP8 GEMM, under both tilings (one 128x128
    grid per symbol; 128x256 tiles over all symbols' codes), against the
    same product formed in float64 from the oracle's codes and scales: per
    128-wide k chunk, sA sB (qA . qB), with qA + qA2/16 for FP8x2, summed
    over the chunks.  What separates them is the MFMA's own accumulation of
    the 128 FP8 products of a chunk, which is not a sequence of IEEE FP32
    additions (measured about 1.5e-5 relative on these operands), so the
    bound is 1e-4, far below what a wrong index, scale or plane gives
    (order 1).  The two tilings run the same MFMA sequence per output (the
    scales, the residual plane's 2^-4 included, in the MFMA's E8M0
    operands) and give the same bits."""
    from oracle import quant
    code = code642()
    oc = oracle_of(code)
    M, K, N = 2048, 384, 512          # Mb = 256; N a multiple of 256
    A = inputs.normal(24, inputs.TAG_A, (M, K))
    B = inputs.normal(24, inputs.TAG_B, (K, N))
    order = [5, 3, 0, 1, 2, 4]
    plan = bpx.Plan(code, order, 0, bpx.MODE_FULL, M, K, N, prec)
    sch = plan.schedule()
    Mb = plan.info()["Mb"]
    n_comp = plan.info()["n_computed"]
    x2 = prec == bpx.PREC_FP8X2
    Bh = np.zeros((K, N))
    sB = {}
    for kb in range(K // 128):
        for nb in range(N // 128):
            s, c = quant.quantize_block(B[kb * 128:(kb + 1) * 128, nb * 128:(nb + 1) * 128])
            sB[kb, nb] = float(s)
            Bh[kb * 128:(kb + 1) * 128, nb * 128:(nb + 1) * 128] = quant.e4m3_decode(c)
    sym = {g: d for g, _, d in oc.symbols()}
    refs = {}
    for g in sch["computed"].tolist():
        blk = quant.coded_block_fp32(A, Mb, sym[g], M)
        ref = np.zeros((Mb, N))
        for rb in range(Mb // 128):
            for kb in range(K // 128):
                t = blk[rb * 128:(rb + 1) * 128, kb * 128:(kb + 1) * 128]
                if x2:
                    s, c1, c2 = quant.quantize_block(t, residual=True)
                    ah = quant.e4m3_decode(c1) + quant.e4m3_decode(c2) / 16.0
                else:
                    s, c1 = quant.quantize_block(t)
                    ah = quant.e4m3_decode(c1)
                for nb in range(N // 128):
                    ref[rb * 128:(rb + 1) * 128, nb * 128:(nb + 1) * 128] += (
                        float(s) * sB[kb, nb] *
                        (ah @ Bh[kb * 128:(kb + 1) * 128, nb * 128:(nb + 1) * 128]))
        refs[g] = ref
    got = {}
    for tile in (0, 1):
        Cd = torch.zeros((M, N), device="cuda")
        ws = bpx.alloc_workspace(plan)
        try:
            bpx.force_tile(tile)
            bpx.coded_gemm(plan, dev(A), dev(B), Cd, ws)
        finally:
            bpx.force_tile(-1)
        Y = host(ws)[:n_comp * Mb * N * 4].view(np.float32)
        C = host(Cd)
        for g, d in zip(sch["computed"].tolist(), sch["dest"].tolist()):
            if d >= 0:
                y = Y[d * Mb * N:(d + 1) * Mb * N].reshape(Mb, N).copy()
            else:
                y = C[(-1 - d) * Mb:(-d) * Mb].copy()
            e = relf(y, refs[g])
            assert e <= 1e-4, (g, tile, prec, e)
            got[tile, g] = y
    for g in sch["computed"].tolist():
        assert np.array_equal(got[1, g], got[0, g]), g


def test_fp8_mojette_end_to_end():
    """Mojette Construction A (k=16, n=24, b=8), 8 of 24 columns erased, at
    the workload's M (Mb = 128, one scale block per data block) and reduced
    K, N, with N a multiple of 256 so that the wide 128x256 FP8 kernel the
    benchmark runs does the products: FP8x2 within 3e-2 of float64; 1-pass
    FP8 reported."""
    code = bpx.Code.mojette(16, 8, 24, 0)
    M, K, N = 16384, 512, 768
    A = inputs.normal(22, inputs.TAG_A, (M, K))
    B = inputs.normal(22, inputs.TAG_B, (K, N))
    R = pipeline.uncoded(A, B)
    errs = {}
    for seed in range(3):
        arrival, lost = inputs.erasure_arrival(seed, 24, 8)
        for prec in (bpx.PREC_FP8X2, bpx.PREC_FP8):
            plan = bpx.Plan(code, arrival, lost, bpx.MODE_ERASURE, M, K, N, prec)
            C = run(plan, A, B)
            errs[(seed, prec, plan.info()["prefix_m"])] = relf(C, R)
    _say("fp8 mojette relF", errs)
    # 1-pass FP8 has no accuracy target: one e4m3 rounding per operand
    # already gives ~3.7e-2 uncoded, and a release through a degree-d bin
    # moves the quantisation error of the whole d-block sum onto one block.
    # It gets a loose sanity bound; FP8x2 must meet the 3e-2 target.
    for (seed, prec, m), e in errs.items():
        assert e <= (TOL_FP8 if prec == bpx.PREC_FP8X2 else 0.1), (seed, prec, m, e)


def test_fp8_mojette_full_size_sampled():
    """The FP8x2 Mojette workload at full size in the benchmark's launch
    (A 16384^2, B 16384x8192 N(0,1), Construction A k=16 n=24 b=8, 8 of 24
    columns erased by seed 0, Mb = 128, wide 128x256 FP8 tiles): two
    sampled rows of every one of the 128 data blocks against float64,
    within 3e-2 overall; the worst block and row are reported."""
    w = inputs.WORKLOADS["fp8_mojette"]
    assert (w.M, w.K, w.N) == (16384, 16384, 8192)
    A, B = inputs.operands(w, seed=0)
    arrival, lost, _ = inputs.arrival_of(w, seed=0)
    code = lib_code(w.code)
    plan = bpx.Plan(code, arrival, lost, bpx.MODE_ERASURE, w.M, w.K, w.N, bpx.PREC_FP8X2)
    inf = plan.info()
    _say("fp8_mojette plan", inf)
    assert inf["decodable"] and inf["Mb"] == 128
    C = run(plan, A, B)
    rows = np.concatenate([[s * 128 + 7, s * 128 + 101] for s in range(128)])
    R = A[rows].astype(np.float64) @ B.astype(np.float64)
    e = relf(C[rows], R)
    worst = worst_errors(C[rows], R, rows, 128)
    _say("fp8_mojette sampled relF", e, "worst row", worst["row"], "at", worst["row_at"],
         "worst block", worst["block"], "at", worst["block_at"])
    assert e <= TOL_FP8
    assert worst["block"] <= 2 * TOL_FP8
    assert np.isfinite(C).all()


def test_fp8_wide_tile_past_4gib_of_codes():
    """Mojette Construction A (k=16, n=24, b=8) in FULL mode at M = K =
    16384: 2112 coded blocks of 128 rows, so each FP8 code plane is 2112 x
    128 x 16384 bytes, past 2^32.  The wide 128x256 kernel (addressing each
    tile from a 64-bit base) must agree with the per-symbol 128x128 tile
    (1e-6: same codes, the MFMA's own summation order) and with float64 on
    two sampled rows of every block (3e-2)."""
    code = bpx.Code.mojette(16, 8, 24, 0)
    M, K, N = 16384, 16384, 256
    A = inputs.normal(24, inputs.TAG_A, (M, K))
    B = inputs.normal(24, inputs.TAG_B, (K, N))
    plan = bpx.Plan(code, list(range(24)), 0, bpx.MODE_FULL, M, K, N, bpx.PREC_FP8X2)
    inf = plan.info()
    _say("fp8 FULL plan", inf)
    assert inf["decodable"] and inf["Mb"] == 128
    assert inf["n_computed"] * 128 * K > 2 ** 32
    C_wide = run(plan, A, B)
    try:
        bpx.force_tile(0)
        C_sym = run(plan, A, B)
    finally:
        bpx.force_tile(-1)
    d = relf(C_wide, C_sym)
    rows = np.concatenate([[s * 128 + 5, s * 128 + 99] for s in range(128)])
    R = A[rows].astype(np.float64) @ B.astype(np.float64)
    e = relf(C_wide[rows], R)
    _say("fp8 FULL wide vs per-symbol", d, "sampled relF", e)
    assert np.isfinite(C_wide).all()
    assert d <= 1e-6
    assert e <= TOL_FP8


def test_fp8_integer_operands_small_chain():
    # Table III depth-9 chain through the FP8x2 path: the relative error
    # stays at the FP8 level (no blow-up through the subtraction chain).
    code = bpx.Code.table3()
    M, K, N = 9 * 64, 512, 256
    A = inputs.normal(23, inputs.TAG_A, (M, K))
    B = inputs.normal(23, inputs.TAG_B, (K, N))
    plan = bpx.Plan(code, [0, 1, 2, 3, 4], 2, bpx.MODE_ERASURE, M, K, N, bpx.PREC_FP8X2)
    C = run(plan, A, B)
    e = relf(C, pipeline.uncoded(A, B))
    _say("fp8x2 depth-9 chain relF", e)
    assert e <= TOL_FP8 * np.sqrt(10)


# ---------------------------------------------------------- grouped path --

def _group_case(seed, count, integer, mult=4):
    """count products with shapes from the batch generator (scaled down),
    codes (6,4,2) or (12,8,2) by k, own seeded erasure patterns."""
    codes_by_k = {4: code642(), 8: lib_code(inputs.CODE_1282)}
    shapes = inputs.batch_shapes(seed, count, lo=128, hi=640, mult=mult)
    plans, As, Bs, Cs, host_ops = [], [], [], [], []
    for i, (M, K, N, k) in enumerate(shapes):
        code = codes_by_k[k]
        n = code.info()["n"]
        arrival, _ = inputs.erasure_arrival(seed * 1000 + i, n, n - k)
        plan = bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, bpx.PREC_BF16X3)
        if integer:
            A = inputs.integers(seed * 1000 + i, inputs.TAG_A, (M, K))
            B = inputs.integers(seed * 1000 + i, inputs.TAG_B, (K, N))
        else:
            A = inputs.normal(seed * 1000 + i, inputs.TAG_A, (M, K))
            B = inputs.normal(seed * 1000 + i, inputs.TAG_B, (K, N))
        plans.append(plan)
        As.append(dev(A))
        Bs.append(dev(B))
        Cs.append(torch.full((M, N), float("nan"), device="cuda"))
        host_ops.append((A, B))
    ws = torch.empty(bpx.group_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    return plans, As, Bs, Cs, ws, host_ops


def test_grouped_integer_exact_and_float_tolerance():
    """Integer operands: every product bit exact.  Float operands: the batch's
    relative Frobenius error (all products together) within the BF16x3 bound
    1e-5, and each product within sqrt(2 d) times it, d its deepest release
    round (independent product errors add in quadrature along a chain)."""
    for integer in (True, False):
        plans, As, Bs, Cs, ws, ops = _group_case(3 if integer else 4, 24, integer)
        g = bpx.Group(plans, As, Bs, Cs, ws)
        g.launch()
        torch.cuda.synchronize()
        num = den = 0.0
        errs = []
        for i, (A, B) in enumerate(ops):
            C = host(Cs[i])
            R = A.astype(np.float64) @ B.astype(np.float64)
            if integer:
                assert np.array_equal(C.astype(np.float64), R), i
                continue
            d = plans[i].info()["depth_max"]
            e = relf(C, R)
            errs.append((i, d, e))
            assert e <= TOL_BF16X3 * np.sqrt(2 * d), (i, d, e)
            num += float(np.sum((C - R) ** 2))
            den += float(np.sum(R ** 2))
        if not integer:
            _say("grouped bf16x3 per-product (i, depth, relF)", errs)
            _say("grouped bf16x3 batch relF", np.sqrt(num / den))
            assert np.sqrt(num / den) <= TOL_BF16X3


def test_batch_full_size_sampled():
    """The bench's batch at full size: 256 products (M, K, N log-uniform in
    [256, 4096]), codes (6,4,2) and (12,8,2) with their own seeded erasures,
    BF16x3, one grouped launch (persistent GEMM and peel over all
    products).  Four sampled rows of every product against float64: the
    whole sample within the BF16x3 bound, each product within sqrt(2 d) of
    it (d its deepest release round)."""
    codes_by_k = {4: code642(), 8: lib_code(inputs.CODE_1282)}
    shapes = inputs.batch_shapes(0, 256)
    plans, As, Bs, Cs, samples = [], [], [], [], []
    for i, (M, K, N, k) in enumerate(shapes):
        code = codes_by_k[k]
        n = code.info()["n"]
        arrival, _ = inputs.erasure_arrival(i, n, n - k)
        plans.append(bpx.Plan(code, arrival, 0, bpx.MODE_STRAGGLER, M, K, N, bpx.PREC_BF16X3))
        g = torch.Generator(device="cuda").manual_seed(1000 + i)
        As.append(torch.randn(M, K, device="cuda", generator=g))
        Bs.append(torch.randn(K, N, device="cuda", generator=g))
        Cs.append(torch.full((M, N), float("nan"), device="cuda"))
        samples.append(np.linspace(0, M - 1, 4).astype(np.int64))
    ws = torch.empty(bpx.group_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    _say("batch full size: products", len(plans))
    grp = bpx.Group(plans, As, Bs, Cs, ws)
    grp.launch()
    torch.cuda.synchronize()
    num = den = 0.0
    for i, rows in enumerate(samples):
        r = torch.from_numpy(rows).cuda()
        Cr = Cs[i].index_select(0, r).cpu().numpy().astype(np.float64)
        R = (As[i].index_select(0, r).cpu().double() @ Bs[i].cpu().double()).numpy()
        assert np.isfinite(Cr).all(), i
        d = plans[i].info()["depth_max"]
        assert relf(Cr, R) <= TOL_BF16X3 * np.sqrt(2 * max(d, 1)), (i, d)
        num += float(np.sum((Cr - R) ** 2))
        den += float(np.sum(R ** 2))
    _say("batch full size sampled relF", np.sqrt(num / den))
    assert np.sqrt(num / den) <= TOL_BF16X3


def test_grouped_graph_replay_matches_eager():
    plans, As, Bs, Cs, ws, ops = _group_case(5, 16, False)
    g = bpx.Group(plans, As, Bs, Cs, ws)
    g.launch()
    torch.cuda.synchronize()
    eager = [c.clone() for c in Cs]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            g.launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for c in Cs:
            c.fill_(float("nan"))               # eager work between replays
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for c, e in zip(Cs, eager):
            assert torch.equal(c, e), rep
        del junk


@pytest.mark.parametrize("prec", [bpx.PREC_F32, bpx.PREC_BF16X3, bpx.PREC_FP8X2])
def test_single_product_graph_replay_matches_eager(prec):
    """One product through the two-launch path captured in a HIP graph, as
    the benchmark times it: the (12,8,4) code, Mb = 256, a shifted-
    exponential arrival (36 coded products, a peel of depth up to 12); FP32
    takes the 256x256 tiles with the short grid split along K and reduced,
    BF16x3 the B split and flat tiles, FP8x2 the B and A quantisation and
    the wide FP8 tiles.  Three replays with eager work in between each
    equal the eager result bit for bit."""
    s_ = inputs.CODE_1284
    code = bpx.Code.search(s_.n, s_.k, s_.b, s_.sigma, s_.seed, s_.restarts, s_.iters,
                           walk=s_.walk)
    perm, _ = inputs.shifted_exp_arrival(0, 12)
    M, K, N = 8192, 1024, 1024
    plan = bpx.Plan(code, list(perm), 0, bpx.MODE_STRAGGLER, M, K, N, prec)
    assert plan.decodable
    plan.upload()
    A = torch.from_numpy(inputs.normal(9, inputs.TAG_A, (M, K))).cuda()
    B = torch.from_numpy(inputs.normal(9, inputs.TAG_B, (K, N))).cuda()
    ws = bpx.alloc_workspace(plan)
    C_eager = torch.empty((M, N), device="cuda")
    bpx.coded_matmul(plan, A, B, C_eager, ws)
    torch.cuda.synchronize()
    C = torch.empty((M, N), device="cuda")
    graph = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            bpx.coded_matmul(plan, A, B, C, ws)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    _say("graph replay", prec, plan.info())
    for rep in range(3):
        C.fill_(float("nan"))
        ws.fill_(0xA5)                          # the workspace is rewritten by every replay
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, C_eager), rep
        del junk


def test_distinct_plans_from_two_threads_on_two_streams():
    """Distinct plan handles used from two host threads at once, each on its
    own stream (default priority): the (6,4,2) code in FP32 (two columns
    erased) and the (12,8,4) code in BF16x3 (straggler prefix), five calls
    each, every result equal to the same call made alone beforehand.  The first call of each thread also uploads its
    plan's tables (under the library's lock)."""
    import threading
    s_ = inputs.CODE_1284
    c1284 = bpx.Code.search(s_.n, s_.k, s_.b, s_.sigma, s_.seed, s_.restarts, s_.iters,
                            walk=s_.walk)
    jobs = []
    arr642, lost642 = inputs.erasure_arrival(40, 6, 2)
    arr1284, _ = inputs.shifted_exp_arrival(41, 12)
    for i, (code, perm, lost, mode, prec, M, K, N) in enumerate(
            [(code642(), arr642, lost642, bpx.MODE_ERASURE, bpx.PREC_F32, 1024, 512, 768),
             (c1284, arr1284, 0, bpx.MODE_STRAGGLER, bpx.PREC_BF16X3, 2048, 512, 512)]):
        ref_plan = bpx.Plan(code, list(perm), lost, mode, M, K, N, prec)
        assert ref_plan.decodable
        A = torch.from_numpy(inputs.normal(40 + i, inputs.TAG_A, (M, K))).cuda()
        B = torch.from_numpy(inputs.normal(40 + i, inputs.TAG_B, (K, N))).cuda()
        want = torch.empty((M, N), device="cuda")
        bpx.coded_matmul(ref_plan, A, B, want, bpx.alloc_workspace(ref_plan))
        torch.cuda.synchronize()
        plan = bpx.Plan(code, list(perm), lost, mode, M, K, N, prec)
        jobs.append((plan, A, B, want, bpx.alloc_workspace(plan),
                     torch.empty((M, N), device="cuda"), torch.cuda.Stream()))
    errors = []

    def body(plan, A, B, want, ws, C, stream):
        try:
            with torch.cuda.stream(stream):
                for _ in range(5):
                    C.fill_(float("nan"))
                    bpx.coded_matmul(plan, A, B, C, ws, stream=stream)
                    stream.synchronize()
                    if not torch.equal(C, want):
                        errors.append("result differs")
        except Exception as e:
            errors.append(repr(e))

    ts = [threading.Thread(target=body, args=j) for j in jobs]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors


def test_grouped_peel_split_mixed_programs_exact():
    """The grouped peel's workgroup ranges are cut by program cost: a group
    mixing products with no peel steps (identity code, every block its own
    symbol), short and long programs, and tiny and large shapes still peels
    every block of every product exactly once (integer operands: exact), and
    the flat GEMM's grouped tile order covers every tile."""
    ident = bpx.Code.identity(4, 2)
    c642 = code642()
    c1282 = lib_code(inputs.CODE_1282)
    cases = [(ident, [0, 1, 2, 3], 64, 96, 128), (c1282, None, 1024, 256, 768),
             (c642, None, 32, 32, 64), (ident, [0, 1, 2, 3], 512, 64, 256),
             (c1282, None, 256, 128, 2048), (c642, None, 1536, 96, 384)]
    plans, As, Bs, Cs, ops = [], [], [], [], []
    for i, (code, arrival, M, K, N) in enumerate(cases):
        if arrival is None:
            n = code.info()["n"]
            arrival, _ = inputs.erasure_arrival(700 + i, n, n - code.info()["k"])
        plans.append(bpx.Plan(code, list(arrival), 0, bpx.MODE_STRAGGLER, M, K, N,
                              bpx.PREC_BF16X3))
        A = inputs.integers(700 + i, inputs.TAG_A, (M, K))
        B = inputs.integers(700 + i, inputs.TAG_B, (K, N))
        As.append(dev(A))
        Bs.append(dev(B))
        Cs.append(torch.full((M, N), float("nan"), device="cuda"))
        ops.append((A, B))
    steps = [p.peel_program()["steps"].shape[0] for p in plans]
    assert min(steps) == 0 and max(steps) > 4, steps
    ws = torch.empty(bpx.group_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    g = bpx.Group(plans, As, Bs, Cs, ws)
    g.launch()
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(ops):
        R = A.astype(np.float64) @ B.astype(np.float64)
        assert np.array_equal(host(Cs[i]).astype(np.float64), R), i


def test_grouped_rejects_undecodable():
    code = bpx.Code.table3()
    good = bpx.Plan(code, [0, 1, 2, 3, 4], 0, bpx.MODE_STRAGGLER, 36, 8, 8, bpx.PREC_BF16X3)
    bad = bpx.Plan(code, [0, 1, 2, 3, 4], 3, bpx.MODE_ERASURE, 36, 8, 8, bpx.PREC_BF16X3)
    A = [torch.zeros((36, 8), device="cuda") for _ in range(2)]
    B = [torch.zeros((8, 8), device="cuda") for _ in range(2)]
    C = [torch.zeros((36, 8), device="cuda") for _ in range(2)]
    ws = torch.empty(bpx.group_workspace_bytes([good, bad]) + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(bpx.BpxError) as e:
        bpx.Group([good, bad], A, B, C, ws)
    assert e.value.status == bpx.E_UNDECODABLE
