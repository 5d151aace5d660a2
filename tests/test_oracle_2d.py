"""Pins of the oracle's two-dimensional form (Sec. III-A, Examples 1-2)
against what the paper states and against plain linear algebra."""
import itertools

import numpy as np

from oracle import codes, pipeline2d
from oracle.peeling import ERASURE, make_plan
from paper_1904_11563_amd import inputs


def test_gray_ratios_of_tables_one_and_three():
    # Example 2: distributed encoding is required for 2/10 of Table I's
    # symbols and 6/15 of Table III's
    assert pipeline2d.gray_ratio(codes.table1()) == 2 / 10
    assert pipeline2d.gray_ratio(codes.table3()) == 6 / 15


def test_table1_gray_cells_are_the_shaded_ones():
    t1 = codes.table1()
    gray = [d for _, _, d in t1.symbols() if pipeline2d.kind(d, 2) == "gray"]
    # v2 + v3 and v1 + v4 (zero-based ids 1, 2 and 0, 3)
    assert sorted(gray) == [(0, 3), (1, 2)]


def test_symbol_products_match_independent_forms():
    rng = np.random.default_rng(5)
    A = rng.integers(-8, 9, size=(6, 5)).astype(np.float64)   # rows a_1 | a_2
    B = rng.integers(-8, 9, size=(5, 4)).astype(np.float64)   # cols b_1 | b_2
    a1, a2 = A[:3], A[3:]
    b1, b2 = B[:, :2], B[:, 2:]
    t1 = codes.table1()
    sym = {d: g for g, _, d in t1.symbols()}
    Y = pipeline2d.coded_products(A, B, t1, list(sym.values()))
    # gray: the K-concatenated product [a_1 | a_2] [b_2 ; b_1]
    assert np.array_equal(Y[sym[(1, 2)]], np.hstack([a1, a2]) @ np.vstack([b2, b1]))
    # shared A block: a_1 (b_1 + b_2); shared B block: (a_1 + a_2) b_1
    assert np.array_equal(Y[sym[(0, 1)]], a1 @ (b1 + b2))
    assert np.array_equal(Y[sym[(0, 2)]], (a1 + a2) @ b1)


def _exact_all_patterns(code, n_lost, M, K, N, seed):
    A = inputs.integers(seed, inputs.TAG_A, (M, K)).astype(np.float64)
    B = inputs.integers(seed, inputs.TAG_B, (K, N)).astype(np.float64)
    R = A @ B
    ok = 0
    for lost in itertools.combinations(range(code.n), n_lost):
        order = [j for j in range(code.n) if j not in lost] + list(lost)
        plan = make_plan(code, order, n_lost, ERASURE)
        if not plan.decodable:
            continue
        C = pipeline2d.coded_matmul_ref(A, B, code, plan)
        assert np.array_equal(C, R), lost
        ok += 1
    return ok


def test_table1_every_two_lost_decodes_exactly():
    # any 2 of the 5 nodes suffice (Example 1), ragged M and N
    assert _exact_all_patterns(codes.table1(), 3, 7, 6, 9, 11) == 10


def test_table3_every_two_lost_decodes_exactly():
    assert _exact_all_patterns(codes.table3(), 2, 10, 4, 8, 12) == 10


def test_grid_side_needs_a_square():
    assert pipeline2d.grid_side(9) == 3
    try:
        pipeline2d.grid_side(8)
    except ValueError:
        return
    raise AssertionError("k*b = 8 accepted")
