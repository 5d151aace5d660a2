"""Pins of the oracle's numeric pipeline (encode, products, peel)."""
from itertools import combinations

import numpy as np
import pytest

from oracle import codes, pipeline
from oracle.peeling import ERASURE, FULL, MIN, STRAGGLER, make_plan


def _int_inputs(seed, M, K, N):
    rng = np.random.default_rng(seed)
    A = rng.integers(-8, 9, size=(M, K)).astype(np.float64)
    B = rng.integers(-8, 9, size=(K, N)).astype(np.float64)
    return A, B


def _orders(c):
    for t in range(c.k, c.n + 1):
        for sub in combinations(range(c.n), t):
            yield list(sub) + [j for j in range(c.n) if j not in sub], c.n - t


@pytest.mark.parametrize("code", [codes.table1(), codes.table3(),
                                  codes.mojette(3, 4, 5, 0), codes.mojette(4, 2, 6, 0),
                                  codes.array_search(6, 4, 2, 3, seed=0, restarts=1, iters=60)],
                         ids=["table1", "table3", "mojA_3x4", "mojA_4x2", "search642"])
def test_integer_inputs_decode_exactly(code):
    # With integer A, B in [-8, 8] and K <= 4096 every float64 operation of
    # encode, products and peel is exact, so the decoded product must equal
    # A.B bit for bit for every decodable erasure pattern.
    M, K, N = 7 * code.kb + 3, 37, 11       # ragged last block
    A, B = _int_inputs(code.kb, M, K, N)
    R = A @ B
    n_dec = 0
    for order, lost in _orders(code):
        plan = make_plan(code, order, lost, ERASURE)
        if not plan.decodable:
            continue
        n_dec += 1
        C = pipeline.coded_matmul_ref(A, B, code, plan)
        assert C.shape == R.shape
        assert np.array_equal(C, R), order
    assert n_dec > 0


def test_integer_exact_full_and_min_modes():
    code = codes.table3()
    A, B = _int_inputs(3, 50, 64, 9)
    for mode in (FULL, MIN, STRAGGLER):
        plan = make_plan(code, [3, 4, 0, 1, 2], 0, mode)
        C = pipeline.coded_matmul_ref(A, B, code, plan)
        assert np.array_equal(C, A @ B)


def test_float_inputs_close_to_uncoded():
    rng = np.random.default_rng(0)
    code = codes.table3()
    A = rng.standard_normal((90, 40)).astype(np.float32)
    B = rng.standard_normal((40, 33)).astype(np.float32)
    plan = make_plan(code, [0, 1, 2, 3, 4], 2, ERASURE)     # depth-9 chain
    C = pipeline.coded_matmul_ref(A, B, code, plan)
    assert pipeline.rel_frobenius(C, pipeline.uncoded(A, B)) < 1e-12


def test_encode_is_block_sum():
    # C_g of Table I symbol v2+v3 (node 1, processor 2) is A_1 + A_2.
    code = codes.table1()
    A = np.arange(8 * 3, dtype=np.float64).reshape(8, 3)
    enc = pipeline.encode(A, code, [1])
    blocks = pipeline.data_blocks(A, 4)
    assert np.array_equal(enc[1], blocks[1] + blocks[2])
    assert np.array_equal(blocks[3], A[6:8])


def test_padding_rows_are_zero():
    A = np.ones((5, 2))
    blocks = pipeline.data_blocks(A, 4)      # Mb = 2, last block has no rows
    assert blocks[2].tolist() == [[1, 1], [0, 0]]
    assert not blocks[3].any()


def test_planted_sign_error_is_caught():
    # The exactness pin must fail for a peel that adds instead of subtracts.
    code = codes.table1()
    A, B = _int_inputs(1, 8, 5, 3)
    plan = make_plan(code, [0, 1, 2, 3, 4], 3, ERASURE)
    Y = pipeline.coded_products(pipeline.encode(A, code, plan.computed), B)
    X = [None] * code.kb
    for s in plan.order():
        acc = Y[plan.releaser[s]].copy()
        for u in plan.sub[s]:
            acc = acc + X[u]          # planted mistake
        X[s] = acc
    assert not np.array_equal(pipeline.assemble(X, 8), A @ B)
