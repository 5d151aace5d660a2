"""The paper's two-dimensional form in float64 (test infrastructure).

Sec. III-A, Examples 1 and 2: A is split into m row blocks a_1..a_m and B
into m column blocks b_1..b_m, and the information symbols are the block
products v = a_r b_c of the m x m grid, numbered row by row (v_1 = a_1 b_1,
v_2 = a_1 b_2, ..., v_{m+1} = a_2 b_1, ...), so k*b = m^2.  A coded symbol is
the sum of its information symbols.  When all of them share an A block (the
same r) it is a_r times a sum of B blocks, and when they share a B block (the
same c) it is a sum of A blocks times b_c: the encode can happen on the
inputs.  Otherwise (the paper's gray cells) the processor has to form the
sum of its products itself.  With the same incidence structure the peel of
Sec. I-A recovers every v exactly in exact arithmetic, and the blocks of
A.B are the recovered v.

Zero-based here: data id s = r*m + c for r, c in [0, m).  Row blocks hold
Mb = ceil(M/m) rows and column blocks Nb = ceil(N/m) columns, zero padded.
"""

from __future__ import annotations

from math import isqrt

import numpy as np

from .pipeline import peel_numeric


def grid_side(kb: int) -> int:
    """m with m*m = kb (the 2-D form needs a square grid)."""
    m = isqrt(kb)
    if m * m != kb:
        raise ValueError("k*b is not a perfect square")
    return m


def rc(s: int, m: int):
    """(r, c) of data id s."""
    return divmod(s, m)


def kind(members, m: int) -> str:
    """'single' (one information symbol), 'a' (all share the B block c: a
    sum of A blocks times b_c), 'b' (all share the A block r: a_r times a
    sum of B blocks) or 'gray' (no common block)."""
    if len(members) == 1:
        return "single"
    rows = {rc(s, m)[0] for s in members}
    cols = {rc(s, m)[1] for s in members}
    if len(cols) == 1:
        return "a"
    if len(rows) == 1:
        return "b"
    return "gray"


def gray_ratio(code) -> float:
    """Fraction of the code's non-empty symbols that are gray."""
    m = grid_side(code.kb)
    syms = [d for _, _, d in code.symbols() if len(d) > 0]
    return sum(kind(d, m) == "gray" for d in syms) / len(syms)


def row_blocks(A: np.ndarray, m: int):
    M, K = A.shape
    Mb = -(-M // m)
    out = []
    for r in range(m):
        blk = np.zeros((Mb, K))
        lo, hi = r * Mb, min((r + 1) * Mb, M)
        if hi > lo:
            blk[: hi - lo] = A[lo:hi]
        out.append(blk)
    return out


def col_blocks(B: np.ndarray, m: int):
    K, N = B.shape
    Nb = -(-N // m)
    out = []
    for c in range(m):
        blk = np.zeros((K, Nb))
        lo, hi = c * Nb, min((c + 1) * Nb, N)
        if hi > lo:
            blk[:, : hi - lo] = B[:, lo:hi]
        out.append(blk)
    return out


def coded_products(A: np.ndarray, B: np.ndarray, code, symbols) -> dict:
    """Y_g = sum over s in N(g) of a_r(s) b_c(s), each block product formed
    and the products summed in ascending s (the definition of the symbol)."""
    m = grid_side(code.kb)
    a = row_blocks(np.asarray(A, dtype=np.float64), m)
    b = col_blocks(np.asarray(B, dtype=np.float64), m)
    sym = {g: d for g, _, d in code.symbols()}
    out = {}
    for g in symbols:
        acc = None
        for s in sym[g]:
            r, c = rc(s, m)
            p = a[r] @ b[c]
            acc = p if acc is None else acc + p
        out[g] = acc
    return out


def assemble(X, M: int, N: int, m: int) -> np.ndarray:
    """Place block v_s = X[s] at block row r, block column c; cut padding."""
    rows = [np.concatenate([X[r * m + c] for c in range(m)], axis=1) for r in range(m)]
    return np.concatenate(rows, axis=0)[:M, :N]


def coded_matmul_ref(A: np.ndarray, B: np.ndarray, code, plan) -> np.ndarray:
    """Coded products -> peel -> assemble in the 2-D form, float64."""
    if not plan.decodable:
        raise ValueError("plan is not decodable")
    Y = coded_products(A, B, code, plan.computed)
    X = peel_numeric(Y, plan, code.kb)
    return assemble(X, A.shape[0], B.shape[1], grid_side(code.kb))
