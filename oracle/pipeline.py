"""Numeric pipeline in float64: encode, coded products, peel, uncoded product.

The product is C = A.B with A (M x K) and B (K x N).  This is the paper's
A^T B with the dot-product length s (Sec. II) playing the role of K and the
k*b information symbols becoming k*b row-blocks of A (B is not split).
Block s holds rows [s*Mb, (s+1)*Mb) of A with Mb = ceil(M / (k*b)); rows past
M are zero.

Because every coded symbol is a plain sum of data blocks, (sum_s A_s) B equals
sum_s (A_s B), so peeling the coded products recovers every A_s B exactly in
exact arithmetic: the decoded C equals A.B.  The uncoded product is therefore
the plain definition the pipeline is checked against.
"""

from __future__ import annotations

import numpy as np


def block_rows(M: int, kb: int) -> int:
    """Rows per data block, Mb = ceil(M / kb)."""
    return -(-M // kb)


def data_blocks(A: np.ndarray, kb: int):
    """The kb row-blocks of A as float64 arrays of shape (Mb, K), zero padded."""
    M, K = A.shape
    Mb = block_rows(M, kb)
    out = []
    for s in range(kb):
        blk = np.zeros((Mb, K), dtype=np.float64)
        lo, hi = s * Mb, min((s + 1) * Mb, M)
        if hi > lo:
            blk[: hi - lo] = A[lo:hi]
        out.append(blk)
    return out


def encode(A: np.ndarray, code, symbols) -> dict:
    """Coded blocks C_g = sum over s in N(g) of A_s, summed in ascending s.

    This is the master-side encode of Sec. II with the XOR of Sec. III-A
    read as a real sum (as Table I writes it).
    """
    blocks = data_blocks(np.asarray(A, dtype=np.float64), code.kb)
    sym = {g: d for g, _, d in code.symbols()}
    out = {}
    for g in symbols:
        acc = np.zeros_like(blocks[0])
        for s in sym[g]:
            acc = acc + blocks[s]
        out[g] = acc
    return out


def coded_products(coded: dict, B: np.ndarray) -> dict:
    """Y_g = C_g . B for every coded block (each virtual worker's products)."""
    B64 = np.asarray(B, dtype=np.float64)
    return {g: c @ B64 for g, c in coded.items()}


def peel_numeric(Y: dict, plan, kb: int):
    """Peel the coded products along the plan's schedule.

    In (depth, s) order: X_s = Y_{g_s} - sum over u in N(g_s)\\{s} of X_u,
    the subtraction taken in ascending u.  This is the BP update of Sec. I-A
    with XOR replaced by real subtraction.
    Returns the list of X_s (None where s was not recovered).
    """
    X = [None] * kb
    for s in plan.order():
        acc = Y[plan.releaser[s]].copy()
        for u in plan.sub[s]:
            acc = acc - X[u]
        X[s] = acc
    return X


def assemble(X, M: int) -> np.ndarray:
    """Stack the recovered blocks and cut the padding rows."""
    return np.concatenate(X, axis=0)[:M]


def coded_matmul_ref(A: np.ndarray, B: np.ndarray, code, plan) -> np.ndarray:
    """Encode -> coded products -> peel -> assemble, all in float64."""
    if not plan.decodable:
        raise ValueError("plan is not decodable")
    coded = encode(A, code, plan.computed)
    Y = coded_products(coded, B)
    X = peel_numeric(Y, plan, code.kb)
    return assemble(X, A.shape[0])


def uncoded(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """The plain product A.B in float64."""
    return np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)


def rel_frobenius(X: np.ndarray, R: np.ndarray) -> float:
    """||X - R||_F / ||R||_F."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    den = np.linalg.norm(R)
    return float(np.linalg.norm(X - R) / (den if den > 0 else 1.0))
