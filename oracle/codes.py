"""Code objects of the paper, in plain Python.

A code has ``n`` columns (the paper's compute nodes).  Column ``j`` holds an
ordered list of coded symbols (the node's processors); each symbol is the set
of data blocks it sums, stored as a sorted tuple of data ids in ``[0, k*b)``.
In the paper a symbol is the XOR of the information symbols v_1..v_{bk}
(Sec. III-A, definition of the [n,k,t,b] array BP-XOR code); over the reals
the same incidence structure gives a real-valued sum (Table I writes the
symbols as ``v_1 + v_2``).

Global symbol index ``g``: symbols are numbered column by column, so ``g`` of
the ``i``-th symbol of column ``j`` is the number of symbols in columns
``0..j-1`` plus ``i``.  For an array code this is ``j*b + i``.  For a Mojette
code ``i`` is the bin index of Eq. (moj1) and empty bins keep their index.

Data ids: the paper's information symbols v_1..v_{bk} map to ids 0..bk-1 in
order.  For the Mojette grid f(z, l) with z in [0, b) and l in [0, k)
(Eq. (moj1)) the cell (z, l) is data id ``l*b + z``.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations
from math import ceil, gcd

from .splitmix import SplitMix64


@dataclass
class Code:
    kind: str                 # "array" or "mojette"
    n: int
    k: int
    b: int
    columns: list             # columns[j] = list of symbols (sorted tuples)
    projections: list = field(default_factory=list)   # Mojette (p, q) per column

    @property
    def kb(self) -> int:
        return self.k * self.b

    def col_sizes(self) -> list:
        return [len(c) for c in self.columns]

    def symbols(self):
        """All symbols as (g, column j, data tuple), g ascending."""
        out = []
        g = 0
        for j, col in enumerate(self.columns):
            for sym in col:
                out.append((g, j, sym))
                g += 1
        return out

    def csr(self):
        """(col_ptr, sym_ptr, sym_data) integer arrays of the code."""
        col_ptr = [0]
        sym_ptr = [0]
        sym_data = []
        for col in self.columns:
            for sym in col:
                sym_data.extend(sym)
                sym_ptr.append(len(sym_data))
            col_ptr.append(len(sym_ptr) - 1)
        return col_ptr, sym_ptr, sym_data

    def max_degree(self) -> int:
        return max(len(s) for col in self.columns for s in col)


def _v(*ids):
    """Paper's v_i (1-based) -> sorted tuple of 0-based data ids."""
    return tuple(sorted(i - 1 for i in ids))


def table1() -> Code:
    """The [5,2,.,2] array BP-XOR code with sigma = 2 of Table I (Example 1).

    Rows are processors 1, 2; columns are nodes 1..5.
    """
    cols = [
        [_v(1), _v(2, 3)],
        [_v(2), _v(1, 4)],
        [_v(3), _v(2, 4)],
        [_v(4), _v(1, 3)],
        [_v(1, 2), _v(3, 4)],
    ]
    return Code("array", n=5, k=2, b=2, columns=cols)


def table3() -> Code:
    """The [5,3,2,3] array BP-XOR code with sigma = 2 of Table III (Example 2).

    Rows are processors 1..3; columns are nodes 1..5.
    """
    cols = [
        [_v(1), _v(3, 4), _v(6, 7)],
        [_v(1, 2), _v(4, 5), _v(7, 8)],
        [_v(2, 3), _v(5, 6), _v(8, 9)],
        [_v(7), _v(9, 1), _v(4, 8)],
        [_v(3), _v(2, 6), _v(9, 5)],
    ]
    return Code("array", n=5, k=3, b=3, columns=cols)


def identity(k: int, b: int) -> Code:
    """The uncoded layout: k columns, b symbols each, symbol (j, i) = block j*b+i.

    Not a construction of the paper; it is the trivial code with n = k that
    every comparison against the uncoded product uses.
    """
    cols = [[(j * b + i,) for i in range(b)] for j in range(k)]
    return Code("identity", n=k, k=k, b=b, columns=cols)


# --------------------------------------------------------------------------
# Mojette (projection-geometry) codes, Sec. III-C.
# --------------------------------------------------------------------------

def _u(t: int) -> int:
    """Discrete unit function u(t) of Eq. (moj1): 1 if t > 0 else 0."""
    return 1 if t > 0 else 0


def mojette_bin_count(p: int, q: int, k: int, b: int) -> int:
    """Projection length b_i = |p|(k-1) + |q|(b-1) + 1 (Sec. III-C)."""
    return abs(p) * (k - 1) + abs(q) * (b - 1) + 1


def mojette_column(p: int, q: int, k: int, b: int) -> list:
    """Bins of projection (p, q) over the k x b grid, per Eq. (moj1).

    Cell (z, l) of f, z in [0, b), l in [0, k), lands in the bin whose
    argument m satisfies m + z*q + l*p = 0; the bin is stored at index
    m + (b-1) q u(q) + (k-1) p u(p).  Returns a list of sorted data-id tuples
    indexed by that bin index (empty bins are empty tuples).  The list length
    is taken from the largest index reached, not from the closed form, so
    that the closed form can be checked against it.
    """
    off = (b - 1) * q * _u(q) + (k - 1) * p * _u(p)
    cells = {}
    for z in range(b):
        for l in range(k):
            m = -(z * q + l * p)
            idx = m + off
            if idx < 0:
                raise ValueError("bin index below zero")
            cells.setdefault(idx, []).append(l * b + z)
    size = max(cells) + 1
    return [tuple(sorted(cells.get(i, ()))) for i in range(size)]


def construction_a_p(n: int) -> list:
    """p values of Construction A: -floor((n-1)/2) .. ceil((n-1)/2), q = 1."""
    lo = -((n - 1) // 2)
    hi = -((-(n - 1)) // 2)        # ceil((n-1)/2)
    return list(range(lo, hi + 1))


def _ceil_odd(x: int) -> int:
    """Smallest odd integer >= x (the paper's ceil_odd of Construction B)."""
    return x if x % 2 != 0 else x + 1


def construction_b_p(n: int) -> list:
    """Odd p values of Construction B, ceil_odd(-n+1) .. ceil_odd(n-1)."""
    lo = _ceil_odd(-n + 1)
    hi = _ceil_odd(n - 1)
    return list(range(lo, hi + 1, 2))


def mojette(k: int, b: int, n: int, qe: int = 0) -> Code:
    """Mojette code with n projections over a k x b grid.

    qe = 0: Construction A (q_i = 1, consecutive p_i).
    qe >= 1: Construction B (q_i = 2**qe, odd p_i).
    Projections are listed in ascending p; column i is projection i.
    """
    if qe == 0:
        ps = construction_a_p(n)
        q = 1
    else:
        ps = construction_b_p(n)
        q = 1 << qe
    assert len(ps) == n
    cols = []
    projs = []
    for p in ps:
        assert gcd(p, q) == 1
        cols.append(mojette_column(p, q, k, b))
        projs.append((p, q))
    return Code("mojette", n=n, k=k, b=b, columns=cols, projections=projs)


def mojette_max_degree(p: int, q: int, k: int, b: int) -> int:
    """sigma_i = min(ceil(b/|p|), ceil(k/|q|)) of the degree theorem (Sec. III-C).

    A zero |p| or |q| leaves the other bound alone.
    """
    cands = []
    if p != 0:
        cands.append(ceil(b / abs(p)))
    if q != 0:
        cands.append(ceil(k / abs(q)))
    return min(cands)


def katz(projs, k: int, b: int) -> bool:
    """Katz criterion (Theorem, Sec. III-C): sum|p| >= b or sum|q| >= k."""
    return sum(abs(p) for p, _ in projs) >= b or sum(abs(q) for _, q in projs) >= k


def phi(x: int) -> int:
    """Utility function of Appendix A: floor(x/2) (floor(x/2) + 1), x >= 0."""
    h = x // 2
    return h * (h + 1)


def lemma_a1(t: int) -> float:
    """Lemma A.1: sum of |p| over the t projections of Construction A."""
    return 0.5 * (phi(t) + phi(t - 1)) if t >= 1 else 0.0


def lemma_b1(t: int) -> int:
    """Lemma B.1: sum of |p| over the t projections of Construction B."""
    return (t * t + 1) // 2 if t % 2 else (t * t) // 2


def overhead_direct(code: Code, need: int) -> float:
    """Worst-case coding overhead over every choice of ``need`` columns.

    The overhead eps is defined by b' = (1 + eps) b, b' being the mean column
    length of the columns used, maximised over the column choices (Sec. III-B
    and its footnote).  Column lengths are the paper's bin counts b_i,
    empty bins included.
    """
    sizes = code.col_sizes()
    best = max(sum(sizes[i] for i in c) for c in combinations(range(code.n), need))
    return best / (need * code.b) - 1.0


def overhead_closed_a(n: int, k: int, b: int) -> float:
    """Exact worst-case overhead of Construction A (Appendix A):
    (k-1)/(2kb) (phi(n) + phi(n-1) - phi(n-k) - phi(n-k-1))."""
    return (k - 1) / (2 * k * b) * (phi(n) + phi(n - 1) - phi(n - k) - phi(max(n - k - 1, 0)))


def overhead_direct_total(code: Code, need: int) -> float:
    """Worst-case overhead in symbols: the largest number of bins (empty ones
    included) that any ``need`` columns hold, divided by the k*b data symbols,
    minus one.  This is the normalisation of the exact overhead expression of
    Appendix B, where ``need`` = ceil(k / 2^qe) projections suffice; for
    Construction A (need = k) it equals ``overhead_direct``."""
    sizes = code.col_sizes()
    best = max(sum(sizes[i] for i in c) for c in combinations(range(code.n), need))
    return best / code.kb - 1.0


def construction_b_needed(k: int, qe: int) -> int:
    """Projections that suffice for Construction B by the Katz criterion
    (Appendix B): t 2^qe >= k, i.e. t = ceil(k / 2^qe)."""
    return -(-k // (1 << qe))


def overhead_closed_b(n: int, k: int, b: int, qe: int) -> float:
    """Exact worst-case overhead of Construction B (Appendix B).

    The t = ceil(k/2^qe) columns with the largest |p| hold
    sum (|p_i| (k-1) + 2^qe (b-1) + 1) bins.  Construction B's n odd p values
    contain those of n - t projections as the n - t smallest |p|, so by Lemma
    B.1 the largest t of them sum to L(n) - L(n-t), L being Lemma B.1's sum.
    Hence eps = (2^qe (b-1) t + (k-1) (L(n) - L(n-t)) + t) / (kb) - 1.
    (The printed exact expression of Appendix B writes the |p| sum with the
    phi of Appendix A, which is Construction A's sum, not B's; this function
    takes B's own p set.)
    """
    t = construction_b_needed(k, qe)
    return ((1 << qe) * (b - 1) * t + (k - 1) * (lemma_b1(n) - lemma_b1(n - t)) + t) \
        / (k * b) - 1.0


def overhead_bracket_b(n: int, k: int, b: int, qe: int):
    """Lower and upper bound on Construction B's overhead from the |p|-sum
    bracket of Appendix B, (t2^2 - t1^2 -+ 1)/2 with t2 = n, t1 = n - t."""
    t = construction_b_needed(k, qe)
    base = (1 << qe) * (b - 1) * t + t
    span = n * n - (n - t) ** 2
    return ((base + (k - 1) * (span - 1) / 2) / (k * b) - 1.0,
            (base + (k - 1) * (span + 1) / 2) / (k * b) - 1.0)


def overhead_approx_a(n: int, k: int, b: int) -> float:
    """Large-b approximation of Appendix A: (k-1)(2n-k)/(4b)."""
    return (k - 1) * (2 * n - k) / (4 * b)


# --------------------------------------------------------------------------
# Deterministic array-code search.
# --------------------------------------------------------------------------
# The paper gives array BP-XOR codes only as the two worked tables and as
# existence bounds (Sec. III-A, III-B).  For other (n, k, b) the code is found
# by a deterministic hill-climb whose every random draw comes from SplitMix64,
# so that an independent implementation reproduces the same code bit for bit.

def _random_symbol(rng: SplitMix64, kb: int, sigma: int) -> tuple:
    d = 1 + rng.below(sigma)
    chosen = []
    while len(chosen) < d:
        x = rng.below(kb)
        if x not in chosen:
            chosen.append(x)
    return tuple(sorted(chosen))


def _peel_masks(masks, full):
    """Round-based peel over bit-masks; returns (known mask, rounds)."""
    known = 0
    rounds = 0
    while known != full:
        rel = 0
        for m in masks:
            r = m & ~known
            if r and (r & (r - 1)) == 0:
                rel |= r
        if not rel:
            break
        known |= rel
        rounds += 1
    return known, rounds


def search_objective(cols_masks, k: int, full: int):
    """(U, F, L, D) of a candidate code given per-column lists of symbol masks.

    U = number of k-column subsets that do not peel.
    F = 1 if all n columns together do not peel, else 0.
    L = sum over all k-column subsets of the data ids left unrecovered
        (a smooth measure of how far the failing subsets get).
    D = sum over the peelable k-column subsets of their peeling rounds.
    """
    n = len(cols_masks)
    allm = [m for c in cols_masks for m in c]
    known, _ = _peel_masks(allm, full)
    F = 0 if known == full else 1
    U = 0
    L = 0
    D = 0
    for sub in combinations(range(n), k):
        ms = [m for j in sub for m in cols_masks[j]]
        kn, r = _peel_masks(ms, full)
        if kn == full:
            D += r
        else:
            U += 1
            L += bin(full & ~kn).count("1")
    return U, F, L, D


def array_search(n: int, k: int, b: int, sigma: int, seed: int,
                 restarts: int, iters: int, walk: int = 0) -> Code:
    """Deterministic search for an [n, k, ., b] array BP-XOR code.

    One SplitMix64(seed) stream drives everything.  Each restart draws the
    n*b symbols in ascending g (a symbol: degree 1 + draw mod sigma, then
    distinct data ids by rejection, each id = draw mod kb).  Each iteration
    draws a position g = draw mod (n*b) and a fresh symbol.  Hill-climb
    (walk = 0): the change is kept when the objective (U, F, L, D, S) does
    not get worse (lexicographic; S = total degree; see
    ``search_objective``), and the restart's result is its final code.
    Plateau walk (walk = 1): the change is kept when (U, F) does not get
    worse (U smaller, or U equal and F not larger), and the restart's result
    is the best code it visited by the whole objective (the first one, on
    ties).  The best result over the restarts wins; ties keep the earlier
    restart.
    """
    kb = k * b
    if not (1 <= sigma <= kb) or kb > 64:
        raise ValueError("search supports 1 <= sigma <= kb <= 64")
    full = (1 << kb) - 1
    rng = SplitMix64(seed)
    G = n * b
    best = None
    best_obj = None
    for _ in range(restarts):
        syms = [_random_symbol(rng, kb, sigma) for _ in range(G)]

        def objective(sy):
            masks = [[sum(1 << x for x in sy[j * b + i]) for i in range(b)] for j in range(n)]
            U, F, L, D = search_objective(masks, k, full)
            return (U, F, L, D, sum(len(s) for s in sy))

        cur = objective(syms)
        run_best, run_syms = cur, list(syms)
        for _ in range(iters):
            g = rng.below(G)
            cand = _random_symbol(rng, kb, sigma)
            old = syms[g]
            syms[g] = cand
            obj = objective(syms)
            if walk:
                keep = obj[0] < cur[0] or (obj[0] == cur[0] and obj[1] <= cur[1])
            else:
                keep = obj <= cur
            if keep:
                cur = obj
                if walk and obj < run_best:
                    run_best, run_syms = obj, list(syms)
            else:
                syms[g] = old
        if not walk:
            run_best, run_syms = cur, list(syms)
        if best_obj is None or run_best < best_obj:
            best_obj = run_best
            best = run_syms
    cols = [[best[j * b + i] for i in range(b)] for j in range(n)]
    return Code("array", n=n, k=k, b=b, columns=cols)
