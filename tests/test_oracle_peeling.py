"""Pins of the oracle's peeling decoder, prefix and schedule."""
from itertools import combinations, permutations

import numpy as np
import pytest

from oracle import codes
from oracle.peeling import (ERASURE, FULL, MIN, STRAGGLER, make_plan, peel,
                            peel_one_at_a_time)
from oracle.splitmix import SplitMix64


def _random_code(rng, n, k, b, sigma):
    kb = k * b
    cols = []
    for _ in range(n):
        col = []
        for _ in range(b):
            d = 1 + rng.below(sigma)
            s = set()
            while len(s) < d:
                s.add(rng.below(kb))
            col.append(tuple(sorted(s)))
        cols.append(col)
    return codes.Code("array", n, k, b, cols)


def _gf2_rank(rows, ncols):
    """Rank over GF(2) of a list of 0/1 integer bit-rows (Gaussian elimination)."""
    rows = list(rows)
    rank = 0
    for bit in range(ncols):
        piv = None
        for i in range(rank, len(rows)):
            if rows[i] >> bit & 1:
                piv = i
                break
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and rows[i] >> bit & 1:
                rows[i] ^= rows[rank]
        rank += 1
    return rank


CODES = [codes.table1(), codes.table3(), codes.mojette(3, 4, 5, 0),
         codes.mojette(4, 3, 6, 1)]


def _random_codes(count=30):
    rng = SplitMix64(1234)
    out = []
    for i in range(count):
        n, k, b, sig = [(6, 4, 2, 3), (5, 3, 3, 2), (8, 5, 2, 4), (4, 2, 4, 3)][i % 4]
        out.append(_random_code(rng, n, k, b, sig))
    return out


def test_confluence():
    # Peeling reaches the same recovered set whatever the release order: the
    # round-based peeler and a one-at-a-time peeler (last candidate first)
    # must agree on every column subset.
    for c in CODES + _random_codes():
        syms_all = c.symbols()
        for t in range(1, c.n + 1):
            for sub in combinations(range(c.n), t):
                syms = [(g, d) for g, j, d in syms_all if j in sub]
                rel, _ = peel(syms, c.kb)
                assert set(rel) == peel_one_at_a_time(syms, c.kb)


def test_peel_success_implies_gf2_full_rank():
    # A BP-decodable set of XOR equations is triangular after a permutation,
    # hence has full rank over GF(2).
    for c in CODES + _random_codes():
        syms_all = c.symbols()
        for t in range(1, c.n + 1):
            for sub in combinations(range(c.n), t):
                syms = [(g, d) for g, j, d in syms_all if j in sub and d]
                rel, _ = peel(syms, c.kb)
                if len(rel) == c.kb:
                    rows = [sum(1 << x for x in d) for _, d in syms]
                    assert _gf2_rank(rows, c.kb) == c.kb


def _xor_decode(c, plan, data):
    """Decode random words with XOR along the plan: the paper's own symbols."""
    sym = {g: d for g, _, d in c.symbols()}
    coded = {}
    for g in plan.computed:
        w = 0
        for s in sym[g]:
            w ^= data[s]
        coded[g] = w
    X = [None] * c.kb
    for s in plan.order():
        w = coded[plan.releaser[s]]
        for u in plan.sub[s]:
            assert X[u] is not None          # subtrahend known before use
            w ^= X[u]
        X[s] = w
    return X


def test_schedule_xor_decodes_exactly():
    rng = SplitMix64(99)
    for c in CODES + _random_codes():
        for trial in range(8):
            arrival = list(range(c.n))
            for i in range(c.n - 1, 0, -1):
                j = rng.below(i + 1)
                arrival[i], arrival[j] = arrival[j], arrival[i]
            for mode in (STRAGGLER, FULL, MIN):
                plan = make_plan(c, arrival, 0, mode)
                if not plan.decodable:
                    continue
                data = [rng.next() for _ in range(c.kb)]
                assert _xor_decode(c, plan, data) == data


def test_schedule_structure():
    for c in CODES + _random_codes():
        sym = {g: d for g, _, d in c.symbols()}
        plan = make_plan(c, list(range(c.n)), 0, FULL)
        for s in range(c.kb):
            g = plan.releaser[s]
            if g < 0:
                continue
            assert set(sym[g]) == set(plan.sub[s]) | {s}
            for u in plan.sub[s]:
                assert plan.depth[u] < plan.depth[s]
            if plan.depth[s] > 1:
                # the chain is tight: some subtrahend was released one round earlier
                assert max(plan.depth[u] for u in plan.sub[s]) == plan.depth[s] - 1
        assert list(plan.computed) == sorted(g for g, d in sym.items() if d)


def test_prefix_is_shortest():
    rng = SplitMix64(5)
    for c in CODES + _random_codes():
        arrival = list(range(c.n))
        for i in range(c.n - 1, 0, -1):
            j = rng.below(i + 1)
            arrival[i], arrival[j] = arrival[j], arrival[i]
        plan = make_plan(c, arrival, 0, STRAGGLER)
        if not plan.decodable:
            continue
        m = plan.prefix_m
        syms = lambda cols: [(g, d) for g, j, d in c.symbols() if j in set(cols)]
        assert len(peel(syms(arrival[:m]), c.kb)[0]) == c.kb
        if m > 1:
            assert len(peel(syms(arrival[: m - 1]), c.kb)[0]) < c.kb
        expect = sorted(g for g, j, d in c.symbols() if j in set(arrival[:m]) and d)
        assert plan.computed == expect


def test_table1_every_pair_in_erasure_mode():
    c = codes.table1()
    for pair in permutations(range(5), 2):
        rest = [j for j in range(5) if j not in pair]
        plan = make_plan(c, list(pair) + rest, 3, ERASURE)
        assert plan.decodable and plan.prefix_m == 2


def test_erasure_undecodable_reports_unrecovered():
    c = codes.table3()
    # two columns cannot carry 9 unknowns
    plan = make_plan(c, [0, 1, 2, 3, 4], 3, ERASURE)
    assert not plan.decodable
    assert plan.prefix_m == 2
    assert len(plan.unrecovered) > 0
    assert all(plan.releaser[s] < 0 for s in plan.unrecovered)


def test_table3_depth_reaches_nine():
    # Columns 1..3 of Table III hold the chain v1, v1+v2, ..., v8+v9: decoded
    # from them alone the chain is released one id per round.
    c = codes.table3()
    plan = make_plan(c, [0, 1, 2, 3, 4], 2, ERASURE)
    assert plan.decodable and plan.prefix_m == 3
    assert plan.max_depth == 9


def test_min_mode_computes_releasers_only():
    c = codes.table3()
    plan = make_plan(c, [4, 3, 0, 1, 2], 0, MIN)
    assert plan.decodable
    assert plan.computed == sorted(set(plan.releaser))


# ------------------------------------------------- hand-worked schedules --

def _golden_code(name):
    from conftest import K3B1_COLUMNS
    if name == "table1":
        return codes.table1()
    if name == "table3":
        return codes.table3()
    assert name == "k3b1"
    return codes.Code("array", n=4, k=3, b=1, columns=K3B1_COLUMNS)


_MODES = {"erasure": ERASURE, "straggler": STRAGGLER, "full": FULL, "min": MIN}


@pytest.mark.parametrize("case", [c["name"] for c in __import__("conftest").load_release_tables()])
def test_release_schedule_matches_hand_worked_table(case):
    # tests/golden/release_tables.txt: releaser and depth of every id worked
    # out by hand with the canonical (degree, g) release rule (Sec. I-A's BP
    # leaves the choice open); two of the cases have several candidates for
    # one id in the same round, one of them of different degrees.
    from conftest import load_release_tables
    c = [x for x in load_release_tables() if x["name"] == case][0]
    code = _golden_code(c["code"])
    plan = make_plan(code, c["arrival"], c["n_lost"], _MODES[c["mode"]])
    assert plan.decodable and plan.prefix_m == c["prefix_m"]
    for s, (g, d) in c["release"].items():
        assert (plan.releaser[s], plan.depth[s]) == (g, d), (case, s)
    assert len(c["release"]) == code.kb


def test_release_rule_prefers_low_degree_then_low_g():
    # the same rule on bare symbol lists: an id with candidates of degrees 3
    # and 2 takes the degree-2 one; equal degrees take the smaller g
    rel, dep = peel([(0, (0,)), (1, (1,)), (2, (0, 1, 2)), (3, (1, 2))], 3)
    assert rel == {0: 0, 1: 1, 2: 3} and dep == {0: 1, 1: 1, 2: 2}
    rel, _ = peel([(5, (0,)), (7, (0, 1)), (9, (0, 1))], 2)
    assert rel == {0: 5, 1: 7}
