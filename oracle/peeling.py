"""BP (peeling) decoding, arrival prefix and release schedule.

The decoder of Sec. I-A: all information nodes start empty; a coded node with
exactly one unknown neighbour releases that neighbour; the released value is
removed from every coded node it touches; this repeats until every
information node is known (success) or no coded node has exactly one unknown
neighbour left (failure).

The paper does not fix the order in which simultaneous releases happen.  This
oracle takes the release in rounds: in round r every symbol whose residual
(its data ids minus those already known) has exactly one element is a
candidate; each data id released in round r takes as its releaser the
candidate with the smallest (degree, g) among those whose residual is that id;
all ids released in round r become known together.  The round index is the
id's depth, which is the length of the longest chain of releases behind it.

Modes (which columns are computed and decoded):
  ERASURE   - the first n - n_lost columns of the arrival order exist; the
              decoder uses the shortest arrival prefix of them that peels.
  STRAGGLER - every column arrives; the shortest peelable prefix is used.
  FULL      - every column is computed and the schedule uses all of them.
  MIN       - as STRAGGLER, but only the releasers are computed.
Time of arrival is the paper's min over decodable subsets of the max worker
time (Eq. (1)); with a fixed arrival order the shortest peelable prefix is
exactly the first moment a decodable set is complete, because peeling success
can only grow as symbols are added.
"""

from __future__ import annotations

from dataclasses import dataclass

ERASURE, STRAGGLER, FULL, MIN = 0, 1, 2, 3


def peel(symbols, kb: int):
    """Round-based peeling.

    symbols: iterable of (g, data tuple); empty tuples are ignored.
    Returns (rel, depth): dicts mapping each recovered data id to its
    releaser g and to its round.
    """
    syms = [(g, frozenset(d)) for g, d in symbols if len(d) > 0]
    rel = {}
    depth = {}
    r = 0
    while len(rel) < kb:
        r += 1
        best = {}
        for g, d in syms:
            res = d.difference(rel.keys())
            if len(res) == 1:
                (s,) = tuple(res)
                key = (len(d), g)
                if s not in best or key < best[s]:
                    best[s] = key
        if not best:
            break
        for s, (_, g) in best.items():
            rel[s] = g
            depth[s] = r
    return rel, depth


def peel_one_at_a_time(symbols, kb: int) -> set:
    """A second peeler used only to check confluence: it releases one data id
    at a time, always taking the last symbol (largest g) that has a single
    unknown id, and returns the set of recovered ids."""
    syms = [(g, set(d)) for g, d in symbols if len(d) > 0]
    known = set()
    while True:
        found = None
        for g, d in reversed(syms):
            res = d - known
            if len(res) == 1:
                found = next(iter(res))
                break
        if found is None:
            return known
        known.add(found)


@dataclass
class Plan:
    decodable: bool
    prefix_m: int             # number of arrival-order columns used
    computed: list            # computed symbol ids g (non-empty), ascending
    releaser: list            # per data id s: g_s, or -1 if not recovered
    depth: list               # per data id s: round, or 0 if not recovered
    sub: list                 # per data id s: sorted tuple N(g_s) \ {s}
    unrecovered: list         # data ids not recovered (empty if decodable)

    @property
    def max_depth(self) -> int:
        return max(self.depth) if self.depth else 0

    def order(self) -> list:
        """Recovered data ids in (depth, s) order: the peel's execution order."""
        return sorted((s for s in range(len(self.releaser)) if self.releaser[s] >= 0),
                      key=lambda s: (self.depth[s], s))


def _column_symbols(code, cols):
    syms = code.symbols()
    allowed = set(cols)
    return [(g, d) for g, j, d in syms if j in allowed and len(d) > 0]


def make_plan(code, arrival, n_lost: int, mode: int) -> Plan:
    """Arrival prefix and release schedule for one arrival pattern.

    arrival: a permutation of the column ids, earliest first.
    """
    n = code.n
    kb = code.kb
    if sorted(arrival) != list(range(n)):
        raise ValueError("arrival must be a permutation of the columns")
    if mode == ERASURE:
        if not 0 <= n_lost <= n:
            raise ValueError("n_lost out of range")
        n_avail = n - n_lost
    else:
        n_avail = n

    if mode == FULL:
        m = n
        syms = _column_symbols(code, arrival)
        rel, dep = peel(syms, kb)
        ok = len(rel) == kb
    else:
        ok = False
        m = 0
        rel, dep, syms = {}, {}, []
        for m in range(1, n_avail + 1):
            syms = _column_symbols(code, arrival[:m])
            rel, dep = peel(syms, kb)
            if len(rel) == kb:
                ok = True
                break
        if not ok:
            m = n_avail
            syms = _column_symbols(code, arrival[:m])
            rel, dep = peel(syms, kb)

    sym_of = {g: d for g, d in syms}
    releaser = [rel.get(s, -1) for s in range(kb)]
    depth = [dep.get(s, 0) for s in range(kb)]
    sub = [tuple(sorted(x for x in sym_of[releaser[s]] if x != s)) if releaser[s] >= 0 else ()
           for s in range(kb)]
    if mode == MIN and ok:
        computed = sorted(set(releaser))
    else:
        computed = sorted(sym_of.keys())
    unrec = [s for s in range(kb) if releaser[s] < 0]
    return Plan(ok, m, computed, releaser, depth, sub, unrec)
