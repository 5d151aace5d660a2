"""The host library used from several threads at once (CPU only): distinct
code and plan handles built concurrently give the same results as one
thread, a shared plan is read concurrently, and each thread's error message
is its own.  ctypes releases the interpreter lock for every library call,
so the calls do overlap."""
import threading

import numpy as np
import pytest

bpx = pytest.importorskip("paper_1904_11563_amd.bpx")
from paper_1904_11563_amd import inputs  # noqa: E402  (seeded generators only)

N_THREADS = 8


def _work(seed):
    """One thread's job: a searched code, a Mojette code, and plans over
    several arrival orders; returns everything it built as plain data."""
    out = []
    code = bpx.Code.search(12, 8, 4, 4, seed, 1, 300)
    out.append(code.columns())
    moj = bpx.Code.mojette(16, 8, 24, seed % 2)
    out.append(moj.columns())
    for a in range(6):
        perm, _ = inputs.shifted_exp_arrival(100 * seed + a, 12)
        plan = bpx.Plan(code, list(perm), 0, bpx.MODE_STRAGGLER, 4096, 256, 512, bpx.PREC_F32)
        inf = plan.info()
        prog = plan.peel_program()
        out.append((inf, prog["steps"].tolist(), prog["subs"].tolist(), prog["n_slots"],
                    plan.schedule()["computed"].tolist()))
    return out


def _run_threads(fn, args):
    results = [None] * len(args)
    errors = []

    def body(i):
        try:
            results[i] = fn(args[i])
        except Exception as e:  # reported after the join
            errors.append((i, repr(e)))

    ts = [threading.Thread(target=body, args=(i,)) for i in range(len(args))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
    return results


def test_distinct_handles_concurrently_match_serial():
    seeds = list(range(N_THREADS))
    serial = [_work(s) for s in seeds]
    for _ in range(3):
        assert _run_threads(_work, seeds) == serial


def test_shared_plan_read_concurrently():
    code = bpx.Code.mojette(8, 4, 12, 1)
    perm, _ = inputs.erasure_arrival(3, 12, 4)
    plan = bpx.Plan(code, list(perm), 4, bpx.MODE_ERASURE, 8192, 512, 1024, bpx.PREC_F32)
    want = (plan.info(), plan.peel_program()["steps"].tolist(),
            plan.schedule()["computed"].tolist())

    def read(_):
        got = []
        for _ in range(50):
            got.append((plan.info(), plan.peel_program()["steps"].tolist(),
                        plan.schedule()["computed"].tolist()))
        return got

    for res in _run_threads(read, list(range(N_THREADS))):
        assert all(g == want for g in res)


def test_error_messages_are_per_thread():
    code = bpx.Code.table1()

    def fail_or_pass(i):
        msgs = []
        for _ in range(200):
            if i % 2:
                # an arrival order that is not a permutation
                try:
                    bpx.Plan(code, [0, 1, 2, 3, 3], 1, bpx.MODE_ERASURE, 64, 64, 64,
                             bpx.PREC_F32)
                    msgs.append("no error")
                except bpx.BpxError as e:
                    msgs.append(str(e))
            else:
                # a negative dimension
                try:
                    bpx.Plan(code, [0, 1, 2, 3, 4], 1, bpx.MODE_ERASURE, 64, 64, -5,
                             bpx.PREC_F32)
                    msgs.append("no error")
                except bpx.BpxError as e:
                    msgs.append(str(e))
        return msgs

    res = _run_threads(fail_or_pass, list(range(N_THREADS)))
    for i, msgs in enumerate(res):
        assert len(set(msgs)) == 1, (i, set(msgs))
    odd = {res[i][0] for i in range(1, N_THREADS, 2)}
    even = {res[i][0] for i in range(0, N_THREADS, 2)}
    assert odd == {"bpx status -1: arrival is not a permutation of the columns"}
    assert even == {"bpx status -1: bad shape or precision"}
