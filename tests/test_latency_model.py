"""The latency model (T = T_e + min over decodable sets of max T_i + T_d,
Sec. II) against order statistics it must reproduce with exponential task
times (Sec. IV-A): the uncoded case waits for the slowest of kb processors,
E = H_kb / mu; Table I's code decodes from any 2 of its 5 columns, so the
cluster term is the 2nd order statistic of 5 column times, each the maximum
of its b = 2 processors.  Host-only: plans, no device."""
import numpy as np
import pytest

from paper_1904_11563_amd import latency

bpx = pytest.importorskip("paper_1904_11563_amd.bpx")


def _mean_se(xs):
    xs = np.asarray(xs, dtype=np.float64)
    return xs.mean(), xs.std(ddof=1) / np.sqrt(len(xs))


def test_uncoded_is_the_maximum_of_kb_exponentials():
    k, b = 4, 2
    code = bpx.Code.identity(k, b)
    smp = latency.sample(bpx, code, 64, 8, 8, 1.0, None, samples=3000, seed=1)
    m, se = _mean_se([s.t_cluster for s in smp])
    H = sum(1.0 / j for j in range(1, k * b + 1))
    assert abs(m - H) < 4 * se
    assert all(s.prefix_m == k for s in smp)
    assert all(s.t_decode == 0.0 and s.t_encode == 0.0 for s in smp)


def test_table1_any_two_of_five_columns():
    code = bpx.Code.table1()
    smp = latency.sample(bpx, code, 40, 8, 8, 1.0, None, samples=3000, seed=2)
    assert all(s.prefix_m == 2 for s in smp)
    m, se = _mean_se([s.t_cluster for s in smp])
    # P(T_(2:5) > t) = (1-G)^5 + 5 G (1-G)^4 with G(t) = (1 - e^-t)^2
    t = np.linspace(0.0, 40.0, 400001)
    G = (1.0 - np.exp(-t)) ** 2
    tail = (1 - G) ** 5 + 5 * G * (1 - G) ** 4
    expect = np.trapezoid(tail, t) if hasattr(np, "trapezoid") else np.trapz(tail, t)
    assert abs(m - expect) < 4 * se


def test_decode_term_is_peel_bytes_over_bandwidth():
    code = bpx.Code.table3()
    M, K, N = 90, 16, 12
    smp = latency.sample(bpx, code, M, K, N, 2.0, 1e9, samples=50, seed=3, mu=0.5)
    for s in smp:
        assert s.t_decode >= 0.0
    # one fixed order: recompute the plan and its bytes by hand
    order = np.array([0, 1, 2, 3, 4], dtype=np.int32)
    plan = bpx.Plan(code, order, 0, bpx.MODE_STRAGGLER, M, K, N)
    rd, wr = latency.peel_bytes(plan, M, N)
    sch = plan.schedule()
    Mb = plan.info()["Mb"]
    n_written = int((np.asarray([sch["dest"][list(sch["computed"]).index(g)]
                                 for g in sch["releaser"]]) >= 0).sum())
    assert wr == n_written * Mb * N * 4
    assert rd >= wr
    summ = latency.summary(smp)
    assert summ["samples"] == 50 and summ["E_T"] >= summ["cluster"]
