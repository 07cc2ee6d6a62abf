"""Host-side tests of the serving loop's admission policy and memory model
(no GPU: workspace sizes are injected, service times simulated)."""
import numpy as np
import pytest

from paper_2607_23494_amd import serving as S


def test_fifo_admission_with_budget_and_slots():
    adm = S.Admission(budget_bytes=10, slots=2)
    sizes = {0: 6, 1: 6, 2: 3, 3: 11}
    arrivals = [(0.0, 0), (0.1, 1), (0.2, 2), (0.3, 3)]
    service = {0: 1.0, 1: 1.0, 2: 1.0, 3: 1.0}
    out = S.schedule(arrivals, service, sizes, adm)
    assert 3 not in out                      # larger than the whole budget: rejected
    assert out[0] == (0.0, 1.0)
    assert out[1] == (1.0, 2.0)              # waited for memory
    assert out[2] == (1.0, 2.0)              # behind request 1 (first come, first served)
    assert adm.used == 0 and adm.active == 0


def test_slots_bound_concurrency_and_budget_is_never_exceeded():
    rng = np.random.default_rng(0)
    n = 200
    sizes = {i: int(rng.integers(1, 50)) for i in range(n)}
    service = {i: float(rng.uniform(0.1, 2.0)) for i in range(n)}
    arrivals = sorted((float(t), i) for i, t in enumerate(np.cumsum(rng.exponential(0.3, n))))
    adm = S.Admission(budget_bytes=100, slots=3)
    out = S.schedule(arrivals, service, sizes, adm, bypass_age=0.0)
    assert len(out) == n
    events = sorted([(a, +1, i) for i, (a, f) in out.items()] + [(f, -1, i) for i, (a, f) in out.items()],
                    key=lambda e: (e[0], e[1]))
    used = active = 0
    for t, kind, i in events:
        used += kind * sizes[i]
        active += kind
        assert used <= 100 and active <= 3
    arr = dict((i, t) for t, i in arrivals)
    order = sorted(out, key=lambda i: (arr[i], i))
    admits = [out[i][0] for i in order]
    assert all(a >= arr[i] for i, a in zip(order, admits))
    assert admits == sorted(admits)          # strict FIFO preserves arrival order
    # with backfilling the budget and slot bounds still hold
    adm = S.Admission(budget_bytes=100, slots=3)
    out2 = S.schedule(arrivals, service, sizes, adm, bypass_age=2.0)
    assert len(out2) == n
    events = sorted([(a, +1, i) for i, (a, f) in out2.items()] + [(f, -1, i) for i, (a, f) in out2.items()],
                    key=lambda e: (e[0], e[1]))
    used = active = 0
    for t, kind, i in events:
        used += kind * sizes[i]
        active += kind
        assert used <= 100 and active <= 3
    mean_wait = lambda o: np.mean([o[i][0] - arr[i] for i in o])
    assert mean_wait(out2) <= mean_wait(out)


def test_backfill_passes_a_blocked_head_until_its_age_bound():
    sizes = {0: 8, 1: 8, 2: 2, 3: 2, 4: 2}
    service = {0: 1.0, 1: 1.0, 2: 0.3, 3: 0.3, 4: 0.3}
    # 0 runs; 1 cannot fit beside it; 2 arrives and fits in the gap
    arrivals = [(0.0, 0), (0.1, 1), (0.2, 2), (0.9, 3), (0.95, 4)]
    fifo = S.schedule(arrivals, service, sizes, S.Admission(10, 4), bypass_age=0.0)
    assert fifo[2][0] == pytest.approx(1.0)                 # strict FIFO: behind request 1
    bf = S.schedule(arrivals, service, sizes, S.Admission(10, 4), bypass_age=0.5)
    assert bf[2][0] == pytest.approx(0.2)                   # passes the blocked head at once
    assert bf[1][0] == pytest.approx(1.0)                   # the head still starts when 0 ends
    # requests 3 and 4 arrive after the head has waited 0.8 s > 0.5 s: no more bypassing
    assert bf[3][0] >= bf[1][0] and bf[4][0] >= bf[1][0]
    never = S.schedule(arrivals, service, sizes, S.Admission(10, 4), bypass_age=5.0)
    assert never[3][0] == pytest.approx(0.9)                # within the bound they pass too


def test_admission_misuse_is_an_error():
    adm = S.Admission(10, 1)
    adm.admit(5)
    assert not adm.fits(1)                   # slot taken
    with pytest.raises(RuntimeError):
        adm.admit(1)
    adm.release(5)
    with pytest.raises(RuntimeError):
        adm.release(5)
    with pytest.raises(ValueError):
        S.Admission(0, 1)


def test_memory_model_counts_field_and_largest_workspace():
    pos = np.zeros((1000, 3), np.float32)
    req = S.Request(0, pos, 100.0, 64, {"xi": {"edges": np.linspace(1, 10, 11)},
                                        "zeta": {"edges": np.linspace(1, 10, 5), "l_max": 2}})
    ws = {"xi": 1000, "zeta": 5000, "assign": 3000}
    b = S.request_bytes(req, lambda k, n, p: ws[k])
    base = 1000 * 12 + 64 ** 3 * 4 + S.field_bytes(64)
    assert b == base + 5000 + 10 * 8 + 3 * 4 * 4 * 8
    req.weight = np.ones(1000, np.float32)
    assert S.request_bytes(req, lambda k, n, p: ws[k]) == b + 4000
    ws["assign"] = 9000                      # the larger of assignment and statistics
    assert S.request_bytes(req, lambda k, n, p: ws[k]) == b + 4000 + 4000


def test_workload_and_arrivals_are_seeded():
    a = S.make_workload(6, seed=5, grids=(32,), n_pts_range=(1e3, 1e4))
    b = S.make_workload(6, seed=5, grids=(32,), n_pts_range=(1e3, 1e4))
    assert [r.stats.keys() for r in a] == [r.stats.keys() for r in b]
    assert all(np.array_equal(x.pos, y.pos) for x, y in zip(a, b))
    S.poisson_arrivals(a, rate=10.0, seed=1)
    t = [r.arrival for r in a]
    assert t == sorted(t) and t[0] > 0
