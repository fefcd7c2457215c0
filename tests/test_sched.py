"""Admission policy of the serving loop, on the CPU: dh_sched_select driven by
a virtual clock with a fake executor (running jobs share the device's rate
equally). Checks the budget and slot limits at every event, completion of
every job, the head-of-line wait limit, and that backfill lowers latency
against one-at-a-time FIFO on the same arrivals."""
import heapq

import numpy as np
import pytest


@pytest.fixture(scope="module")
def dh():
    import paper_1808_01478_amd as dh
    return dh


def simulate(dh, arrivals, need, work, budget, slots, limit, rate=1.0, by_work=False):
    """Event-driven processor-sharing simulation; returns per-job (start, end)
    and a log of (time, used_bytes, running). by_work passes the jobs' work to
    the policy (shortest work first)."""
    n = len(arrivals)
    start = np.full(n, np.nan)
    end = np.full(n, np.nan)
    remaining = np.array(work, float)
    queue, running, log = [], set(), []
    used = 0
    t = 0.0
    next_arrival = 0
    while next_arrival < n or queue or running:
        # admit
        if queue and len(running) < slots:
            waited = [t - arrivals[q] for q in queue]
            pick = dh.sched_select([need[q] for q in queue], waited, budget - used,
                                   slots - len(running), limit,
                                   [work[q] for q in queue] if by_work else None)
            chosen = [queue[k] for k in pick]
            for q in chosen:
                queue.remove(q)
                running.add(q)
                start[q] = t
                used += need[q]
        log.append((t, used, len(running)))
        # next event: an arrival or the first completion under sharing
        share = rate / max(1, len(running))
        t_done = min((remaining[q] / share for q in running), default=np.inf)
        t_arr = arrivals[next_arrival] - t if next_arrival < n else np.inf
        dt = min(t_done, t_arr)
        assert np.isfinite(dt), "deadlock: nothing running, nothing arriving, queue stuck"
        for q in running:
            remaining[q] -= dt * share
        t += dt
        for q in [q for q in running if remaining[q] <= 1e-12]:
            running.remove(q)
            end[q] = t
            used -= need[q]
        while next_arrival < n and arrivals[next_arrival] <= t + 1e-15:
            queue.append(next_arrival)
            next_arrival += 1
    return start, end, log


def trace(seed, n=300):
    rng = np.random.Generator(np.random.PCG64(seed))
    arrivals = np.cumsum(rng.exponential(0.5, size=n))
    size = np.exp(rng.uniform(np.log(1e3), np.log(2e6), size=n))
    need = (size * 64).astype(np.int64)            # bytes ~ points
    work = (size / 1e5) ** 2                        # pairs ~ N^2
    return arrivals, need, work


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("slots,budget", [(4, 64 << 20), (4, 160 << 20), (2, 1 << 40), (1, 1 << 40)])
def test_limits_and_completion(dh, seed, slots, budget):
    arrivals, need, work = trace(seed)
    need = np.minimum(need, budget)                 # every job fits alone
    start, end, log = simulate(dh, arrivals, need, work, budget, slots, limit=2.0)
    assert np.all(np.isfinite(end)), "some job never finished"
    assert np.all(start >= arrivals - 1e-12)
    for _, used, running in log:
        assert used <= budget and running <= slots


def test_head_wait_limit_stops_backfill(dh):
    # a huge job at the head cannot fit while small ones run; once it has
    # waited past the limit, nothing behind it may start before it
    budget = 100
    arrivals = np.array([0.0, 0.01] + list(0.02 + 0.05 * np.arange(40)))
    need = np.array([60, 70] + [20] * 40)
    work = np.array([1.0, 5.0] + [0.2] * 40)
    limit = 0.5
    start, end, _ = simulate(dh, arrivals, need, work, budget, slots=4, limit=limit)
    big = 1
    assert np.all(np.isfinite(end))
    for q in range(2, len(arrivals)):
        if arrivals[q] > arrivals[big] and start[q] > arrivals[big] + limit + 1e-9:
            assert start[q] >= start[big] - 1e-12, f"job {q} jumped the starving head"


def test_backfill_beats_fifo(dh):
    arrivals, need, work = trace(7)
    budget = 1 << 40
    _, end_c, _ = simulate(dh, arrivals, need, work, budget, slots=4, limit=2.0)
    _, end_f, _ = simulate(dh, arrivals, need, work, budget, slots=1, limit=2.0)
    lat_c = np.percentile(end_c - arrivals, 50)
    lat_f = np.percentile(end_f - arrivals, 50)
    assert lat_c < lat_f, (lat_c, lat_f)


def test_select_edge_cases(dh):
    assert dh.sched_select([], [], 100, 4, 1.0) == []
    assert dh.sched_select([10], [0.0], 100, 0, 1.0) == []
    assert dh.sched_select([10, 10, 10], [0, 0, 0], 100, 2, 1.0) == [0, 1]
    assert dh.sched_select([200, 10], [0.5, 0.1], 100, 4, 1.0) == [1]
    assert dh.sched_select([200, 10], [1.5, 0.1], 100, 4, 1.0) == []
    assert dh.sched_select([30, 40, 50], [0, 0, 0], 100, 4, 1.0) == [0, 1]


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("slots", [1, 2])
def test_shortest_work_first_lowers_latency(dh, seed, slots):
    """With jobs queueing (few slots, offered load below one), admitting the
    least work first lowers mean and median latency against arrival order;
    the worst latency grows by at most the wait limit."""
    arrivals, need, work = trace(seed)
    budget, limit, rate = 1 << 40, 10.0, 80.0
    _, end_a, _ = simulate(dh, arrivals, need, work, budget, slots, limit, rate)
    start, end_w, log = simulate(dh, arrivals, need, work, budget, slots, limit, rate,
                                 by_work=True)
    assert np.all(np.isfinite(end_w)) and np.all(start >= arrivals - 1e-12)
    assert all(running <= slots for _, _, running in log)
    lat_a, lat_w = end_a - arrivals, end_w - arrivals
    assert lat_w.mean() < 0.95 * lat_a.mean()
    assert np.percentile(lat_w, 50) <= np.percentile(lat_a, 50)
    assert lat_w.max() <= lat_a.max() + limit


def test_wait_limit_bounds_passing_over(dh):
    """Shortest work first: a large job is passed over by smaller ones only
    until it has waited the limit; after that no job arriving later starts
    before it."""
    arrivals = np.array([0.0] + list(0.01 + 0.02 * np.arange(200)))
    need = np.array([10] * 201)
    work = np.array([50.0] + [0.05] * 200)
    limit = 0.5
    start, end, _ = simulate(dh, arrivals, need, work, 1000, slots=1, limit=limit,
                             by_work=True)
    assert np.all(np.isfinite(end))
    big = 0
    assert start[big] <= arrivals[big] + limit + 0.05 + 1e-9     # one small job's length late at most
    for q in range(1, len(arrivals)):
        if start[q] > arrivals[big] + limit + 0.05 + 1e-9:
            assert start[q] >= start[big] - 1e-12, f"job {q} jumped the large job past its limit"


def test_select_by_work(dh):
    assert dh.sched_select([10, 10, 10], [0, 0, 0], 100, 2, 1.0, work=[5.0, 1.0, 3.0]) == [1, 2]
    # a job past the limit goes first whatever its work
    assert dh.sched_select([10, 10, 10], [0, 2.0, 0], 100, 1, 1.0, work=[1.0, 9.0, 2.0]) == [1]
    # and one that does not fit stops everything
    assert dh.sched_select([10, 500, 10], [0, 2.0, 0], 100, 3, 1.0, work=[1.0, 9.0, 2.0]) == []
