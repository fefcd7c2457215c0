"""The serving loop on the GPU: every job's result in a concurrent mix is
bit-identical to the same job run alone (same kernels, integer sums), also
when the jobs' work items share pair-kernel launches (continuous batching),
binary64 jobs equal the oracle, jobs drawn as the serving workload draws
them equal the oracle (binary64) or lie within the binary32 edge bound, jobs
of the serving workload's full sizes are exact, the budget bounds the admitted footprints, and bad jobs fail
alone."""
import math
import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def job_mix(seed=21, n_jobs=18, n_hi=12_000):
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for j in range(n_jobs):
        job = workloads.serving_job(rng, j, 0.0, n_lo=200, n_hi=n_hi, bins=(1000, 10_000, 50_000))
        prec = int(rng.integers(0, 2))
        jobs.append((job.frame, prec))
    return jobs


def alone(frame, prec):
    import paper_1808_01478_amd as dh
    return dh.histo(frame.coords, frame.offsets, frame.box_type, frame.box, frame.r_max,
                    frame.n_bins, prec)


def alone_with_oor(frame, prec):
    """(histograms, out-of-range counts) of one dh_histo_async call."""
    import paper_1808_01478_amd as dh
    from gpu_util import run_gpu
    with dh.Context(0) as ctx:
        return run_gpu(ctx, frame, prec)


def test_mix_equals_alone_and_oracle():
    import paper_1808_01478_amd as dh
    jobs = job_mix()
    print(f"\n[case] serving mix of {len(jobs)} jobs", flush=True)
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=4) as srv:
        ids = [srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, p)
               for f, p in jobs]
        results = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["max_running"] >= 2, st          # jobs did overlap
    for (f, p), (h, oor, times) in zip(jobs, results):
        ref, ref_oor = alone_with_oor(f, p)
        assert np.array_equal(h, ref), f"{f.name} prec={p}: mix differs from alone"
        assert np.array_equal(oor, ref_oor), f"{f.name} prec={p}: out-of-range differs"
        assert times[2] >= times[1] >= 0 and times[0] >= 0
    for (f, p), (h, _, _) in list(zip(jobs, results))[:6]:
        if p == 1:
            assert np.array_equal(h, oracle.frame_histogram(f).hist), f.name


def test_serving_workload_jobs_against_oracle():
    """Jobs drawn exactly as the measured serving workload draws them (seed 5:
    50 warm-up jobs, then the measured ones; N log-uniform in [1e3, 2e6], no
    box, orthorhombic or triclinic, 1-3 species, 1k/10k/50k bins): the
    measured jobs of at most 30,000 points among the first 120, each served in
    binary32 (the workload's precision) and binary64, all at once. binary64
    equals the oracle bit for bit; binary32 lies within the edge-pair bound of
    the oracle, histograms and out-of-range counts."""
    import paper_1808_01478_amd as dh
    from gpu_util import fp32_bound_violations, oor_bound_violations
    rng = np.random.Generator(np.random.PCG64(5))
    drawn = [workloads.serving_job(rng, j, 0.0).frame for j in range(50 + 120)]
    jobs = [f for f in drawn[50:] if f.n <= 30_000]
    assert len(jobs) >= 40
    print(f"\n[case] serving workload: {len(jobs)} measured jobs of at most 30,000 points, "
          f"both precisions", flush=True)
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=8) as srv:
        ids = [(srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, 0),
                srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, 1))
               for f in jobs]
        res = [(srv.wait(a), srv.wait(b)) for a, b in ids]
        st = srv.stats()
    assert st["completed"] == 2 * len(jobs) and st["failed"] == 0
    for f, ((h32, o32, _), (h64, o64, _)) in zip(jobs, res):
        w = oracle.edge_window(f.coords, f.box, f.r_max)
        ref = oracle.frame_histogram(f, edge_window=w)
        assert np.array_equal(h64, ref.hist), f"{f.name}: binary64 differs from the oracle"
        assert np.array_equal(o64, ref.out_of_range), f"{f.name}: binary64 out-of-range"
        bad = fp32_bound_violations(h32, ref.hist, ref.edges)
        bad += oor_bound_violations(o32, ref.out_of_range, ref.edges)
        assert not bad, f"{f.name}: " + "; ".join(bad[:5])


def test_budget_back_pressure():
    import paper_1808_01478_amd as dh
    jobs = job_mix(seed=22, n_jobs=10, n_hi=30_000)
    # footprint of the largest job, plus a little: at most one or two run at once
    probe = []
    with dh.Server(0, hbm_budget_bytes=1 << 40, max_inflight=1) as s1:
        for f, p in jobs:
            probe.append(s1.wait(s1.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max,
                                           f.n_bins, p))[0])
    def footprint(f, p):
        # coordinates, staged copy, histograms, out-of-range and pair counts
        return f.n * 24 + f.n * (32 if p else 16) + f.n_hist * f.n_bins * 8 + 2 * f.n_hist * 8
    sizes = [footprint(f, p) for f, p in jobs]
    budget = int(max(sizes) * 1.2)
    with dh.Server(0, hbm_budget_bytes=budget, max_inflight=4, head_wait_limit_s=0.05) as srv:
        ids = [srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, p)
               for f, p in jobs]
        got = [srv.wait(i)[0] for i in ids]
        st = srv.stats()
    assert st["peak_bytes"] <= budget
    for a, b in zip(got, probe):
        assert np.array_equal(a, b)


def test_bad_jobs_fail_alone():
    import paper_1808_01478_amd as dh
    f = workloads.random_frame(601, [500, 300], workloads.BOX_ORTHO, n_bins=100)
    # the small job needs about 40 kB, the big one about 11.6 MB (coordinates,
    # staged copy, histogram): an 8 MB budget admits one and refuses the other
    with dh.Server(0, hbm_budget_bytes=8 << 20, max_inflight=2) as srv:
        good = srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, 0)
        with pytest.raises(dh.DisthistError) as e:
            srv.submit(f.coords, f.offsets, f.box_type, f.box, -1.0, f.n_bins, 0)
        assert e.value.code == -1
        big = workloads.random_frame(602, [200_000], workloads.BOX_NONE, n_bins=10)
        with pytest.raises(dh.DisthistError) as e:
            srv.submit(big.coords, big.offsets, 0, None, big.r_max, 50_000, 1)
        assert e.value.code == -4                   # larger than the whole budget
        h, _, _ = srv.wait(good)
        assert np.array_equal(h, alone(f, 0))
        assert srv.status(12345) == -1


def test_poisson_arrivals_overlap():
    """Jobs arriving while others run are admitted and finish; latency is
    measured from submission."""
    import paper_1808_01478_amd as dh
    jobs = job_mix(seed=23, n_jobs=12, n_hi=40_000)
    rng = np.random.Generator(np.random.PCG64(5))
    gaps = rng.exponential(0.002, size=len(jobs))
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=4) as srv:
        ids = []
        for (f, p), g in zip(jobs, gaps):
            time.sleep(g)
            ids.append(srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, p))
        res = [srv.wait(i) for i in ids]
    for (f, p), (h, _, t) in zip(jobs, res):
        assert np.array_equal(h, alone(f, p))
        assert math.isfinite(t[2]) and t[2] > 0


def test_small_job_overtakes_huge_job():
    """A job submitted while a huge one runs starts at the huge job's next
    launch boundary and finishes long before it (bounded launches)."""
    import paper_1808_01478_amd as dh
    huge = workloads.random_frame(611, [1_000_000], workloads.BOX_NONE, n_bins=1000)
    small = workloads.random_frame(612, [3000, 1000], workloads.BOX_ORTHO, n_bins=1000)
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=4) as srv:
        warm = srv.submit(small.coords, small.offsets, small.box_type, small.box, small.r_max,
                          small.n_bins, 0)
        srv.wait(warm)
        big = srv.submit(huge.coords, huge.offsets, huge.box_type, huge.box, huge.r_max,
                         huge.n_bins, 0)
        t0 = time.perf_counter()
        while srv.status(big) == dh.JOB_QUEUED and time.perf_counter() - t0 < 5.0:
            time.sleep(0.001)
        time.sleep(0.02)
        sid = srv.submit(small.coords, small.offsets, small.box_type, small.box, small.r_max,
                         small.n_bins, 0)
        h, _, t_small = srv.wait(sid)
        still_running = srv.status(big) == dh.JOB_RUNNING
        hb, _, t_big = srv.wait(big)
    assert np.array_equal(h, alone(small, 0))
    assert int(hb.sum()) <= huge.total_pairs()
    print(f"\nsmall job {t_small[2] * 1e3:.1f} ms, huge job {t_big[2] * 1e3:.1f} ms", flush=True)
    assert still_running, "the small job waited for the whole huge job"
    assert t_small[2] < 0.25 * t_big[2]


@pytest.mark.parametrize("policy", ["shortest", "arrival"])
def test_launch_order_policy(policy):
    """Two slots, a huge job running and a small one submitted behind it:
    least-work-first computes the small job at the huge job's next launch
    boundary; arrival order runs the huge job's launches first, so the small
    job finishes after it. Results are the same either way."""
    import paper_1808_01478_amd as dh
    huge = workloads.random_frame(621, [1_200_000], workloads.BOX_NONE, n_bins=1000)
    small = workloads.random_frame(622, [2000, 1000], workloads.BOX_ORTHO, n_bins=1000)
    pol = dh.SCHED_SHORTEST if policy == "shortest" else dh.SCHED_ARRIVAL
    print(f"\n[case] policy {policy}", flush=True)
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=2, policy=pol) as srv:
        with pytest.raises(dh.DisthistError):
            srv.set_policy(7)
        srv.wait(srv.submit(small.coords, small.offsets, small.box_type, small.box, small.r_max,
                            small.n_bins, 0))
        t0 = time.perf_counter()
        big = srv.submit(huge.coords, huge.offsets, huge.box_type, huge.box, huge.r_max,
                         huge.n_bins, 0)
        while srv.status(big) == dh.JOB_QUEUED and time.perf_counter() - t0 < 5.0:
            time.sleep(0.001)
        time.sleep(0.02)
        t_sub = time.perf_counter() - t0
        sid = srv.submit(small.coords, small.offsets, small.box_type, small.box, small.r_max,
                         small.n_bins, 0)
        h, _, t_small = srv.wait(sid)
        hb, _, t_big = srv.wait(big)
    assert np.array_equal(h, alone(small, 0))
    assert np.array_equal(hb, alone(huge, 0))
    end_small, end_big = t_sub + t_small[2], t_big[2]
    print(f"small job ends at {end_small * 1e3:.1f} ms, huge job at {end_big * 1e3:.1f} ms",
          flush=True)
    if policy == "shortest":
        assert end_small < 0.5 * end_big
    else:
        # (the small kernel may run beside the huge job's last launch)
        assert end_small >= 0.8 * end_big


def test_job_admitted_mid_run_shares_a_launch():
    """A small job submitted while a large one of the same kind runs joins
    the next launch (continuous batching: the launch carries work items of
    both frames), and both results equal their runs alone, out-of-range
    counts included."""
    import paper_1808_01478_amd as dh
    big = workloads.random_frame(631, [600_000, 300_000], workloads.BOX_ORTHO,
                                 box=workloads.ortho_box(80.0, 84.0, 88.0), r_max=30.0,
                                 n_bins=4000)
    small = workloads.random_frame(632, [3000, 1500], workloads.BOX_ORTHO,
                                   box=workloads.ortho_box(12.0, 13.0, 14.0), r_max=6.0,
                                   n_bins=1000)
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=4) as srv:
        b = srv.submit(big.coords, big.offsets, big.box_type, big.box, big.r_max, big.n_bins, 0)
        t0 = time.perf_counter()
        while srv.status(b) == dh.JOB_QUEUED and time.perf_counter() - t0 < 5.0:
            time.sleep(0.001)
        time.sleep(0.03)
        sid = srv.submit(small.coords, small.offsets, small.box_type, small.box, small.r_max,
                         small.n_bins, 0)
        hs, os_, _ = srv.wait(sid)
        still_running = srv.status(b) == dh.JOB_RUNNING
        hb, ob, _ = srv.wait(b)
        st = srv.stats()
    print(f"\n[case] launches {st['launches']}, shared {st['shared_launches']}, "
          f"most jobs in one launch {st['max_jobs_per_launch']}", flush=True)
    assert still_running, "the small job waited for the whole large job"
    assert st["shared_launches"] >= 1 and st["max_jobs_per_launch"] >= 2, st
    ref_s, ref_so = alone_with_oor(small, 0)
    ref_b, ref_bo = alone_with_oor(big, 0)
    assert np.array_equal(hs, ref_s) and np.array_equal(os_, ref_so)
    assert np.array_equal(hb, ref_b) and np.array_equal(ob, ref_bo)


def test_serving_workload_sizes():
    """Jobs of the serving workload's sizes in one server: a 2,000,000-point
    triclinic job with 50,000 bins (two bin windows), a 1,000,000-point job
    without a box, an orthorhombic job, and small ones, submitted at once and
    sharing launches; each equals its run alone (histograms and out-of-range
    counts), and the binary64 job of 150,000 points equals the oracle."""
    import paper_1808_01478_amd as dh
    rng = np.random.Generator(np.random.PCG64(641))
    vol = 2_000_000 / workloads.DENSITY
    tric_box = workloads.random_triclinic_cell(rng, vol)
    jobs = [
        (workloads.random_frame(642, [1_000_000, 600_000, 400_000], workloads.BOX_TRICLINIC,
                                box=tric_box, r_max=0.49 * workloads.min_width(tric_box),
                                n_bins=50_000), 0),
        (workloads.random_frame(643, [1_000_000], workloads.BOX_NONE,
                                extent=(1_000_000 / workloads.DENSITY) ** (1 / 3),
                                n_bins=10_000), 0),
        (workloads.random_frame(644, [90_000, 60_000], workloads.BOX_ORTHO,
                                box=workloads.ortho_box(40.0, 44.0, 48.0), r_max=20.0,
                                n_bins=1000), 1),
    ]
    jobs += [(f, int(p)) for f, p in job_mix(seed=645, n_jobs=6, n_hi=50_000)]
    print(f"\n[case] serving sizes: {[f.n for f, _ in jobs]}", flush=True)
    with dh.Server(0, hbm_budget_bytes=8 << 30, max_inflight=8) as srv:
        ids = [srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, p)
               for f, p in jobs]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    print(f"[case] launches {st['launches']}, shared {st['shared_launches']}", flush=True)
    for (f, p), (h, o, _) in zip(jobs, res):
        print(f"[case] alone {f.name} N={f.n} bins={f.n_bins} prec={p}", flush=True)
        ref_h, ref_o = alone_with_oor(f, p)
        assert np.array_equal(h, ref_h), f"{f.name}: served differs from alone"
        assert np.array_equal(o, ref_o), f"{f.name}: out-of-range differs from alone"
    f, p = jobs[2]
    print(f"[case] oracle {f.name} N={f.n}", flush=True)
    ref = oracle.frame_histogram(f)
    assert np.array_equal(res[2][0], ref.hist) and np.array_equal(res[2][1], ref.out_of_range)
