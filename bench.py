#!/usr/bin/env python3
"""Throughput of the pair-distance histogram on one MI355X.

One step is one full pass of the hot path over one frame already resident in
HBM: stage the binary64 coordinates (convert / wrap / pad), zero the output,
run the pair kernel (distances, minimum image, binning into LDS
sub-histograms, flush to uint64, out-of-range counts).

Default workload (the largest single-frame one): N = 1,000,000 clustered
points in the triclinic cell a=(50,0,0), b=(15,48,0), c=(10,12,45), species
50/30/20 % (6 histograms), r_max = 22, 20,000 bins, 499,999,500,000 pairs per
step. The headline value is binary32; the binary64 rate is reported beside
it, and the 100,000-point orthorhombic frame as a sub-object.

Prints ONE JSON line. Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# algorithmic FLOPs per pair of the canonical op sequence (add, sub, mul,
# sqrt, rint, min: 1; fma: 2)
FLOPS_PER_PAIR = {0: 10, 1: 22, 2: 34, 3: 268}
# an image of the search costs 3 adds, mul + 2 fma (8 FLOPs) and a minimum;
# the canonical search adds 26 images to the 34 FLOPs of the reduced pair
IMAGE_FLOPS = 9
SEARCH_FLOPS = 26 * IMAGE_FLOPS
PEAK_TFLOPS = {0: 157.3, 1: 78.6}        # MI355X vector FP32 / FP64
KERNEL_NAME = "pairs_kernel"


DESCRIPTIONS = {
    "ortho100k": "ortho100k: N=100,000 uniform, species 60,000/40,000, periodic cube L=40, "
                 "r_max=20, 10,000 bins",
    "tiny": "tiny: N=5,000 uniform in [0,10)^3, 1 species, no box, r_max=10*sqrt(3), 1,000 bins",
    "triclinic1M": "triclinic1M: N=1,000,000 clustered, species 50/30/20 %, cell a=(50,0,0) "
                   "b=(15,48,0) c=(10,12,45), r_max=22, 20,000 bins",
}


def workload_desc(name: str) -> str:
    return DESCRIPTIONS[name]


def workload(name: str):
    if name == "ortho100k":
        return workloads.ortho(), DESCRIPTIONS[name]
    if name == "tiny":
        return workloads.tiny(), DESCRIPTIONS[name]
    if name == "triclinic1M":
        return workloads.triclinic(), DESCRIPTIONS[name]
    raise SystemExit(f"unknown workload {name}")


def box_kind(frame) -> int:
    if frame.box_type != 2:
        return frame.box_type
    return 3 if 2 * frame.r_max >= workloads.min_width(frame.box) * (1 - 1e-9) else 2


def kernel_source_hash() -> str:
    """Hash of the device code (the kernel file and its shared header) with
    comments and whitespace removed: counters taken on other code are stale."""
    import re
    h = hashlib.sha256()
    for f in ("dh_kernels.hip", "dh_internal.h"):
        with open(os.path.join(ROOT, "paper_1808_01478_amd", "csrc", f)) as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", "", code, flags=re.S)
        code = re.sub(r"//[^\n]*", "", code)
        h.update(re.sub(r"\s+", "", code).encode())
    return h.hexdigest()[:16]


def traffic_for(workload_name: str, precision: int, launches_bytes_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
        rec = t.get(f"{workload_name}/{'fp64' if precision else 'fp32'}")
        if not rec or rec.get("source_hash") != kernel_source_hash():
            return None
        return float(rec["hbm_bytes_per_launch"])
    except Exception:
        return None


def progress(what: str):
    """One line per bench section on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {what}", file=sys.stderr, flush=True)


def time_path(ctx, frame, precision, steps, warmup):
    import torch
    dev = torch.device("cuda")
    x = torch.from_numpy(frame.coords).to(dev)
    out = torch.empty((frame.n_hist, frame.n_bins), dtype=torch.int64, device=dev)
    oor = torch.empty((frame.n_hist,), dtype=torch.int64, device=dev)

    def step():
        ctx.histo_async(x, frame.offsets, frame.box_type, frame.box, frame.r_max, frame.n_bins,
                        precision, out, oor)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    start = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    end = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        start[k].record()
        step()
        end[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = ctx.profile_read()
    ctx.profile(False)
    step_ms = sorted(s.elapsed_time(e) for s, e in zip(start, end))
    counts = out.cpu().numpy().view(np.uint64)
    oor_h = oor.cpu().numpy().view(np.uint64)
    return {
        "hist": counts,
        "oor": oor_h,
        "wall_s": t1 - t0,
        "kernel_ms_avg": kern_ms / max(1, launches),
        "launches": launches,
        "step_ms_p50": float(np.percentile(step_ms, 50)),
        "step_ms_p99": float(np.percentile(step_ms, 99)),
    }


def time_host_buffers(frame, precision, steps):
    """Synchronous dh_histo from host memory: the host-to-device copy of the
    coordinates, the whole path and the copy of the histograms back."""
    import paper_1808_01478_amd as dh
    args = (frame.coords, frame.offsets, frame.box_type, frame.box, frame.r_max, frame.n_bins,
            precision)
    dh.histo(*args)
    t0 = time.perf_counter()
    for _ in range(steps):
        h = dh.histo(*args)
    t1 = time.perf_counter()
    assert int(h.sum()) <= frame.total_pairs()
    return {"value": frame.total_pairs() * steps / (t1 - t0), "unit": "pairs/s",
            "steps": steps, "ms_per_step": (t1 - t0) * 1e3 / steps}


def bench_wide(frame, bins=(250_000, 1_000_000, 4_000_000), steps=3):
    """Histograms wider than LDS on the bench frame, binary32: LDS bin windows
    against uint64 global atomics, and which one the default shape takes."""
    import torch
    import paper_1808_01478_amd as dh
    dev = torch.device("cuda")
    x = torch.from_numpy(frame.coords).to(dev)
    rows = []
    with dh.Context(0) as c:
        for nb in bins:
            out = torch.empty((frame.n_hist, nb), dtype=torch.int64, device=dev)
            row = {"n_bins": nb}
            for label, knobs in (("default", None), ("lds_windows", 0), ("global_atomics", 1)):
                if knobs is None:
                    c.set_config(None)
                else:
                    c.set_config(dict(r=8, copies=1, tj=256, noclamp=1, occ_cap=0,
                                      items_per_wg=8, threads=0, wide=knobs))
                args = (x, frame.offsets, frame.box_type, frame.box, frame.r_max, nb, dh.FP32, out)
                c.histo_async(*args)
                torch.cuda.synchronize()
                c.profile(True)
                for _ in range(steps):
                    c.histo_async(*args)
                ms, n = c.profile_read()
                c.profile(False)
                cfg = c.last_config()
                row[label] = {"kernel_ms": ms / n, "pairs_per_s": frame.total_pairs() / (ms / n * 1e-3),
                              "mode": ["lds", "lds_windows", "global_atomics"][cfg["mode"]],
                              "windows": cfg["sweeps"], "threads": cfg["threads"]}
            rows.append(row)
        c.set_config(None)
    return {"workload": "ortho100k frame with wider histograms, binary32", "rows": rows}


def bench_image_search(steps=3):
    """A triclinic frame whose cut-off exceeds half the smallest cell width,
    so the 27-image search runs: 200,000 uniform points (density of the bench
    frame), species 120,000/80,000, r_max = 0.8 of the smallest width,
    4,000 bins."""
    import torch
    import paper_1808_01478_amd as dh
    fr = workloads.image_search()
    x, box, offs, r_max, n = fr.coords, fr.box, list(fr.offsets), fr.r_max, fr.n
    pairs = n * (n - 1) // 2
    out = {"workload": "image search: 200,000 uniform points in a skewed triclinic cell, "
                       "species 120,000/80,000, r_max = 0.8 of the smallest width, 4,000 bins",
           "pairs": pairs,
           "flops": f"{FLOPS_PER_PAIR[2]} per pair (Eq. 5 reduction, root, scale) plus "
                    f"{IMAGE_FLOPS} per image evaluated by the search (the kernel counts the "
                    "searched pairs and the images it evaluated for them: only the images "
                    "of each vector's octant list); canonical_search_flops counts all 26 "
                    "images of every searched pair instead"}
    xt = torch.from_numpy(x).cuda()
    h = torch.empty((3, 4000), dtype=torch.int64, device="cuda")
    with dh.Context(0) as c:
        for prec, name in ((dh.FP32, "fp32"), (dh.FP64, "fp64")):
            c.histo_async(xt, offs, dh.BOX_TRICLINIC, box, r_max, 4000, prec, h)
            torch.cuda.synchronize()
            c.profile(True)
            for _ in range(steps):
                c.histo_async(xt, offs, dh.BOX_TRICLINIC, box, r_max, 4000, prec, h)
            ms, k = c.profile_read()
            c.profile(False)
            torch.cuda.synchronize()
            searched = c.searched_pairs()
            images = c.searched_images()
            ms /= k
            flops = pairs * FLOPS_PER_PAIR[2] + images * IMAGE_FLOPS
            ach = flops / (ms * 1e-3) / 1e12
            canon = (pairs * FLOPS_PER_PAIR[2] + searched * SEARCH_FLOPS) / (ms * 1e-3) / 1e12
            out[name] = {"kernel_ms": ms, "pairs_per_s": pairs / (ms * 1e-3),
                         "searched_pairs": searched, "searched_frac": searched / pairs,
                         "images_per_searched_pair": images / max(1, searched),
                         "achieved_tflops": ach, "roofline_frac": ach / PEAK_TFLOPS[prec],
                         "canonical_search_flops": {"achieved_tflops": canon,
                                                    "roofline_frac": canon / PEAK_TFLOPS[prec]}}
    return out


def bench_trajectory_file(ctx, n_frames: int = 48, interval: int = 8):
    """The trajectory engine on a file: n_frames frames of 100,000 uniform
    points (species 60,000/40,000) in orthorhombic cells that breathe by up to
    2 % around the bench cube, r_max = 20, 10,000 bins, binary32, histograms
    summed over intervals of `interval` frames; time from the call to the last
    record written, file reads and copies included."""
    import tempfile
    from paper_1808_01478_amd import trajfile
    import paper_1808_01478_amd as dh
    rng = np.random.Generator(np.random.PCG64(77))
    n, L = 100_000, 40.0
    xs, boxes = [], []
    for f in range(n_frames):
        e = L * (1.0 + 0.02 * np.sin(0.3 * f) * np.array([1.0, 0.7, -0.5]))
        boxes.append(workloads.ortho_box(*e))
        xs.append(rng.uniform(0.0, 1.0, size=(n, 3)) * e)
    d = tempfile.mkdtemp(prefix="dh_traj_")
    path, res = os.path.join(d, "bench.dhtraj"), os.path.join(d, "bench.dhres")
    trajfile.write_trajectory(path, xs, workloads.BOX_ORTHO, boxes)
    del xs
    offs = [0, 60_000, n]
    pairs = n * (n - 1) // 2 * n_frames
    threads = len(os.sched_getaffinity(0))
    with dh.Trajectory(path) as t:
        # warm-up on the first interval (kernel loading), then the timed run
        t.histo(ctx, offs, 20.0, 10_000, dh.FP32, res + ".warm", interval=interval,
                frame_end=interval)
        t0 = time.perf_counter()
        done = t.histo(ctx, offs, 20.0, 10_000, dh.FP32, res, interval=interval)
        wall = time.perf_counter() - t0
        # the same with a CPU worker on the host's threads beside the GPU
        t0 = time.perf_counter()
        done_h, cpu_frames = t.histo_hybrid(ctx, offs, 20.0, 10_000, dh.FP32, res + ".hyb",
                                            threads - 1 if threads > 1 else 1, interval=interval)
        wall_h = time.perf_counter() - t0
    for q in (path, res, res + ".warm", res + ".hyb"):
        os.remove(q)
    os.rmdir(d)
    return {"workload": f"trajectory file: {n_frames} frames of 100,000 points in breathing "
                        f"orthorhombic cells, r_max 20, 10,000 bins, binary32, sums over "
                        f"{interval}-frame intervals", "intervals": done,
            "value": pairs / wall, "unit": "pairs/s", "ms_per_frame": wall * 1e3 / n_frames,
            "hybrid_cpu_worker": {"value": pairs / wall_h, "unit": "pairs/s",
                                  "intervals": done_h, "frames_on_cpu": cpu_frames,
                                  "cpu_threads": threads - 1 if threads > 1 else 1}}


def bench_trajectory(ctx, n_frames: int, steps: int):
    """The trajectory workload (512 orthorhombic frames, N log-uniform in
    [1e4, 2e5], 1-4 species, 4,096 bins) in binary32: one batched graph
    replay per step against one dh_histo_async call per frame."""
    import torch
    import paper_1808_01478_amd as dh
    frames = workloads.trajectory(n_frames)
    dev = torch.device("cuda")
    bufs = []
    for f in frames:
        bufs.append({"d_coords": torch.from_numpy(f.coords).to(dev), "offsets": f.offsets,
                     "box_type": f.box_type, "box": f.box, "r_max": f.r_max, "n_bins": f.n_bins,
                     "d_out": torch.empty((f.n_hist, f.n_bins), dtype=torch.int64, device=dev)})
    pairs = sum(f.total_pairs() for f in frames)
    batch = dh.Batch(ctx, bufs, dh.FP32, graph=True)
    batch.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.launch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    snap = [b["d_out"].clone() for b in bufs]

    def per_frame():
        for f, b in zip(frames, bufs):
            ctx.histo_async(b["d_coords"], f.offsets, f.box_type, f.box, f.r_max, f.n_bins,
                            dh.FP32, b["d_out"])
    per_frame()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        per_frame()
    torch.cuda.synchronize()
    t_frames = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a, b["d_out"]) for a, b in zip(snap, bufs))
    info = batch.info()
    batch.close()
    return {
        "workload": f"trajectory: {n_frames} orthorhombic frames, N log-uniform [1e4, 2e5], "
                    "1-4 species, r_max = half the shortest edge, 4,096 bins, binary32",
        "pairs_per_run": pairs,
        "batched_graph": {"value": pairs / t_batch, "unit": "pairs/s", "ms_per_run": t_batch * 1e3,
                          "items": info["items"], "pair_launches": info["launches"]},
        "per_frame_launches": {"value": pairs / t_frames, "unit": "pairs/s",
                               "ms_per_run": t_frames * 1e3, "launches": n_frames},
        "speedup": t_frames / t_batch,
        "identical_results": bool(same),
        "identical_results_frames": len(bufs),
    }


def run_trace(server_args, frames, gaps, progress: str = ""):
    """Submits frames at the given inter-arrival gaps (seconds) to a new
    server; returns per-job latencies and the makespan. With progress set,
    prints a line to stderr every 250 completed jobs."""
    import threading
    import paper_1808_01478_amd as dh
    with dh.Server(0, **server_args) as srv:
        ids, t_sub = [None] * len(frames), [0.0] * len(frames)
        submitted = [threading.Event() for _ in frames]
        failure = []
        t0 = time.perf_counter()

        def client():
            t_next = t0
            try:
                for k, (f, g) in enumerate(zip(frames, gaps)):
                    t_next += g
                    delay = t_next - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    t_sub[k] = time.perf_counter() - t0
                    ids[k] = srv.submit(f.coords, f.offsets, f.box_type, f.box, f.r_max,
                                        f.n_bins, dh.FP32)
                    submitted[k].set()
            except BaseException as e:  # the waits below must not block on it
                failure.append(e)
                for ev in submitted:
                    ev.set()
        th = threading.Thread(target=client)
        th.start()
        # wait for each job as soon as it is submitted, in submission order
        lat = []
        for k in range(len(frames)):
            submitted[k].wait()
            if failure:
                break
            _, _, times = srv.wait(ids[k])
            lat.append(times[2])
            if progress and (k + 1) % 250 == 0:
                print(f"[serving] {progress}: {k + 1} jobs done", file=sys.stderr, flush=True)
        th.join()
        if failure:
            raise failure[0]
        st = srv.stats()
    end = max(t + l for t, l in zip(t_sub, lat))
    return np.array(lat), end, st


GOLDEN = {"triclinic1M": os.path.join(ROOT, "tests", "golden", "triclinic1M.npz")}


def check_against_golden(name, frame, r32, r64):
    """The step's histograms against the oracle's stored full-size result
    (written by tests/golden/make_golden.py from the oracle alone): binary64
    bit for bit, binary32 within the per-edge bound. None when no stored
    result exists for the workload or it was made from other input bytes."""
    path = GOLDEN.get(name)
    if path is None or not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from golden.make_golden import input_hash
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    if str(g["input_sha256"][0]) != input_hash(frame):
        return {"against": os.path.relpath(path, ROOT), "input_matches": False}
    out = {"against": os.path.relpath(path, ROOT), "input_matches": True}
    if r64 is not None:
        out["fp64_bit_exact"] = bool(np.array_equal(r64["hist"], g["hist"]) and
                                     np.array_equal(r64["oor"], g["oor"]))
    worst, ok = 0, True
    for h in range(frame.n_hist):
        d = np.abs(np.cumsum(r32["hist"][h].astype(np.int64)) -
                   np.cumsum(g["hist"][h].astype(np.int64)))
        e = g["edges"][h].astype(np.int64)
        ok &= bool((d <= e).all())
        worst = max(worst, int(d.max()))
        ok &= abs(int(r32["oor"][h]) - int(g["oor"][h])) <= int(e[-1])
    out["fp32_within_edge_bound"] = ok
    out["fp32_max_cumulative_difference"] = worst
    out["edge_pairs"] = int(g["edges"].sum())
    return out


def bench_frame(ctx, name: str, steps: int, fp64_steps: int, warmup: int, frame=None):
    """One single-frame workload in binary32 and binary64: pairs/s over the
    timed steps' wall clock, the pair kernel's HIP-event average and its FLOP
    roofline fraction."""
    import paper_1808_01478_amd as dh
    fr, desc = workload(name) if frame is None else (frame, workload_desc(name))
    frame = fr
    kind = box_kind(frame)
    pairs = frame.total_pairs()
    out = {"workload": desc, "pairs_per_step": pairs, "flops_per_pair": FLOPS_PER_PAIR[kind]}
    res = {}
    for prec, key, k in ((dh.FP32, "fp32", steps), (dh.FP64, "fp64", fp64_steps)):
        if k <= 0:
            continue
        progress(f"{name} {key}, {k} steps")
        r = time_path(ctx, frame, prec, k, warmup if prec == dh.FP32 else 1)
        res[key] = r
        ach = pairs * FLOPS_PER_PAIR[kind] / (r["kernel_ms_avg"] * 1e-3) / 1e12
        out[key] = {"value": pairs * k / r["wall_s"], "unit": "pairs/s", "steps": k,
                    "ms_per_step": r["wall_s"] * 1e3 / k, "kernel_ms_avg": r["kernel_ms_avg"],
                    "achieved_tflops": ach, "roofline_frac": ach / PEAK_TFLOPS[prec],
                    "launch_shape": ctx.last_config(),
                    "latency_ms": {"p50": r["step_ms_p50"], "p99": r["step_ms_p99"]}}
    return frame, out, res


def serving_frames(n_jobs: int, n_warm: int, seed: int = 5):
    rng = np.random.Generator(np.random.PCG64(seed))
    frames = [workloads.serving_job(rng, j, 0.0).frame for j in range(n_warm + n_jobs)]
    return frames[:n_warm], frames[n_warm:]


def batched_rate(frames):
    """The batched path (dh_batch: all frames planned once, one persistent
    launch per class of frames) on the same frames, binary32: pairs/s and
    jobs/s of one run, frames already resident."""
    import torch
    import paper_1808_01478_amd as dh
    dev = torch.device("cuda")
    bufs = [{"d_coords": torch.from_numpy(f.coords).to(dev), "offsets": f.offsets,
             "box_type": f.box_type, "box": f.box, "r_max": f.r_max, "n_bins": f.n_bins,
             "d_out": torch.empty((f.n_hist, f.n_bins), dtype=torch.int64, device=dev)}
            for f in frames]
    with dh.Context(0) as ctx:
        batch = dh.Batch(ctx, bufs, dh.FP32, graph=False)
        batch.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.launch()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        batch.close()
    pairs = sum(f.total_pairs() for f in frames)
    del bufs
    torch.cuda.empty_cache()
    return {"pairs_per_s": pairs / dt, "jobs_per_s": len(frames) / dt, "seconds": dt}


def bench_serving(n_jobs: int, n_warm: int = 50, n_capacity: int = 200, seed: int = 5,
                  load: float = 0.75, slots: int = 8):
    """Histogram jobs with N log-uniform in [1e3, 2e6], box none/orthorhombic/
    triclinic, 1-3 species, 1k/10k/50k bins, binary32, Poisson arrivals at
    `load` times the saturated job rate C of the batched path on the same
    mix (measured on the first n_capacity jobs, which also run saturated
    through the server), n_jobs measured jobs after n_warm warm-up jobs:
    the server's default (continuous batching, `slots` resident jobs, least
    remaining work first) with an 8 GiB and a 256 MiB HBM budget, against
    one job at a time in arrival order (FIFO), on the same arrivals."""
    import paper_1808_01478_amd as dh
    warm, frames = serving_frames(n_jobs, n_warm, seed)
    pairs = sum(f.total_pairs() for f in frames)
    cont = {"hbm_budget_bytes": 8 << 30, "max_inflight": slots}
    fifo = {"hbm_budget_bytes": 8 << 30, "max_inflight": 1, "policy": dh.SCHED_ARRIVAL}
    run_trace(cont, warm, [0.0] * len(warm))
    cap_frames = frames[:n_capacity]
    batched = batched_rate(cap_frames)
    progress(f"serving: batched path {batched['jobs_per_s']:.1f} jobs/s")
    cap_pairs = sum(f.total_pairs() for f in cap_frames)
    _, sat_end, sat_st = run_trace(cont, cap_frames, [0.0] * len(cap_frames))
    capacity = batched["jobs_per_s"]
    lam = load * capacity
    gaps = np.random.Generator(np.random.PCG64(seed * 100)).exponential(1.0 / lam, size=n_jobs)
    out = {"workload": f"serving: {n_jobs} jobs after {n_warm} warm-up jobs, N log-uniform "
                       "[1e3, 2e6], box none/ortho/triclinic, 1-3 species, bins 1k/10k/50k, "
                       f"binary32, Poisson arrivals at {load} of the batched path's job rate",
           "pairs": pairs, "load": load, "arrival_rate_per_s": lam,
           "saturated": {"jobs": len(cap_frames),
                         "batched_path": batched,
                         "server": {"pairs_per_s": cap_pairs / sat_end,
                                    "jobs_per_s": len(cap_frames) / sat_end,
                                    "launches": sat_st["launches"],
                                    "shared_launches": sat_st["shared_launches"]},
                         "server_vs_batched": (cap_pairs / sat_end) / batched["pairs_per_s"]}}
    runs = (("continuous_batching", cont), ("continuous_batching_256MiB",
                                            dict(cont, hbm_budget_bytes=256 << 20)),
            ("fifo_one_at_a_time", fifo))
    for name, args in runs:
        progress(f"serving: {name}, {n_jobs} jobs")
        lat, end, st = run_trace(args, frames, gaps, progress=name)
        out[name] = {"p50_ms": float(np.percentile(lat, 50) * 1e3),
                     "p90_ms": float(np.percentile(lat, 90) * 1e3),
                     "p99_ms": float(np.percentile(lat, 99) * 1e3),
                     "throughput_pairs_per_s": pairs / end, "jobs_per_s": n_jobs / end,
                     "budget_bytes": args["hbm_budget_bytes"], "slots": args["max_inflight"],
                     "max_running": st["max_running"], "peak_bytes": st["peak_bytes"],
                     "launches": st["launches"], "shared_launches": st["shared_launches"],
                     "max_jobs_per_launch": st["max_jobs_per_launch"]}
    return out


def bench_serving_sweep(policy: str, n_jobs: int = 1000, n_warm: int = 50, seed: int = 5,
                        loads=(0.25, 0.5, 0.75, 0.9), n_capacity: int = 200, slots: int = 8):
    """The full serving protocol for one policy: n_warm warm-up jobs, then
    n_jobs measured jobs (N log-uniform in [1e3, 2e6], box none/orthorhombic/
    triclinic, 1-3 species, 1k/10k/50k bins, binary32) at Poisson arrival
    rates of each load times the saturated job rate C of the batched path
    (measured on the first n_capacity jobs), with an 8 GiB budget; for the
    default policy also one run at 0.75 with a 256 MiB budget (admission
    back-pressure). policy: "shortest" (the server's default: continuous
    batching, `slots` resident jobs, least remaining work first) or "fifo"
    (arrival order, one job at a time). The arrivals of a load are the same
    for both policies. Prints one progress line per run to stderr."""
    import paper_1808_01478_amd as dh
    warm, frames = serving_frames(n_jobs, n_warm, seed)
    pairs = sum(f.total_pairs() for f in frames)
    fifo = {"hbm_budget_bytes": 8 << 30, "max_inflight": 1, "policy": dh.SCHED_ARRIVAL}
    if policy == "fifo":
        args = fifo
    elif policy == "shortest":
        args = {"hbm_budget_bytes": 8 << 30, "max_inflight": slots, "policy": dh.SCHED_SHORTEST}
    else:
        raise ValueError(policy)
    t0 = time.perf_counter()
    run_trace(args, warm, [0.0] * len(warm))
    capacity = batched_rate(frames[:n_capacity])["jobs_per_s"]
    print(f"[serving] {policy}: batched-path capacity {capacity:.2f} jobs/s "
          f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    runs = [(k, lam, args) for k, lam in enumerate(loads)]
    if policy == "shortest":
        runs.append((loads.index(0.75) if 0.75 in loads else len(loads), 0.75,
                     dict(args, hbm_budget_bytes=256 << 20)))
    out = {"policy": policy, "jobs": n_jobs, "warmup_jobs": n_warm, "pairs": pairs,
           "batched_jobs_per_s": capacity, "runs": []}
    for k, lam, a in runs:
        gaps = np.random.Generator(np.random.PCG64(seed * 100 + k)).exponential(
            1.0 / (lam * capacity), size=n_jobs)
        lat, end, st = run_trace(a, frames, gaps, progress=f"load {lam}")
        row = {"load": lam, "budget_bytes": a["hbm_budget_bytes"],
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "p90_ms": float(np.percentile(lat, 90) * 1e3),
               "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "jobs_per_s": n_jobs / end, "throughput_pairs_per_s": pairs / end,
               "max_running": st["max_running"], "peak_bytes": st["peak_bytes"],
               "launches": st["launches"], "shared_launches": st["shared_launches"]}
        out["runs"].append(row)
        print(f"[serving] {policy} load {lam} budget {a['hbm_budget_bytes'] >> 20} MiB: "
              f"p50 {row['p50_ms']:.1f} ms p99 {row['p99_ms']:.1f} ms "
              f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    return out


def cpu_tuned(frame):
    """The library's cache-blocked, vectorized CPU kernel (dh_cpu_histo) on
    the whole 100,000-point orthorhombic frame, binary32 and binary64, the
    same host threads as the oracle: context for the oracle baseline, not the
    target."""
    import paper_1808_01478_amd as dh
    # the library's default: the affinity mask, at most OMP_NUM_THREADS
    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit() and int(os.environ["OMP_NUM_THREADS"]) > 0:
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    out = {"unit": "pairs/s", "cores": threads, "sample": "the whole frame, once per precision"}
    for prec, name in ((dh.FP32, "fp32"), (dh.FP64, "fp64")):
        t0 = time.perf_counter()
        dh.cpu_histo(frame.coords, frame.offsets, frame.box_type, frame.box, frame.r_max,
                     frame.n_bins, prec, 0)
        out[name] = frame.total_pairs() / (time.perf_counter() - t0)
    return out


def host_cores():
    """Physical cores and logical CPUs from lscpu, and the CPUs this process
    may run on."""
    import subprocess
    info = {"lscpu_physical_cores": None, "lscpu_cpus": None,
            "affinity_cpus": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in txt.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if "Core(s) per socket" in kv and "Socket(s)" in kv:
            info["lscpu_physical_cores"] = int(kv["Core(s) per socket"]) * int(kv["Socket(s)"])
        if "CPU(s)" in kv:
            info["lscpu_cpus"] = int(kv["CPU(s)"])
        info["model"] = kv.get("Model name")
    except Exception:
        pass
    return info


def cpu_baseline(frame, target_s: float = 12.0, target_1t_s: float = 5.0):
    """The oracle (plain FP64 double loop, OpenMP) on the first M points of
    every species of the same frame, M sized for about target_s seconds on
    all the threads it gets, and again on one thread (about target_1t_s)."""
    import oracle
    oracle.build(force=False)
    frac = np.array(frame.species_sizes(), np.float64) / frame.n

    def sample(m_total):
        return frame.subset([max(1, int(m_total * f)) for f in frac])

    def timed(target, n_threads):
        cal = sample(4000 if n_threads == 1 else 6000)
        t0 = time.perf_counter()
        oracle.frame_histogram(cal, n_threads=n_threads)
        rate = cal.total_pairs() / max(time.perf_counter() - t0, 1e-3)
        m = max(4000, min(int(np.sqrt(2.0 * rate * target)), frame.n))
        sub = sample(m)
        reps, done = 0, 0.0
        t0 = time.perf_counter()
        while reps == 0 or done < 0.5 * target:
            oracle.frame_histogram(sub, n_threads=n_threads)
            reps += 1
            done = time.perf_counter() - t0
        return sub, reps, done

    sub, reps, done = timed(target_s, 0)
    sub1, reps1, done1 = timed(target_1t_s, 1)
    cores = host_cores()

    def what(f, r, d):
        w = "the whole frame" if f.n == frame.n else \
            f"the first {f.n} points of the frame (species kept in proportion)"
        return f"{w}, {r} run(s), {f.total_pairs() * r} pairs in {d:.1f} s, binary64"

    return {
        "value": sub.total_pairs() * reps / done,
        "unit": "pairs/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": what(sub, reps, done),
        "one_thread": {"value": sub1.total_pairs() * reps1 / done1, "unit": "pairs/s",
                       "sample": what(sub1, reps1, done1)},
        "host": cores,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="triclinic1M",
                    choices=("triclinic1M", "ortho100k", "tiny"))
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="timed binary64 steps (default: as many as --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=1000,
                    help="measured jobs of the serving comparison (0 = skip)")
    ap.add_argument("--no-tune", action="store_true",
                    help="built-in launch shape instead of tuning on the first warm-up call")
    ap.add_argument("--trajectory-frames", type=int, default=512,
                    help="frames of the batched trajectory comparison (0 = skip)")
    ap.add_argument("--no-wide", dest="wide", action="store_false",
                    help="skip the wide-histogram comparison")
    ap.add_argument("--ortho-steps", type=int, default=20,
                    help="binary32 steps on the 100,000-point orthorhombic frame, reported as "
                         "a sub-object (half as many binary64 steps; 0 = skip)")
    ap.add_argument("--serving-sweep", choices=("shortest", "fifo"), default=None,
                    help="run only the full serving protocol for one policy (1000 jobs at "
                         "each of four loads, several minutes) and print its JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the histogram of a frame runs on a single "
              "MI355X, and runs on more than one GPU are not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1808_01478_amd as dh

    if args.serving_sweep:
        print(json.dumps({"serving_sweep": bench_serving_sweep(args.serving_sweep)}), flush=True)
        return

    frame, desc = workload(args.workload)
    kind = box_kind(frame)
    pairs = frame.total_pairs()
    ctx = dh.Context(0)
    if not args.no_tune:
        # shapes from the committed cache; a bucket missing from it is tuned
        # on the first warm-up call
        from paper_1808_01478_amd.tune import DEFAULT_CACHE
        ctx.set_tuning(dh.TUNE_ON, DEFAULT_CACHE if os.path.exists(DEFAULT_CACHE) else None)
        # the library-owned context of the synchronous entry point reads its
        # tuning mode from the environment when it is created
        if os.path.exists(DEFAULT_CACHE):
            os.environ.setdefault("DH_TUNE", str(dh.TUNE_CACHED))
            os.environ.setdefault("DH_TUNE_CACHE", DEFAULT_CACHE)
    fp64_steps = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps)
    _, head, res = bench_frame(ctx, args.workload, args.steps, fp64_steps, max(1, args.warmup),
                               frame)
    r32, r64 = res["fp32"], res.get("fp64")
    progress("checking the step's histograms against the stored oracle result")
    parity = check_against_golden(args.workload, frame, r32, r64)

    value = pairs * args.steps / r32["wall_s"]
    ach32 = head["fp32"]["achieved_tflops"]
    traffic = traffic_for(args.workload, 0, None)
    line = {
        "metric": "pair-distances binned/sec (1 MI355X, FP32 vs FP64) + p50/p99 job latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "n": frame.n,
            "species": frame.species_sizes(),
            "n_bins": frame.n_bins,
            "r_max": frame.r_max,
            "pairs_per_step": pairs,
            "flops_per_pair": FLOPS_PER_PAIR[kind],
            "launch_shape": head["fp32"]["launch_shape"],
            "tuned": not args.no_tune,
        },
        "latency_ms": {"p50": r32["step_ms_p50"], "p99": r32["step_ms_p99"]},
        "fp64": head.get("fp64"),
        "parity": parity,
        "roofline": {
            "bound": "alu",
            "kernel": KERNEL_NAME,
            "achieved": ach32,
            "peak": PEAK_TFLOPS[0],
            "unit": "TFLOP/s",
            "frac": ach32 / PEAK_TFLOPS[0],
            "traffic": traffic,
            "kernel_ms_avg": r32["kernel_ms_avg"],
            "flops_per_launch": pairs * FLOPS_PER_PAIR[kind],
        },
        "cpu_baseline": None,
    }
    if args.ortho_steps > 0 and args.workload != "ortho100k":
        _, sub, _ = bench_frame(ctx, "ortho100k", args.ortho_steps, max(1, args.ortho_steps // 2),
                                3)
        line["ortho100k"] = sub
    # PCIe-inclusive rate of the synchronous host-buffer entry point
    progress("host buffers")
    line["host_buffers"] = time_host_buffers(frame, dh.FP32, max(1, args.steps // 4))
    line["host_buffers"]["fp64"] = time_host_buffers(frame, dh.FP64, max(1, args.steps // 4))
    if args.serving_jobs > 0:
        progress(f"serving, {args.serving_jobs} jobs")
        line["serving"] = bench_serving(args.serving_jobs)
        line["latency_ms"]["serving_p50"] = line["serving"]["continuous_batching"]["p50_ms"]
        line["latency_ms"]["serving_p99"] = line["serving"]["continuous_batching"]["p99_ms"]
    if args.wide:
        progress("wide histograms")
        line["wide"] = bench_wide(workloads.ortho())
        progress("image search")
        line["image_search"] = bench_image_search()
    if args.trajectory_frames > 0:
        progress(f"trajectory, {args.trajectory_frames} frames")
        line["trajectory"] = bench_trajectory(ctx, args.trajectory_frames, max(1, args.steps // 5))
        progress("trajectory file")
        line["trajectory_file"] = bench_trajectory_file(ctx)
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(frame)
        progress("tuned CPU kernel")
        line["cpu_tuned"] = cpu_tuned(workloads.ortho())
    ctx.close()
    del torch
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
