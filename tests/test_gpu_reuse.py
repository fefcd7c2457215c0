"""Repeated calls on one context: a call whose plan equals the previous one
(same frame shape, box, bins and output buffers, new coordinates) reuses the
work blob already on the device; its counts and out-of-range counts must
still be those of the oracle for the new coordinates, and a call with a
different shape in between must not disturb it."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def frame_like(seed, n=(2500, 1500), n_bins=800):
    """Uniform points in one fixed orthorhombic cell (the plan depends only on
    the shape, so frames of different seeds share it)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = workloads.ortho_box(12.0, 11.0, 13.0)
    x = rng.uniform(0.0, 1.0, size=(sum(n), 3)) * np.array([12.0, 11.0, 13.0])
    return workloads.Frame(np.ascontiguousarray(x), np.array([0, n[0], sum(n)], np.int64),
                           workloads.BOX_ORTHO, box, 5.5, n_bins, f"reuse-{seed}")


def test_same_plan_new_coordinates():
    import torch
    import paper_1808_01478_amd as dh
    dev = torch.device("cuda")
    frames = [frame_like(800 + k) for k in range(4)]
    other = frame_like(900, n=(1000, 700), n_bins=300)
    h = frames[0].n_hist
    out = torch.empty((h, frames[0].n_bins), dtype=torch.int64, device=dev)
    oor = torch.empty((h,), dtype=torch.int64, device=dev)
    out2 = torch.empty((other.n_hist, other.n_bins), dtype=torch.int64, device=dev)
    oor2 = torch.empty((other.n_hist,), dtype=torch.int64, device=dev)
    with dh.Context(0) as ctx:
        # a new frame each call into the same buffers, a different shape in
        # the middle, then binary64 on the same buffers
        seq = [(frames[0], 0), (frames[1], 0), (other, 0), (frames[2], 0), (frames[3], 0),
               (frames[3], 1), (frames[0], 1)]
        for fr, prec in seq:
            print(f"\n[case] {fr.name} precision={prec}", flush=True)
            o, r = (out2, oor2) if fr is other else (out, oor)
            x = torch.from_numpy(fr.coords).to(dev)
            ctx.histo_async(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, prec, o, r)
            torch.cuda.synchronize()
            got = o.cpu().numpy().view(np.uint64)
            got_oor = r.cpu().numpy().view(np.uint64)
            assert list(got.sum(axis=1).astype(np.int64) + got_oor.astype(np.int64)) == \
                fr.hist_pairs(), f"{fr.name}: counts and out-of-range do not add up"
            if prec == 1:
                ref = oracle.frame_histogram(fr)
                assert np.array_equal(got, ref.hist), fr.name
                assert np.array_equal(got_oor, ref.out_of_range), fr.name
            else:
                # binary32: the same as a fresh context's
                with dh.Context(0) as fresh:
                    o3 = torch.empty_like(o)
                    r3 = torch.empty_like(r)
                    fresh.histo_async(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins,
                                      prec, o3, r3)
                    torch.cuda.synchronize()
                assert np.array_equal(got, o3.cpu().numpy().view(np.uint64)), fr.name
                assert np.array_equal(got_oor, r3.cpu().numpy().view(np.uint64)), fr.name
