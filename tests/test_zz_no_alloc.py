"""dh_histo_noalloc (the allocation-free entry point for callers that cannot
allocate) against dh_histo_async on the same frames: identical histograms and
out-of-range counts in both precisions, on consecutive calls whose second
input is smaller (the shared scratch keeps the previous call's contents), and
binary64 equal to the oracle."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SKEW = np.array([[10.0, 0, 0], [3.0, 9.5, 0], [-2.0, 3.5, 9.0]])


def _named(frame, name):
    frame.name = name
    return frame


def frames():
    w = workloads.min_width(SKEW)
    return [
        workloads.random_frame(501, [4000, 2500], workloads.BOX_ORTHO, n_bins=1000),
        workloads.random_frame(502, [1500, 700, 300], workloads.BOX_TRICLINIC, box=SKEW,
                               r_max=0.45 * w, n_bins=512),
        workloads.random_frame(503, [1100, 900], workloads.BOX_TRICLINIC, box=SKEW,
                               r_max=0.8 * w, n_bins=300),
        workloads.random_frame(504, [2201, 5, 0, 37], workloads.BOX_NONE, r_max=9.0, n_bins=777),
        workloads.random_frame(505, [1800, 1000], workloads.BOX_ORTHO, n_bins=60_000),
        workloads.random_frame(506, [1600, 900], workloads.BOX_ORTHO, n_bins=3_000_000),
        workloads.random_frame(507, [1], workloads.BOX_NONE, n_bins=16),
        workloads.tiny(n=3000),
        _named(workloads.triclinic(n=66_000), "tric-clustered-66k-sorted"),
    ]


def _run_both(dh, ctx, fr, prec):
    import torch
    dev = torch.device("cuda")
    x = torch.from_numpy(np.ascontiguousarray(fr.coords)).to(dev)
    a = torch.full((fr.n_hist, fr.n_bins), -1, dtype=torch.int64, device=dev)
    ao = torch.full((fr.n_hist,), -1, dtype=torch.int64, device=dev)
    b = torch.full_like(a, -1)
    bo = torch.full_like(ao, -1)
    dh.histo_noalloc(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, prec, a, ao)
    ctx.histo_async(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, prec, b, bo)
    torch.cuda.synchronize()
    return (a.cpu().numpy().view(np.uint64), ao.cpu().numpy().view(np.uint64),
            b.cpu().numpy().view(np.uint64), bo.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_async(prec):
    import paper_1808_01478_amd as dh
    with dh.Context(0) as ctx:
        for fr in frames():
            print(f"\n[case] noalloc {fr.name} N={fr.n} bins={fr.n_bins} prec={prec}", flush=True)
            h, o, ref_h, ref_o = _run_both(dh, ctx, fr, prec)
            assert np.array_equal(h, ref_h), f"{fr.name}: {int((h != ref_h).sum())} bins differ"
            assert np.array_equal(o, ref_o), fr.name
            if prec == 1 and fr.n_bins <= 60_000:
                ref = oracle.frame_histogram(fr)
                assert np.array_equal(h, ref.hist) and np.array_equal(o, ref.out_of_range), fr.name


def test_noalloc_second_call_smaller():
    """Two calls in a row, the second with a smaller input: the second must
    not see anything of the first in the shared scratch."""
    import paper_1808_01478_amd as dh
    big = workloads.random_frame(511, [6000, 3000], workloads.BOX_ORTHO, n_bins=2000)
    small = big.subset([700, 300])
    with dh.Context(0) as ctx:
        for prec in (0, 1):
            for fr in (big, small):
                print(f"\n[case] noalloc consecutive {fr.name} N={fr.n} prec={prec}", flush=True)
                h, o, ref_h, ref_o = _run_both(dh, ctx, fr, prec)
                assert np.array_equal(h, ref_h) and np.array_equal(o, ref_o), fr.name


def test_noalloc_rejects_oversize_frame():
    import paper_1808_01478_amd as dh
    import torch
    n = 2_000_000   # 64 MB of binary64 staging, beyond the 48 MiB scratch
    x = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    out = torch.full((1, 10), -1, dtype=torch.int64, device="cuda")
    with pytest.raises(dh.DisthistError) as e:
        dh.histo_noalloc(x, [0, n], dh.BOX_NONE, None, 1.0, 10, dh.FP64, out)
    assert e.value.code == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert (out.cpu() == -1).all()
