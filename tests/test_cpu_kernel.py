"""The tuned CPU kernel (dh_cpu_histo) against the oracle, on the CPU: the
binary64 canonical sequence gives identical counts on every parity frame,
binary32 stays within the edge-pair bound, and the thread count changes
nothing."""
import numpy as np
import pytest

import oracle
from cases import parity_cases
from gpu_util import fp32_bound_violations

CASES = [f for f in parity_cases() if f.n_bins <= 100_000]


@pytest.fixture(scope="module")
def dh():
    import paper_1808_01478_amd as dh
    return dh


@pytest.mark.parametrize("frame", CASES, ids=[f.name for f in CASES])
def test_fp64_equals_oracle(dh, frame):
    h, oor = dh.cpu_histo(frame.coords, frame.offsets, frame.box_type, frame.box, frame.r_max,
                          frame.n_bins, dh.FP64, n_threads=4)
    ref = oracle.frame_histogram(frame)
    assert np.array_equal(h, ref.hist), f"{int((h != ref.hist).sum())} bins differ"
    assert np.array_equal(oor, ref.out_of_range)


@pytest.mark.parametrize("frame", CASES[:9], ids=[f.name for f in CASES[:9]])
def test_fp32_edge_bound(dh, frame):
    h, oor = dh.cpu_histo(frame.coords, frame.offsets, frame.box_type, frame.box, frame.r_max,
                          frame.n_bins, dh.FP32, n_threads=4)
    w = oracle.edge_window(frame.coords, frame.box, frame.r_max)
    ref = oracle.frame_histogram(frame, edge_window=w)
    assert list(h.sum(axis=1).astype(np.int64) + oor.astype(np.int64)) == frame.hist_pairs()
    bad = fp32_bound_violations(h, ref.hist, ref.edges)
    assert not bad, "; ".join(bad[:5])


def test_threads_do_not_matter(dh):
    fr = CASES[2]
    a = dh.cpu_histo(fr.coords, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, dh.FP32, 1)
    for t in (2, 7, 0):
        b = dh.cpu_histo(fr.coords, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins,
                         dh.FP32, t)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_invalid_arguments(dh):
    fr = CASES[0]
    with pytest.raises(dh.DisthistError):
        dh.cpu_histo(fr.coords, fr.offsets, fr.box_type, fr.box, -1.0, fr.n_bins, dh.FP64)
    with pytest.raises(dh.DisthistError):
        dh.cpu_histo(fr.coords, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, dh.FP64, -2)
    x = fr.coords.copy()
    x[3, 1] = np.nan
    with pytest.raises(dh.DisthistError):
        dh.cpu_histo(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, dh.FP64)
