"""The stored oracle results of the full-size workloads (tests/golden/*.npz,
written by tests/golden/make_golden.py from the oracle alone): they belong to
the inputs the generators make on this host, and they satisfy what Algorithm 1
fixes independently of any arithmetic: every pair of a histogram is counted
once, in a bin or out of range."""
import numpy as np
import pytest

import oracle
import workloads
from golden.make_golden import frames_for, input_hash, load

NAMES = ["triclinic1M", "image_search200k", "trajectory32"]


@pytest.mark.parametrize("name", NAMES)
def test_golden_matches_inputs(name):
    g = load(name)
    frames = frames_for(name)
    off = g["hist_offsets"]
    assert len(off) == len(frames) + 1 and len(g["input_sha256"]) == len(frames)
    for k, fr in enumerate(frames):
        assert str(g["input_sha256"][k]) == input_hash(fr), f"{fr.name}: input differs"
        h = g["hist"][off[k]:off[k + 1]]
        oor = g["oor"][off[k]:off[k + 1]]
        e = g["edges"][off[k]:off[k + 1]]
        assert h.dtype == np.uint64 and h.shape == (fr.n_hist, fr.n_bins)
        assert e.shape == h.shape and oor.shape == (fr.n_hist,)
        total = h.sum(axis=1).astype(np.int64) + oor.astype(np.int64)
        assert list(total) == fr.hist_pairs(), fr.name
        assert g["window"][k] == oracle.edge_window(fr.coords, fr.box, fr.r_max)
        # an edge pair lies within the window of one edge: at most every pair
        assert int(e.sum()) <= fr.total_pairs()
