"""The device binary64 root against the oracle (IEEE sqrt) on the arguments
where a root that is not correctly rounded shows: squared distances whose
roots lie within about 3e-17 of an ulp of a rounding midpoint, those nearest
to squared midpoints, and those next to squared midpoints just below and
above integers, where with s = n_bins / r_max = 1 (or 2) a root one ulp off
moves the pair into the neighbouring bin. Per pair through dh_pair_t_async,
and as histograms in every accumulation mode (one LDS histogram, LDS bin
windows, uint64 global atomics with more than 2^20 bins, where every pair
takes the correctly rounded root)."""
import numpy as np
import pytest

import midpoints
import oracle
import workloads
from gpu_util import run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.close()


def _pair_t_gpu(ctx, coords, pi, pj, r_max, n_bins):
    import torch
    dev = torch.device("cuda")
    x = torch.from_numpy(coords).to(dev)
    dpi = torch.from_numpy(pi.astype(np.int32)).to(dev)
    dpj = torch.from_numpy(pj.astype(np.int32)).to(dev)
    t = torch.empty(len(pi), dtype=torch.float64, device=dev)
    ctx.pair_t_async(x, workloads.BOX_NONE, None, r_max, n_bins, 1, dpi, dpj, t)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_pair_t_at_midpoints(ctx):
    rng = np.random.Generator(np.random.PCG64(5151))
    qs = midpoints.hardest_q() + midpoints.hard_q(rng, 2000, -30, 40, k=2)
    qs += midpoints.edge_q(list(range(1, 300)) + [1023, 1024, 1025, 4095, 4096, 65535], k=2)
    print(f"\n[case] pair_t at {len(qs)} midpoint arguments", flush=True)
    coords, pi, pj = midpoints.pair_coords(qs)
    t_ref = oracle.pair_t(coords, workloads.BOX_NONE, None, 4096.0, 4096, pi, pj)
    assert np.array_equal(t_ref, np.sqrt(np.asarray(qs)))      # s = 1: t is the root
    t = _pair_t_gpu(ctx, coords, pi, pj, 4096.0, 4096)
    bad = np.nonzero(t != t_ref)[0]
    assert len(bad) == 0, f"{len(bad)} roots differ, first q={qs[bad[0]]!r}"


EDGE_INTS = list(range(1, 2000, 7)) + [1024, 2048, 4095]


@pytest.mark.parametrize("r_max,n_bins", [(4096.0, 4096), (2048.0, 4096), (100_000.0, 100_000),
                                          (1_048_576.0, 1_048_576)],
                         ids=["lds-s1", "lds-s2", "windows-s1", "global-s1"])
def test_histogram_at_bin_edges(ctx, r_max, n_bins):
    qs = midpoints.edge_q(EDGE_INTS, k=3)
    qs += [q for q in midpoints.hardest_q(exps=(0, 5, 10)) if q < 4000.0 ** 2]
    coords, _, _ = midpoints.pair_coords(qs)
    fr = workloads.Frame(coords, np.array([0, len(coords)], np.int64), workloads.BOX_NONE, None,
                         r_max, n_bins, f"midpoint-edges-{n_bins}")
    print(f"\n[case] {fr.name} N={fr.n}", flush=True)
    ref = oracle.frame_histogram(fr)
    h, oor = run_gpu(ctx, fr, 1)
    assert np.array_equal(h, ref.hist), f"{int((h != ref.hist).sum())} bins differ"
    assert np.array_equal(oor, ref.out_of_range)
