"""Binary32 bin rule on inputs built to hit it: exactly integer t (ties,
which go to the even neighbour) and t = 0 (coincident points, bin -1 of the
bit rule, counted in bin 0 through the guard word).

Points of an integer lattice in a periodic cube of edge 8 have fixed-point
differences that are exact multiples of 2^29, so their binary32 squared
distances and roots are exact, and with an odd integer n_bins / r_max the
scaled distance t of every pair at integer distance is an odd or even
integer exactly. Every device mode (one LDS histogram with and without
clamping, LDS bin windows, global atomics) must give the same binary32
counts, within the oracle's edge-pair bound; binary64 must equal the
oracle."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import fp32_bound_violations, run_gpu

pytestmark = pytest.mark.gpu

KNOBS = ("r", "copies", "tj", "noclamp", "occ_cap", "items_per_wg", "threads", "wide")
MODE_LDS, MODE_SWEEP, MODE_GLOBAL = 0, 1, 2


def knobs(noclamp=1, wide=48):
    return dict(zip(KNOBS, (4, 1, 256, noclamp, 0, 8, 512, wide)))


def lattice_frame(n_bins, r_max=4.0, seed=71):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(8.0)
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    dup = lat[rng.integers(0, len(lat), size=100)]            # coincident with lattice points
    uni = rng.uniform(0.0, 8.0, size=(400, 3))
    x = np.ascontiguousarray(np.concatenate([lat, dup, uni]))
    # two species so that cross histograms see the coincident points too
    return workloads.Frame(x, np.array([0, 600, len(x)], np.int64), workloads.BOX_ORTHO,
                           workloads.ortho_box(8.0, 8.0, 8.0), r_max, n_bins,
                           f"lattice-{n_bins}")


def coincident_pairs(fr):
    """Pairs at distance exactly 0 per histogram, in the histogram order."""
    from collections import Counter
    off = fr.offsets
    keys = [Counter(map(tuple, fr.coords[off[s]:off[s + 1]])) for s in range(len(off) - 1)]
    k = len(keys)
    out = [sum(c * (c - 1) // 2 for c in keys[s].values()) for s in range(k)]
    for s in range(k):
        for t in range(s + 1, k):
            out.append(sum(c * keys[t].get(p, 0) for p, c in keys[s].items()))
    return out


def check_against_oracle(fr, h32, h64):
    w = oracle.edge_window(fr.coords, fr.box, fr.r_max)
    ref = oracle.frame_histogram(fr, edge_window=w)
    assert np.array_equal(h64, ref.hist), f"{fr.name}: binary64 differs from the oracle"
    bad = fp32_bound_violations(h32, ref.hist, ref.edges)
    assert not bad, "; ".join(bad[:5])
    return ref


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.set_config(None)
    c.close()


def test_lds_clamped_unclamped_and_global_agree(ctx):
    """12 bins over r_max = 4 (t = 3r): lattice pairs at distance 1 and 3
    sit exactly on the odd edges 3 and 9."""
    fr = lattice_frame(12)
    print(f"\n[case] {fr.name} N={fr.n}", flush=True)
    got = {}
    for name, kn in (("noclamp", knobs(noclamp=1)), ("clamp", knobs(noclamp=0)),
                     ("global", knobs(wide=1))):
        ctx.set_config(kn)
        got[name] = run_gpu(ctx, fr, 0)
        cfg = ctx.last_config()
        assert cfg["mode"] == (MODE_GLOBAL if name == "global" else MODE_LDS), (name, cfg)
    h64, _ = run_gpu(ctx, fr, 1)
    ctx.set_config(None)
    for name in ("clamp", "global"):
        assert np.array_equal(got[name][0], got["noclamp"][0]), f"{name} differs from noclamp"
        assert np.array_equal(got[name][1], got["noclamp"][1]), f"{name}: out-of-range differs"
    ref = check_against_oracle(fr, got["noclamp"][0], h64)
    # the ties really occur: binary32 moves the pairs at t = 3 and t = 9 down
    assert not np.array_equal(got["noclamp"][0], ref.hist)
    # the coincident pairs (t = 0) are all counted, in bin 0
    same = coincident_pairs(fr)
    assert sum(same) > 0
    assert np.all(got["noclamp"][0][:, 0] >= np.array(same, np.uint64))


def test_bin_windows_and_global_agree(ctx):
    """60,004 bins over r_max = 4 (t = 15001 r, two LDS bin windows): the
    same rule in windows as with global atomics."""
    fr = lattice_frame(60_004)
    print(f"\n[case] {fr.name} N={fr.n}", flush=True)
    ctx.set_config(knobs())
    sw = run_gpu(ctx, fr, 0)
    cfg = ctx.last_config()
    assert cfg["mode"] == MODE_SWEEP and cfg["sweeps"] >= 2, cfg
    ctx.set_config(knobs(wide=1))
    gl = run_gpu(ctx, fr, 0)
    assert ctx.last_config()["mode"] == MODE_GLOBAL
    h64, _ = run_gpu(ctx, fr, 1)
    ctx.set_config(None)
    assert np.array_equal(sw[0], gl[0]) and np.array_equal(sw[1], gl[1])
    check_against_oracle(fr, sw[0], h64)
