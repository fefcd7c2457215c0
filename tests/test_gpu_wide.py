"""The global-atomic accumulation mode (histograms wider than LDS) against
the oracle and against the LDS modes.

Both modes compute every pair's t with the same arithmetic and only count
differently (uint64 global atomics against LDS sub-histograms flushed into
uint64), so binary64 must equal the oracle bit for bit and binary32 must
equal the LDS path bit for bit, on every parity frame, at full size, and at
the largest bin count the library accepts."""
import numpy as np
import pytest

import oracle
import workloads
from cases import parity_cases
from gpu_util import fp32_bound_violations, run_gpu

pytestmark = pytest.mark.gpu

CASES = parity_cases()
KNOBS = ("r", "copies", "tj", "noclamp", "occ_cap", "items_per_wg", "threads", "wide")
MODE_LDS, MODE_SWEEP, MODE_GLOBAL = 0, 1, 2


def knobs(wide, r=8, tj=256, threads=256):
    return dict(zip(KNOBS, (r, 1, tj, 1, 0, 8, threads, wide)))


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.set_config(None)
    c.close()


@pytest.mark.parametrize("frame", CASES, ids=[f.name for f in CASES])
def test_global_mode_parity(ctx, frame):
    print(f"\n[case] global {frame.name} N={frame.n} bins={frame.n_bins}", flush=True)
    ctx.set_config(None)
    lds32, lds_oor32 = run_gpu(ctx, frame, 0)
    ctx.set_config(knobs(wide=1))
    g64, g_oor64 = run_gpu(ctx, frame, 1)
    assert ctx.last_config()["mode"] == MODE_GLOBAL or frame.total_pairs() == 0
    g32, g_oor32 = run_gpu(ctx, frame, 0)
    ctx.set_config(None)
    ref = oracle.frame_histogram(frame)
    assert np.array_equal(g64, ref.hist), f"{int((g64 != ref.hist).sum())} bins differ"
    assert np.array_equal(g_oor64, ref.out_of_range)
    assert np.array_equal(g32, lds32), "binary32: global atomics differ from LDS"
    assert np.array_equal(g_oor32, lds_oor32)


@pytest.mark.parametrize("r,tj,threads", [(4, 128, 512), (8, 256, 1024), (4, 256, 256)])
def test_global_mode_shapes(ctx, r, tj, threads):
    fr = CASES[2]
    ctx.set_config(knobs(wide=1, r=r, tj=tj, threads=threads))
    got = [run_gpu(ctx, fr, p)[0] for p in (0, 1)]
    ctx.set_config(None)
    ref = [run_gpu(ctx, fr, p)[0] for p in (0, 1)]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_mode_selection(ctx):
    """Default shapes: one LDS histogram when it fits, bin windows up to a few
    dozen windows, global atomics beyond; the automatic workgroup size is
    1024 threads when one 256-thread workgroup would fill a CU's LDS."""
    ctx.set_config(None)
    small = workloads.random_frame(31, [500], workloads.BOX_NONE, n_bins=1000)
    mid = workloads.random_frame(32, [500], workloads.BOX_NONE, n_bins=60_000)
    many = workloads.random_frame(33, [500], workloads.BOX_NONE, n_bins=1_000_000)
    wide = workloads.random_frame(36, [500], workloads.BOX_NONE, n_bins=4_000_000)
    cfgs = []
    for f in (small, mid, many, wide):
        run_gpu(ctx, f, 0)
        cfgs.append(ctx.last_config())
    assert [c["mode"] for c in cfgs] == [MODE_LDS, MODE_SWEEP, MODE_SWEEP, MODE_GLOBAL], cfgs
    assert [c["threads"] for c in cfgs[:3]] == [256, 1024, 1024], cfgs
    ctx.set_config(knobs(wide=0))
    run_gpu(ctx, wide, 0)
    cfg = ctx.last_config()
    ctx.set_config(None)
    assert cfg["mode"] == MODE_SWEEP and cfg["sweeps"] > 100


def test_max_bins(ctx):
    """The largest accepted bin counts: binary64 with n_bins = 2^24 in global
    mode against the oracle; binary32 with n_bins = 2^22 in global mode
    against 100+ LDS bin windows (both bin alike)."""
    fr = workloads.random_frame(34, [3000], workloads.BOX_NONE, r_max=17.0, n_bins=1 << 24)
    print(f"\n[case] max bins N={fr.n}", flush=True)
    ctx.set_config(None)
    g64, oor64 = run_gpu(ctx, fr, 1)
    assert ctx.last_config()["mode"] == MODE_GLOBAL
    ref = oracle.frame_histogram(fr, n_threads=4)   # per-thread copies of 128 MiB
    assert np.array_equal(g64, ref.hist) and np.array_equal(oor64, ref.out_of_range)
    f32 = workloads.Frame(fr.coords, fr.offsets, fr.box_type, fr.box, fr.r_max, 1 << 22,
                          "max-bins-binary32")
    g32, _ = run_gpu(ctx, f32, 0)
    assert ctx.last_config()["mode"] == MODE_GLOBAL
    ctx.set_config(knobs(wide=0))
    s32, _ = run_gpu(ctx, f32, 0)
    assert ctx.last_config()["sweeps"] > 100
    ctx.set_config(None)
    assert np.array_equal(g32, s32)
    ref32 = oracle.frame_histogram(f32, edge_window=oracle.edge_window(f32.coords, f32.box,
                                                                       f32.r_max), n_threads=4)
    bad = fp32_bound_violations(g32, ref32.hist, ref32.edges)
    assert not bad, "; ".join(bad[:5])


def test_full_size_wide(ctx):
    """The 100k-point periodic frame with 250,000 bins: binary64 global
    atomics and binary64 bin windows both equal the oracle; binary32 global
    equals binary32 windows and stays within the edge-pair bound."""
    base = workloads.ortho()
    fr = workloads.Frame(base.coords, base.offsets, base.box_type, base.box, base.r_max,
                         250_000, "ortho100k-250k-bins")
    print(f"\n[case] {fr.name}", flush=True)
    out = {}
    for wide in (1, 0):
        ctx.set_config(knobs(wide=wide, r=8))
        out[wide, 0] = run_gpu(ctx, fr, 0)
        ctx.set_config(knobs(wide=wide, r=4, tj=128, threads=512))
        out[wide, 1] = run_gpu(ctx, fr, 1)
        assert ctx.last_config()["mode"] == (MODE_GLOBAL if wide else MODE_SWEEP)
    ctx.set_config(None)
    w = oracle.edge_window(fr.coords, fr.box, fr.r_max)
    ref = oracle.frame_histogram(fr, edge_window=w)
    for wide in (1, 0):
        assert np.array_equal(out[wide, 1][0], ref.hist), f"wide={wide}: binary64 differs"
        assert np.array_equal(out[wide, 1][1], ref.out_of_range)
    assert np.array_equal(out[1, 0][0], out[0, 0][0])
    bad = fp32_bound_violations(out[1, 0][0], ref.hist, ref.edges)
    assert not bad, "; ".join(bad[:5])


def test_tuner_picks_a_mode(tmp_path):
    import json
    import paper_1808_01478_amd as dh
    fr = workloads.random_frame(35, [3000, 2000], workloads.BOX_ORTHO, n_bins=300_000)
    path = str(tmp_path / "tune.json")
    with dh.Context(0) as c:
        ref, _ = run_gpu(c, fr, 0)
        c.set_tuning(dh.TUNE_ON, path)
        h, _ = run_gpu(c, fr, 0)
        cfg = c.last_config()
    assert np.array_equal(h, ref)
    (key, kn), = json.load(open(path))["entries"].items()
    assert kn[7] in (0, 1)
    assert cfg["mode"] == (MODE_GLOBAL if kn[7] == 1 else MODE_SWEEP)
