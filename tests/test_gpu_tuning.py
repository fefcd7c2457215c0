"""Launch shapes change speed, never counts: every knob combination must give
bit-identical histograms (this is also the race test: integer sums commute,
so any difference would be a missing barrier or a lost update). The tuner
caches its choice per bucket and a cache file is reused by a new context."""
import itertools
import json

import numpy as np
import pytest

import workloads
from gpu_util import run_gpu

pytestmark = pytest.mark.gpu

SKEW = np.array([[10.0, 0, 0], [3.0, 9.5, 0], [-2.0, 3.5, 9.0]])


def same_knobs(cfg, knobs, names):
    """last_config reports the workgroup size launched; a stored 0 means the
    automatic choice, which may be any size."""
    return all(cfg[n] == v for n, v in zip(names, knobs) if not (n == "threads" and v == 0))


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.set_config(None)
    c.close()


FRAMES = [
    workloads.random_frame(501, [5000, 3000], workloads.BOX_ORTHO,
                           box=workloads.ortho_box(20.0, 20.0, 20.0), r_max=10.0, n_bins=2000),
    workloads.random_frame(502, [4000, 1500, 700], workloads.BOX_TRICLINIC, box=SKEW,
                           r_max=0.45 * workloads.min_width(SKEW), n_bins=1500),
    workloads.random_frame(503, [3000], workloads.BOX_NONE, r_max=8.0, n_bins=45_000),
    workloads.triclinic(n=8000),
    # spatially sorted staging (at least 65,536 points): triclinic, and
    # orthorhombic in binary64
    workloads.triclinic(n=70_000),
    workloads.random_frame(504, [40_000, 26_000], workloads.BOX_ORTHO,
                           box=workloads.ortho_box(30.0, 32.0, 34.0), r_max=14.0, n_bins=3000),
]

SHAPES = [dict(zip(("r", "copies", "tj", "noclamp", "occ_cap", "items_per_wg", "threads",
                    "wide"), v))
          for v in itertools.product((4, 8), (1, 2, 4), (128, 256), (0, 1), (0, 1), (4, 16),
                                     (256, 512, 1024), (0, 1, 3))]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("fi", range(len(FRAMES)))
def test_all_shapes_identical(ctx, precision, fi):
    fr = FRAMES[fi]
    print(f"\n[case] shapes frame={fi} prec={precision}", flush=True)
    ctx.set_config(None)
    ref, ref_oor = run_gpu(ctx, fr, precision)
    rng = np.random.Generator(np.random.PCG64(fi * 2 + precision))
    for k in rng.choice(len(SHAPES), 12, replace=False):
        ctx.set_config(SHAPES[k])
        h, oor = run_gpu(ctx, fr, precision)
        cfg = ctx.last_config()
        assert all(cfg[n] == v for n, v in SHAPES[k].items() if n != "threads")
        assert np.array_equal(h, ref), f"shape {SHAPES[k]} changed the counts"
        assert np.array_equal(oor, ref_oor)
    ctx.set_config(None)


@pytest.mark.parametrize("precision", [0, 1])
def test_sorted_frame_every_mode(ctx, precision):
    """The spatially sorted triclinic frame (ragged i-blocks, diagonal items,
    lanes past the end of an item) in every accumulation mode: four LDS
    copies leave room for a third of its 20,000 bins, so it runs as bin
    windows; `wide` = 1 forces uint64 global atomics. Counts and out-of-range
    counts equal the default single LDS histogram's."""
    fr = FRAMES[4]
    print(f"\n[case] sorted frame, all modes, prec={precision}", flush=True)
    ctx.set_config(None)
    ref, ref_oor = run_gpu(ctx, fr, precision)
    assert ctx.last_config()["mode"] == 0
    for knobs, mode in (([4, 4, 256, 1, 0, 8, 1024, 0], 1), ([8, 4, 128, 0, 0, 4, 512, 0], 1),
                        ([8, 1, 256, 1, 0, 8, 256, 1], 2), ([4, 2, 128, 1, 1, 16, 256, 1], 2)):
        ctx.set_config(knobs)
        h, oor = run_gpu(ctx, fr, precision)
        cfg = ctx.last_config()
        assert cfg["mode"] == mode, (knobs, cfg)
        if mode == 1:
            assert cfg["sweeps"] >= 2, cfg
        assert np.array_equal(h, ref), f"shape {knobs} changed the counts"
        assert np.array_equal(oor, ref_oor)
    ctx.set_config(None)


def test_invalid_shape_rejected(ctx):
    import paper_1808_01478_amd as dh
    for bad in ([3, 1, 256, 1, 0, 8, 256, 3], [8, 3, 256, 1, 0, 8, 256, 3],
                [8, 1, 64, 1, 0, 8, 256, 3], [8, 1, 256, 2, 0, 8, 256, 3],
                [8, 1, 256, 1, -1, 8, 256, 3], [8, 1, 256, 1, 0, 0, 256, 3],
                [8, 1, 256, 1, 0, 8, 128, 3], [8, 1, 256, 1, 0, 8, 2048, 3],
                [8, 1, 256, 1, 0, 8, 256, -1], [8, 1, 256, 1, 0, 8, 256, 1 << 20]):
        with pytest.raises(dh.DisthistError):
            ctx.set_config(bad)
    with pytest.raises(ValueError):
        ctx.set_config([8, 1, 256, 1, 0, 8, 256])       # one knob short


def test_tuner_caches_and_reuses(tmp_path):
    import paper_1808_01478_amd as dh
    path = str(tmp_path / "tune.json")
    fr = FRAMES[0]
    with dh.Context(0) as c1:
        c1.set_config(None)
        ref, _ = run_gpu(c1, fr, 0)
        c1.set_tuning(dh.TUNE_ON, path)
        h, _ = run_gpu(c1, fr, 0)          # tunes on this call
        assert np.array_equal(h, ref)
        chosen = c1.last_config()
    data = json.load(open(path))
    assert len(data["entries"]) == 1
    (key, knobs), = data["entries"].items()
    assert key.startswith("gfx") and "|p0|" in key
    assert same_knobs(chosen, knobs, dh.KNOB_NAMES)
    with dh.Context(0) as c2:
        c2.set_tuning(dh.TUNE_CACHED, path)
        h2, _ = run_gpu(c2, fr, 0)
        assert np.array_equal(h2, ref)
        assert same_knobs(c2.last_config(), knobs, dh.KNOB_NAMES)


def test_handwritten_cache_is_used(tmp_path):
    import paper_1808_01478_amd as dh
    fr = FRAMES[1]
    with dh.Context(0) as c:
        c.set_tuning(dh.TUNE_ON, str(tmp_path / "probe.json"))
        run_gpu(c, fr, 1)
        key = next(iter(json.load(open(tmp_path / "probe.json"))["entries"]))
    path = tmp_path / "hand.json"
    path.write_text(json.dumps({"version": 3, "entries": {key: [4, 2, 128, 0, 1, 4, 512, 2]}}))
    with dh.Context(0) as c:
        c.set_tuning(dh.TUNE_CACHED, str(path))
        run_gpu(c, fr, 1)
        cfg = c.last_config()
        assert [cfg[n] for n in dh.KNOB_NAMES] == [4, 2, 128, 0, 1, 4, 512, 2]


@pytest.mark.parametrize("precision", [0, 1])
def test_bounded_launches_identical(ctx, precision):
    """Splitting a frame into many bounded launches (each with its own work
    counter and flushes) leaves every count unchanged, in all three
    accumulation modes."""
    import paper_1808_01478_amd as dh
    frames = FRAMES + [
        workloads.random_frame(504, [6000, 2500], workloads.BOX_ORTHO, n_bins=300_000),
    ]
    ctx.set_config(None)
    try:
        for fi, fr in enumerate(frames):
            print(f"\n[case] bounded launches frame={fi} prec={precision}", flush=True)
            ctx.set_launch_pairs(0)
            ref, ref_oor = run_gpu(ctx, fr, precision)
            for limit in (1 << 24, 1 << 26):
                ctx.set_launch_pairs(limit)
                h, oor = run_gpu(ctx, fr, precision)
                assert np.array_equal(h, ref), f"frame {fi}: limit {limit} changed the counts"
                assert np.array_equal(oor, ref_oor)
        with pytest.raises(dh.DisthistError):
            ctx.set_launch_pairs(-1)
        with pytest.raises(dh.DisthistError):
            ctx.set_launch_pairs(1000)
    finally:
        ctx.set_launch_pairs(0)


def test_bounded_launches_full_size(ctx):
    fr = workloads.ortho()
    ctx.set_config(None)
    ctx.set_launch_pairs(0)
    ref, _ = run_gpu(ctx, fr, 0)
    try:
        for limit in (3 << 33, 1 << 30):
            ctx.set_launch_pairs(limit)
            h, _ = run_gpu(ctx, fr, 0)
            assert np.array_equal(h, ref), f"limit {limit}"
    finally:
        ctx.set_launch_pairs(0)
