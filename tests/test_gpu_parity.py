"""HIP path vs the CPU oracle, element by element, through the C ABI.

binary64: bit-exact histograms and out-of-range counts.
binary32: within the edge-pair bound (per-edge cumulative difference at most
the number of pairs whose binary64 distance lies within 4 ulp32(S) of that
edge, S = max(|coordinate|, |box entry|, r_max))."""
import math

import numpy as np
import pytest

import oracle
import workloads
from cases import parity_cases
from gpu_util import fp32_bound_violations, oor_bound_violations, run_gpu

pytestmark = pytest.mark.gpu

CASES = parity_cases()


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("frame", CASES, ids=[f.name for f in CASES])
def test_fp64_bit_exact(ctx, frame):
    print(f"\n[case] {frame.name} N={frame.n} k={frame.n_species} bins={frame.n_bins}", flush=True)
    ref = oracle.frame_histogram(frame)
    h, oor = run_gpu(ctx, frame, 1)
    assert np.array_equal(h, ref.hist), \
        f"{frame.name}: {int((h != ref.hist).sum())} bins differ"
    assert np.array_equal(oor, ref.out_of_range)


@pytest.mark.parametrize("frame", CASES, ids=[f.name for f in CASES])
def test_fp32_edge_bound(ctx, frame):
    print(f"\n[case] {frame.name} fp32", flush=True)
    w = oracle.edge_window(frame.coords, frame.box, frame.r_max)
    ref = oracle.frame_histogram(frame, edge_window=w)
    h, oor = run_gpu(ctx, frame, 0)
    bad = fp32_bound_violations(h, ref.hist, ref.edges)
    bad += oor_bound_violations(oor, ref.out_of_range, ref.edges)
    assert not bad, f"{frame.name}: " + "; ".join(bad[:5])


def test_sync_api_matches_async(ctx):
    import paper_1808_01478_amd as dh
    fr = CASES[2]
    for prec in (0, 1):
        a = dh.histo(fr.coords, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, prec)
        b, _ = run_gpu(ctx, fr, prec)
        assert np.array_equal(a, b)


def test_repeatable_and_stream_independent(ctx):
    import torch
    fr = CASES[8]
    first = run_gpu(ctx, fr, 0)[0]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        second = run_gpu(ctx, fr, 0, stream=s)[0]
    third = run_gpu(ctx, fr, 0)[0]
    assert np.array_equal(first, second) and np.array_equal(first, third)


def test_empty_and_single(ctx):
    import paper_1808_01478_amd as dh
    h = dh.histo(np.zeros((0, 3)), [0, 0], 0, None, 1.0, 8, 0)
    assert h.shape == (1, 8) and not h.any()
    h = dh.histo(np.zeros((1, 3)), [0, 1, 1], 1, np.eye(3) * 5, 1.0, 8, 1)
    assert h.shape == (3, 8) and not h.any()


@pytest.mark.parametrize("box_type", [0, 1, 2])
def test_pair_t_matches_oracle(ctx, box_type):
    """Per-pair scaled distance: binary64 identical to the oracle (this pins
    the device sqrt as correctly rounded), binary32 within the window."""
    import torch
    if box_type == 2:
        fr = workloads.triclinic(n=50_000)
    elif box_type == 1:
        fr = workloads.ortho(n=50_000)
    else:
        fr = workloads.tiny()
    rng = np.random.Generator(np.random.PCG64(5 + box_type))
    m = 400_000
    pi = rng.integers(0, fr.n, size=m)
    pj = rng.integers(0, fr.n, size=m)
    ref = oracle.pair_t(fr.coords, fr.box_type, fr.box, fr.r_max, fr.n_bins, pi, pj)
    dev = torch.device("cuda")
    x = torch.from_numpy(fr.coords).to(dev)
    dpi = torch.from_numpy(pi.astype(np.int32)).to(dev)
    dpj = torch.from_numpy(pj.astype(np.int32)).to(dev)
    t = torch.empty(m, dtype=torch.float64, device=dev)
    ctx.pair_t_async(x, fr.box_type, fr.box, fr.r_max, fr.n_bins, 1, dpi, dpj, t)
    torch.cuda.synchronize()
    t64 = t.cpu().numpy()
    assert np.array_equal(t64, ref), f"{int((t64 != ref).sum())} of {m} differ"
    ctx.pair_t_async(x, fr.box_type, fr.box, fr.r_max, fr.n_bins, 0, dpi, dpj, t)
    torch.cuda.synchronize()
    t32 = t.cpu().numpy()
    win = oracle.edge_window(fr.coords, fr.box, fr.r_max) * fr.n_bins / fr.r_max
    err = np.abs(t32 - ref)
    assert err.max() <= win, f"max |t32 - t64| = {err.max():.3g} > window {win:.3g}"


def test_sqrt_exact_on_perfect_squares(ctx):
    import torch
    rng = np.random.Generator(np.random.PCG64(9))
    # integer points: q is an integer; t = sqrt(q) * 1 exactly when n_bins = r_max
    x = rng.integers(0, 1 << 20, size=(4096, 3)).astype(np.float64)
    r_max = float(1 << 22)
    i, j = np.triu_indices(4096, 1)
    sel = rng.choice(len(i), 500_000, replace=False)
    pi, pj = i[sel], j[sel]
    ref = oracle.pair_t(x, 0, None, r_max, int(r_max), pi, pj)
    dev = torch.device("cuda")
    t = torch.empty(len(pi), dtype=torch.float64, device=dev)
    ctx.pair_t_async(torch.from_numpy(x).to(dev), 0, None, r_max, int(r_max), 1,
                     torch.from_numpy(pi.astype(np.int32)).to(dev),
                     torch.from_numpy(pj.astype(np.int32)).to(dev), t)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    assert np.array_equal(got, ref)
    d = x[pj] - x[pi]
    q = (d * d).sum(axis=1)
    sq = np.array([math.isqrt(int(v)) for v in q])
    perfect = sq * sq == q
    assert np.array_equal(got[perfect], sq[perfect].astype(np.float64))


def test_sqrt_wide_range_and_mixed_waves(ctx):
    """binary64 per-pair t against the oracle for squared distances from
    1e-300 to 1e300: waves mix lanes that take the fast square root with
    lanes that need the library path (tiny, zero), and every result must be
    bit-identical to the correctly rounded oracle."""
    import torch
    rng = np.random.Generator(np.random.PCG64(17))
    m = 1 << 16
    mant = rng.uniform(1.0, 2.0, size=(m, 3))
    expo = rng.integers(-500, 500, size=(m, 1))
    pts = np.ldexp(mant * rng.choice([-1.0, 1.0], size=(m, 3)), expo)
    pts[rng.random(m) < 0.05] = 0.0                      # exact zeros: q = 0
    coords = np.concatenate([np.zeros((1, 3)), pts])
    pi = np.zeros(m, np.int64)
    pj = np.arange(1, m + 1, dtype=np.int64)
    r_max, n_bins = 1.0, 1 << 20
    ref = oracle.pair_t(coords, 0, None, r_max, n_bins, pi, pj)
    dev = torch.device("cuda")
    t = torch.empty(m, dtype=torch.float64, device=dev)
    ctx.pair_t_async(torch.from_numpy(coords).to(dev), 0, None, r_max, n_bins, 1,
                     torch.from_numpy(pi.astype(np.int32)).to(dev),
                     torch.from_numpy(pj.astype(np.int32)).to(dev), t)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    assert np.array_equal(got, ref, equal_nan=True), f"{int((got != ref).sum())} differ"
