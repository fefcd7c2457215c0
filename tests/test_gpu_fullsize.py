"""The full-size workloads in the launch configuration that bench.py times.

ortho100k (N=100,000, 2 species, 10,000 bins): binary64 bit-exact against the
oracle over all 4,999,950,000 pairs (run here), binary32 within the edge-pair
bound. triclinic1M (N=1,000,000 clustered, 3 species, 20,000 bins,
499,999,500,000 pairs) and the image-search frame (N=200,000 in a skewed
cell, r_max = 0.8 of the smallest width, the 27-image search running): against
the oracle's full histograms, out-of-range and edge counts stored in
tests/golden/ (written by tests/golden/make_golden.py, which calls only the
oracle), binary64 bit for bit and binary32 within the per-edge bound; plus
sampled pairs one by one.

The device's out-of-range counts are its pair count less the flushed in-range
counts, so bins + out-of-range = pairs holds by construction and is not used
as evidence here."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import fp32_bound_violations, oor_bound_violations, run_gpu
from golden.make_golden import input_hash, load as load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.close()


def test_ortho100k_full(ctx):
    fr = workloads.ortho()
    print(f"\n[case] ortho100k oracle ({oracle.max_threads()} threads)", flush=True)
    w = oracle.edge_window(fr.coords, fr.box, fr.r_max)
    ref = oracle.frame_histogram(fr, edge_window=w)
    print("[case] ortho100k gpu fp64", flush=True)
    h64, oor64 = run_gpu(ctx, fr, 1)
    assert np.array_equal(h64, ref.hist)
    assert np.array_equal(oor64, ref.out_of_range)
    print("[case] ortho100k gpu fp32", flush=True)
    h32, oor32 = run_gpu(ctx, fr, 0)
    bad = fp32_bound_violations(h32, ref.hist, ref.edges)
    bad += oor_bound_violations(oor32, ref.out_of_range, ref.edges)
    assert not bad, "; ".join(bad[:5])


def _against_golden(ctx, fr, name):
    """Binary64 bit-exact and binary32 within the edge-pair bound against the
    stored oracle result of workload `name`."""
    g = load_golden(name)
    assert str(g["input_sha256"][0]) == input_hash(fr), \
        f"{name}: the generated input differs from the one the stored oracle result was made from"
    print(f"\n[case] {name} gpu fp64 against the stored oracle result", flush=True)
    h64, oor64 = run_gpu(ctx, fr, 1)
    assert np.array_equal(h64, g["hist"]), f"{name}: {int((h64 != g['hist']).sum())} bins differ"
    assert np.array_equal(oor64, g["oor"])
    print(f"[case] {name} gpu fp32 against the edge-pair bound", flush=True)
    h32, oor32 = run_gpu(ctx, fr, 0)
    bad = fp32_bound_violations(h32, g["hist"], g["edges"])
    bad += oor_bound_violations(oor32, g["oor"], g["edges"])
    assert not bad, f"{name}: " + "; ".join(bad[:5])


def test_triclinic1m_full(ctx):
    fr = workloads.triclinic()
    _against_golden(ctx, fr, "triclinic1M")
    # sampled pairs of the full frame, one by one: binary64 scaled distances
    # equal to the oracle's, binary32 within the edge window
    import torch
    print("[case] triclinic1M sampled pairs", flush=True)
    rng = np.random.Generator(np.random.PCG64(41))
    m = 200_000
    pi = rng.integers(0, fr.n, size=m)
    pj = rng.integers(0, fr.n, size=m)
    t_ref = oracle.pair_t(fr.coords, fr.box_type, fr.box, fr.r_max, fr.n_bins, pi, pj)
    dev = torch.device("cuda")
    x = torch.from_numpy(fr.coords).to(dev)
    dpi = torch.from_numpy(pi.astype(np.int32)).to(dev)
    dpj = torch.from_numpy(pj.astype(np.int32)).to(dev)
    t = torch.empty(m, dtype=torch.float64, device=dev)
    ctx.pair_t_async(x, fr.box_type, fr.box, fr.r_max, fr.n_bins, 1, dpi, dpj, t)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), t_ref)
    ctx.pair_t_async(x, fr.box_type, fr.box, fr.r_max, fr.n_bins, 0, dpi, dpj, t)
    torch.cuda.synchronize()
    win = oracle.edge_window(fr.coords, fr.box, fr.r_max) * fr.n_bins / fr.r_max
    assert np.abs(t.cpu().numpy() - t_ref).max() <= win


def test_image_search_full(ctx):
    import torch
    fr = workloads.image_search()
    _against_golden(ctx, fr, "image_search200k")
    # the kernel's search counts of that last (binary32) call: some but not
    # all pairs are searched, each over at least its octant list (7 images
    # for this cell) and at most all 27
    torch.cuda.synchronize()
    searched, images = ctx.searched_pairs(), ctx.searched_images()
    assert 0 < searched < fr.total_pairs()
    assert 7 * searched <= images <= 27 * searched, (searched, images)
    # sampled pairs of the full frame (searched images included), one by one
    print("[case] image search sampled pairs", flush=True)
    rng = np.random.Generator(np.random.PCG64(43))
    m = 100_000
    pi = rng.integers(0, fr.n, size=m)
    pj = rng.integers(0, fr.n, size=m)
    t_ref = oracle.pair_t(fr.coords, fr.box_type, fr.box, fr.r_max, fr.n_bins, pi, pj)
    dev = torch.device("cuda")
    x = torch.from_numpy(fr.coords).to(dev)
    dpi = torch.from_numpy(pi.astype(np.int32)).to(dev)
    dpj = torch.from_numpy(pj.astype(np.int32)).to(dev)
    t = torch.empty(m, dtype=torch.float64, device=dev)
    ctx.pair_t_async(x, fr.box_type, fr.box, fr.r_max, fr.n_bins, 1, dpi, dpj, t)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), t_ref)
    ctx.pair_t_async(x, fr.box_type, fr.box, fr.r_max, fr.n_bins, 0, dpi, dpj, t)
    torch.cuda.synchronize()
    win = oracle.edge_window(fr.coords, fr.box, fr.r_max) * fr.n_bins / fr.r_max
    assert np.abs(t.cpu().numpy() - t_ref).max() <= win
