"""The CPU oracle against its pins (exact brute force, closed forms,
invariants, special cases, the ideal-gas law). No GPU needed."""
import numpy as np
import pytest

import oracle
import pins
import workloads


@pytest.fixture(scope="module")
def lib(oracle_lib):
    return oracle.load()


@pytest.mark.parametrize("name", [c[0] for c in pins.exact_cases()])
def test_exact_bruteforce(lib, name):
    pins.pin_exact(lib, names={name})


def test_crafted_integer_distances(lib):
    pins.pin_crafted(lib)


def test_pair_counts(lib):
    pins.pin_pair_counts(lib)


def test_partition_and_relabel(lib):
    pins.pin_partition(lib)


def test_special_boxes(lib):
    pins.pin_special_boxes(lib)


def test_image_search(lib):
    pins.pin_images(lib)


def test_ideal_gas(lib):
    pins.pin_ideal_gas(lib)


def test_tiny_all_pairs_in_range(lib):
    # every distance in [0,10)^3 is below 10*sqrt(3) = r_max
    fr = workloads.tiny()
    r = oracle.frame_histogram(fr)
    assert int(r.hist.sum()) == 12_497_500 and int(r.out_of_range[0]) == 0


def test_pair_t_matches_histogram(lib):
    fr = workloads.random_frame(77, [60], workloads.BOX_TRICLINIC, n_bins=50)
    i, j = np.triu_indices(60, 1)
    t = oracle.pair_t(fr.coords, fr.box_type, fr.box, fr.r_max, fr.n_bins, i, j)
    h = np.bincount(t[t < fr.n_bins].astype(np.int64), minlength=fr.n_bins)
    assert np.array_equal(h, oracle.frame_histogram(fr).hist[0].astype(np.int64))


def test_edge_counts(lib):
    fr = workloads.random_frame(78, [80, 40], workloads.BOX_ORTHO, n_bins=30)
    w = 1e-3
    r = oracle.frame_histogram(fr, edge_window=w)
    # direct count of |t - k| <= w*s from per-pair t
    s = fr.n_bins / fr.r_max
    offs = fr.offsets
    pairs = [(np.triu_indices(80, 1)), None, None]
    i0, j0 = np.triu_indices(80, 1)
    i1, j1 = np.triu_indices(40, 1)
    i2, j2 = np.meshgrid(np.arange(80), np.arange(80, 120), indexing="ij")
    for h, (pi, pj) in enumerate([(i0, j0), (i1 + 80, j1 + 80), (i2.ravel(), j2.ravel())]):
        t = oracle.pair_t(fr.coords, fr.box_type, fr.box, fr.r_max, fr.n_bins, pi, pj)
        want = np.zeros(fr.n_bins, np.int64)
        for k in range(1, fr.n_bins + 1):
            want[k - 1] = int(np.sum(np.abs(t - k) <= w * s))
        assert np.array_equal(r.edges[h].astype(np.int64), want)
    del pairs, offs


def test_invalid_arguments(lib):
    fr = workloads.random_frame(79, [10], workloads.BOX_ORTHO)
    with pytest.raises(ValueError):
        oracle.histogram(fr.coords, fr.offsets, 1, fr.box, -1.0, 10)
    bad = fr.box.copy(); bad[1, 0] = 0.5          # off-diagonal in an orthorhombic box
    with pytest.raises(ValueError):
        oracle.histogram(fr.coords, fr.offsets, 1, bad, 3.0, 10)
    with pytest.raises(ValueError):
        oracle.histogram(fr.coords, [0, 5, 3], 1, fr.box, 3.0, 10)


def test_edge_window_values():
    """The binary32 tolerance window 4 ulp32(S), S = max(max |coordinate|,
    max |box entry|, r_max): exact values on the three single-frame
    workloads (S = 10*sqrt(3), 40 and about 75), and on crafted S at and
    just below powers of two, against numpy's float32 spacing."""
    assert oracle.edge_window(workloads.tiny().coords, None, 10.0 * np.sqrt(3.0)) == 7.62939453125e-06
    fr = workloads.ortho(n=1000)
    assert oracle.edge_window(fr.coords, fr.box, fr.r_max) == 1.52587890625e-05
    fr = workloads.triclinic(n=20_000)
    assert oracle.edge_window(fr.coords, fr.box, fr.r_max) == 3.0517578125e-05
    pts = np.zeros((2, 3))
    for e in (-3, 0, 4, 5, 9):
        s = 2.0 ** e
        below = np.nextafter(s, 0.0)
        # S exactly 2^e: ulp32 is the spacing of float32 at 2^e
        want = 4.0 * float(np.spacing(np.float32(s)))
        assert oracle.edge_window(pts, None, s) == want
        pts2 = pts.copy()
        pts2[1, 2] = -s                       # |coordinate| sets S, sign ignored
        assert oracle.edge_window(pts2, None, 0.5 * s) == want
        box = np.diag([0.25 * s, s, 0.5 * s])  # box entry sets S
        assert oracle.edge_window(pts, box, 0.125 * s) == want
        # S just below 2^e lies in the binade below: half the window
        assert oracle.edge_window(pts, None, below) == want / 2
        assert oracle.edge_window(pts, None, below) == 4.0 * float(np.spacing(np.float32(s / 2)))
