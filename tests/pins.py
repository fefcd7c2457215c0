"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Each ``pin_*`` function takes an oracle handle (the ctypes library of the
oracle, or of a planted-mistake variant of it) and raises AssertionError when
the oracle disagrees with an independent statement of the result:

* exact rational brute force on tiny frames (nearest image by enumeration),
* crafted frames with integer distances (closed forms),
* the pair-count identity of Algorithm 1 and its single-species variant,
* species partition and relabelling identities,
* special boxes that reduce to simpler ones,
* the ideal-gas closed form for uniform points in a periodic cell.

``tests/test_oracle_pins.py`` runs them on the oracle; ``tests/test_oracle_mutants.py``
runs them on planted mistakes and requires each mistake to fail at least one.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import workloads
from exact_ref import exact_histogram

BOX_NONE, BOX_ORTHO, BOX_TRICLINIC = 0, 1, 2


def _run(lib, frame, **kw):
    return oracle.histogram(frame.coords, frame.offsets, frame.box_type, frame.box,
                            frame.r_max, frame.n_bins, lib=lib, **kw)


def _frame(coords, sizes, box_type, box, r_max, n_bins):
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return workloads.Frame(np.ascontiguousarray(np.asarray(coords, np.float64)), offs, box_type,
                           None if box is None else np.asarray(box, np.float64), float(r_max),
                           int(n_bins))


# --------------------------------------------------------------------------- #
# exact brute force
# --------------------------------------------------------------------------- #

SKEW_BOX = np.array([[10.0, 0, 0], [3.0, 9.5, 0], [-2.0, 3.5, 9.0]])


def exact_cases():
    """(name, frame, reach) for the exact brute-force pins."""
    rng = np.random.Generator(np.random.PCG64(11))
    out = []
    out.append(("none", workloads.random_frame(101, [9, 6, 7], BOX_NONE, r_max=9.0, n_bins=17), 0))
    x = rng.uniform(-20, 20, size=(14, 3))
    out.append(("none-wide", _frame(x, [8, 6], BOX_NONE, None, 30.0, 11), 0))
    out.append(("ortho", workloads.random_frame(102, [8, 7], BOX_ORTHO, r_max=4.4, n_bins=23), 3))
    box = workloads.ortho_box(10.0, 9.0, 11.0)
    x = rng.uniform(-15, 25, size=(13, 3))
    out.append(("ortho-unwrapped-long", _frame(x, [6, 7], BOX_ORTHO, box, 8.5, 19), 5))
    out.append(("tric", workloads.random_frame(103, [10, 8], BOX_TRICLINIC, box=SKEW_BOX,
                                               r_max=0.45 * workloads.min_width(SKEW_BOX),
                                               n_bins=21), 3))
    out.append(("tric-search", workloads.random_frame(104, [9, 7], BOX_TRICLINIC, box=SKEW_BOX,
                                                      r_max=0.75 * workloads.min_width(SKEW_BOX),
                                                      n_bins=15), 3))
    tb = workloads.TRICLINIC_BOX
    x = rng.uniform(0, 1, size=(15, 3)) @ tb
    out.append(("tric-c3box", _frame(x, [5, 4, 6], BOX_TRICLINIC, tb, 22.0, 40), 3))
    x = rng.uniform(0, 1, size=(12, 3)) @ tb
    out.append(("tric-c3box-search", _frame(x, [12], BOX_TRICLINIC, tb, 27.0, 9), 3))
    x = rng.uniform(-1.5, 2.5, size=(12, 3)) @ SKEW_BOX
    out.append(("tric-unwrapped", _frame(x, [7, 5], BOX_TRICLINIC, SKEW_BOX,
                                         0.4 * workloads.min_width(SKEW_BOX), 13), 4))
    return out


def pin_exact(lib, names=None):
    for name, fr, reach in exact_cases():
        if names and name not in names:
            continue
        ref_h, ref_o, near = exact_histogram(fr.coords, fr.offsets, fr.box, fr.r_max, fr.n_bins,
                                             reach=reach)
        assert near == 0, f"{name}: {near} pairs within 1e-9 of an edge (choose another seed)"
        got = _run(lib, fr)
        assert np.array_equal(got.hist, ref_h), f"{name}: histogram differs from exact brute force"
        assert np.array_equal(got.out_of_range, ref_o), f"{name}: out-of-range differs"


# --------------------------------------------------------------------------- #
# crafted integer distances (closed forms)
# --------------------------------------------------------------------------- #

def crafted_cases():
    """(name, frame, expected {(h, bin): count}, expected out_of_range per h)."""
    cases = []
    # Pythagorean quadruples: |v| is an integer, so with n_bins = r_max (dr = 1)
    # every pair lands exactly on the lower edge of bin |v| (half-open bins).
    vecs = [((3, 4, 0), 5), ((1, 2, 2), 3), ((2, 3, 6), 7), ((1, 4, 8), 9),
            ((2, 6, 9), 11), ((0, 0, 0), 0), ((0, 0, 12), 12)]
    for v, r in vecs:
        base = np.array([1.0, -2.0, 0.5])
        x = np.array([base, base + np.array(v, float)])
        fr = _frame(x, [2], BOX_NONE, None, 12.0, 12)
        exp = {} if r >= 12 else {(0, r): 1}
        cases.append((f"vec{v}", fr, exp, [1 if r >= 12 else 0]))
        # dr = 1/2: bin 2r
        fr2 = _frame(x, [2], BOX_NONE, None, 12.0, 24)
        exp2 = {} if r >= 12 else {(0, 2 * r): 1}
        cases.append((f"vec{v}-half", fr2, exp2, [1 if r >= 12 else 0]))
    # orthorhombic minimum image: separation 17 along x in a 20-box is 3
    box = workloads.ortho_box(20.0, 30.0, 40.0)
    x = np.array([[1.0, 1.0, 1.0], [18.0, 1.0, 1.0], [1.0, 27.0, 37.0]])
    # pairs: (0,1): 3 ; (0,2): (0,-4,-4)... -> d=(0,26,36) -> (0,-4,-4): sqrt(32)
    # (1,2): (-17,26,36) -> (3,-4,-4): sqrt(41)
    fr = _frame(x, [3], BOX_ORTHO, box, 10.0, 10)
    cases.append(("ortho-mic", fr, {(0, 3): 1, (0, 5): 1, (0, 6): 1}, [0]))
    # triclinic reduction: a=(10,0,0) b=(4,10,0) c=(0,0,10); d=(7,14,0) reduces to (3,4,0)
    tb = np.array([[10.0, 0, 0], [4.0, 10.0, 0], [0, 0, 10.0]])
    x = np.array([[0.0, 0.0, 0.0], [7.0, 14.0, 0.0]])
    fr = _frame(x, [1, 1], BOX_TRICLINIC, tb, 4.75, 19)  # dr = 0.25: bin 20 -> out of range
    cases.append(("tric-mic-oor", fr, {}, [0, 0, 1]))
    fr = _frame(x, [1, 1], BOX_TRICLINIC, tb, 5.0, 20)   # dr = 0.25: bin 20 -> r = r_max: out
    cases.append(("tric-mic-edge", fr, {}, [0, 0, 1]))
    fr = _frame(x, [1, 1], BOX_TRICLINIC, tb, 6.0, 24)   # dr = 0.25: bin 20
    cases.append(("tric-mic", fr, {(2, 20): 1}, [0, 0, 0]))
    return cases


def pin_crafted(lib):
    for name, fr, exp, exp_oor in crafted_cases():
        got = _run(lib, fr)
        want = np.zeros_like(got.hist)
        for (h, b), c in exp.items():
            want[h, b] = c
        assert np.array_equal(got.hist, want), f"{name}: {np.argwhere(got.hist)} != {exp}"
        assert list(got.out_of_range) == exp_oor, f"{name}: out of range {got.out_of_range}"


# --------------------------------------------------------------------------- #
# invariants and identities
# --------------------------------------------------------------------------- #

def pin_pair_counts(lib):
    for fr in [workloads.random_frame(201, [50, 1, 0, 37], BOX_NONE, r_max=5.0, n_bins=33),
               workloads.random_frame(202, [41, 29], BOX_ORTHO, n_bins=50),
               workloads.random_frame(203, [20, 33, 17], BOX_TRICLINIC, n_bins=40),
               workloads.random_frame(204, [60], BOX_TRICLINIC, box=SKEW_BOX,
                                      r_max=0.8 * workloads.min_width(SKEW_BOX), n_bins=40)]:
        got = _run(lib, fr)
        tot = got.hist.sum(axis=1) + got.out_of_range
        assert list(tot) == fr.hist_pairs(), f"{fr.name}: pair counts {list(tot)} != {fr.hist_pairs()}"
    # every pair in range: the whole N(N-1)/2 lands in the histogram
    fr = workloads.tiny(n=400)
    got = _run(lib, fr)
    assert int(got.hist.sum()) == 400 * 399 // 2 and int(got.out_of_range[0]) == 0


def pin_partition(lib):
    for bt in (BOX_NONE, BOX_ORTHO, BOX_TRICLINIC):
        fr = workloads.random_frame(300 + bt, [45, 35], bt, n_bins=37)
        split = _run(lib, fr)
        union = _run(lib, _frame(fr.coords, [80], bt, fr.box, fr.r_max, fr.n_bins))
        assert np.array_equal(union.hist[0], split.hist.sum(axis=0)), f"box {bt}: partition"
        # relabelling: swapping the two species permutes the histograms
        sw = np.concatenate([fr.coords[45:], fr.coords[:45]])
        swapped = _run(lib, _frame(sw, [35, 45], bt, fr.box, fr.r_max, fr.n_bins))
        assert np.array_equal(swapped.hist[0], split.hist[1])
        assert np.array_equal(swapped.hist[1], split.hist[0])
        assert np.array_equal(swapped.hist[2], split.hist[2]), f"box {bt}: cross relabel"
        # permuting points inside a species leaves everything unchanged
        p = np.random.Generator(np.random.PCG64(bt)).permutation(45)
        perm = np.concatenate([fr.coords[:45][p], fr.coords[45:]])
        pr = _run(lib, _frame(perm, [45, 35], bt, fr.box, fr.r_max, fr.n_bins))
        assert np.array_equal(pr.hist, split.hist), f"box {bt}: permutation"


def pin_special_boxes(lib):
    # a periodic box much larger than the point cloud is the non-periodic case
    fr = workloads.random_frame(401, [30, 25], BOX_NONE, r_max=12.0, n_bins=29)
    big = _frame(fr.coords, [30, 25], BOX_ORTHO, workloads.ortho_box(100.0, 200.0, 300.0),
                 fr.r_max, fr.n_bins)
    assert np.array_equal(_run(lib, fr).hist, _run(lib, big).hist), "big ortho != none"
    # a triclinic cell with zero off-diagonal entries is the orthorhombic cell
    for r_max in (4.0, 7.0):   # without and with the image search
        fo = workloads.random_frame(402, [33, 21], BOX_ORTHO, r_max=r_max, n_bins=31)
        ft = _frame(fo.coords, [33, 21], BOX_TRICLINIC, fo.box, fo.r_max, fo.n_bins)
        a, b = _run(lib, fo), _run(lib, ft)
        assert np.array_equal(a.hist, b.hist) and np.array_equal(a.out_of_range, b.out_of_range), \
            f"diagonal triclinic != ortho at r_max={r_max}"


def pin_images(lib):
    # below half the minimum width, the reduction alone is the nearest image
    w = workloads.min_width(SKEW_BOX)
    fr = workloads.random_frame(501, [70], BOX_TRICLINIC, box=SKEW_BOX, r_max=0.49 * w, n_bins=40)
    assert np.array_equal(_run(lib, fr).hist, _run(lib, fr, image_mode=oracle.IMAGES_125).hist)
    # beyond it, 27 neighbours of the reduced vector reach the nearest image
    fr = workloads.random_frame(502, [70], BOX_TRICLINIC, box=SKEW_BOX, r_max=0.9 * w, n_bins=40)
    a = _run(lib, fr)
    b = _run(lib, fr, image_mode=oracle.IMAGES_125)
    assert np.array_equal(a.hist, b.hist) and np.array_equal(a.out_of_range, b.out_of_range)


# --------------------------------------------------------------------------- #
# ideal gas
# --------------------------------------------------------------------------- #

def ideal_gas_check(hist, pairs, edges, volume, z_max=6.0):
    """Uniform iid points in a periodic cell, bins inside w_min/2: the bin
    count is a sum of pairwise independent Bernoulli variables (difference
    vectors of distinct pairs are independent on the torus), so
    E = P p, Var = P p (1-p), p = 4/3 pi (e_hi^3 - e_lo^3) / V."""
    p = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3) / volume
    mean = pairs * p
    sd = np.sqrt(pairs * p * (1 - p))
    z = (hist.astype(np.float64) - mean) / sd
    chi2 = float(np.sum(z * z))
    return z, chi2


def pin_ideal_gas(lib):
    for bt, box in ((BOX_ORTHO, workloads.ortho_box(12.0, 10.0, 11.0)), (BOX_TRICLINIC, SKEW_BOX)):
        rng = np.random.Generator(np.random.PCG64(600 + bt))
        n = 3000
        x = rng.uniform(0, 1, size=(n, 3)) @ box
        r_max = 0.5 * workloads.min_width(box)
        nb = 40
        fr = _frame(x, [1800, 1200], bt, box, r_max, nb)
        got = _run(lib, fr)
        vol = abs(float(np.linalg.det(box)))
        edges = np.linspace(0, r_max, nb + 1)
        for h, pairs in enumerate(fr.hist_pairs()):
            z, chi2 = ideal_gas_check(got.hist[h], pairs, edges, vol)
            assert np.max(np.abs(z)) < 6.0, f"box {bt} h{h}: max |z| = {np.max(np.abs(z)):.2f}"
            # chi2 with nb dof: mean nb, sd sqrt(2 nb); 8 sd is far out
            assert chi2 < nb + 8 * math.sqrt(2 * nb), f"box {bt} h{h}: chi2 = {chi2:.1f}"


ALL_PINS = [pin_exact, pin_crafted, pin_pair_counts, pin_partition, pin_special_boxes,
            pin_images, pin_ideal_gas]
