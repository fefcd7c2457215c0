"""The image lists of the 27-image search (dh_search_images, host logic of
the library): for each octant of a reduced vector's fractional coordinates
the kernels search only the listed images. Checked in exact rational
arithmetic on the cell's binary64 entries: every image left out of an
octant's list is farther than the vector itself at every vertex of the
octant's box (so, g being linear, everywhere in it), and on random points of
each octant the minimum over the list equals the minimum over all 27 images
(Sec. 2.3's neighbouring images)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import paper_1808_01478_amd as dh
import workloads

SHIFTS = list(itertools.product((-1, 0, 1), repeat=3))  # index m = 9(i+1) + 3(j+1) + (k+1)
ZERO = 13


def cells():
    out = {"orthogonal": workloads.ortho_box(9.0, 10.0, 11.0),
           "skew": np.array([[10.0, 0, 0], [3.0, 9.5, 0], [-2.0, 3.5, 9.0]]),
           "sheared": np.array([[9.0, 0, 0], [4.4, 8.0, 0], [-4.3, 3.9, 7.5]]),
           "triclinic1M": workloads.TRICLINIC_BOX.copy(),
           "image_search": workloads.image_search().box}
    rng = np.random.Generator(np.random.PCG64(77))
    for k in range(6):
        ax, by, cz = rng.uniform(5.0, 15.0, 3)
        out[f"random{k}"] = np.array([[ax, 0, 0],
                                      [rng.uniform(-0.5, 0.5) * ax, by, 0],
                                      [rng.uniform(-0.5, 0.5) * ax, rng.uniform(-0.5, 0.5) * by,
                                       cz]])
    return out


CELLS = cells()


def exact_rows(box):
    return [[Fraction(float(v)) for v in row] for row in box]


def cart(f, B):
    return [sum(f[r] * B[r][c] for r in range(3)) for c in range(3)]


def q_of(f, n, B):
    v = cart([f[k] + n[k] for k in range(3)], B)
    return sum(x * x for x in v)


@pytest.mark.parametrize("name", sorted(CELLS))
def test_left_out_images_are_farther(name):
    B = exact_rows(CELLS[name])
    lists, counts, full = dh.search_images(CELLS[name])
    half = Fraction(1, 2)
    for o in range(8):
        kept = set(int(m) for m in lists[o, :counts[o]])
        assert all(int(m) == ZERO for m in lists[o, counts[o]:])
        assert ZERO not in kept
        box = [(-half, Fraction(0)) if (o >> k) & 1 else (Fraction(0), half) for k in range(3)]
        for m, n in enumerate(SHIFTS):
            if m == ZERO or m in kept:
                continue
            # g(f) = |B(f + n)|^2 - |B f|^2 > 0 at every vertex of the octant
            for v in itertools.product(*box):
                assert q_of(v, n, B) > q_of(v, (0, 0, 0), B), (name, o, n, v)
        # octants searched in full are the ones with more than 12 images
        assert bool((full >> o) & 1) == (counts[o] > 12)


@pytest.mark.parametrize("name", sorted(CELLS))
def test_list_minimum_equals_full_minimum(name):
    B = exact_rows(CELLS[name])
    lists, counts, _ = dh.search_images(CELLS[name])
    rng = np.random.Generator(np.random.PCG64(5))
    for o in range(8):
        kept = [SHIFTS[int(m)] for m in lists[o, :counts[o]]]
        for _ in range(40):
            u = rng.uniform(0.0, 0.5, 3)
            f = [Fraction(float(-x if (o >> k) & 1 else x)) for k, x in enumerate(u)]
            full_min = min(q_of(f, n, B) for n in SHIFTS)
            list_min = min([q_of(f, (0, 0, 0), B)] + [q_of(f, n, B) for n in kept])
            assert list_min == full_min, (name, o, f)


def test_orthogonal_cell_keeps_the_seven_images_towards_the_vector():
    lists, counts, full = dh.search_images(CELLS["orthogonal"])
    assert full == 0
    for o in range(8):
        sign = [1 if (o >> k) & 1 else -1 for k in range(3)]
        want = sorted(9 * (i + 1) + 3 * (j + 1) + (k + 1)
                      for i in (0, sign[0]) for j in (0, sign[1]) for k in (0, sign[2])
                      if (i, j, k) != (0, 0, 0))
        assert sorted(int(m) for m in lists[o, :counts[o]]) == want


def test_lists_are_short_for_the_bench_cells():
    for name in ("image_search", "triclinic1M", "skew", "sheared"):
        _, counts, full = dh.search_images(CELLS[name])
        assert full == 0 and counts.max() <= 9, (name, counts)


def test_rejects_bad_boxes():
    with pytest.raises(dh.DisthistError):
        dh.search_images(np.array([[10.0, 0, 0], [6.0, 9.0, 0], [0.0, 0.0, 9.0]]))  # |bx| > ax/2
    with pytest.raises(dh.DisthistError):
        dh.search_images(np.array([[10.0, 1.0, 0], [0.0, 9.0, 0], [0.0, 0.0, 9.0]]))  # not lower-triangular
