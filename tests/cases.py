"""Seeded frames shared by the GPU parity tests: every box kind, ragged and
empty species, unwrapped coordinates, r_max beyond half the cell, image
search, clustered points, bin windows, coincident points, all pairs out of
range, a single bin, and a trajectory frame."""
import numpy as np

import workloads

SKEW = np.array([[10.0, 0, 0], [3.0, 9.5, 0], [-2.0, 3.5, 9.0]])


def _frame(coords, sizes, box_type, box, r_max, n_bins, name):
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return workloads.Frame(np.ascontiguousarray(coords, np.float64), offs, box_type,
                           None if box is None else np.asarray(box, np.float64), float(r_max),
                           int(n_bins), name)


def parity_cases():
    rng = np.random.Generator(np.random.PCG64(2024))
    out = [workloads.tiny()]
    out.append(workloads.random_frame(11, [2500, 1, 0, 1337], workloads.BOX_NONE, r_max=12.0,
                                      n_bins=97))
    out[-1].name = "none-4species-ragged"
    out.append(workloads.random_frame(12, [3001, 2047], workloads.BOX_ORTHO, n_bins=1000))
    out[-1].name = "ortho-2species"
    box = workloads.ortho_box(10.0, 11.0, 12.0)
    out.append(_frame(rng.uniform(-30, 50, size=(2900, 3)), [1900, 1000], workloads.BOX_ORTHO,
                      box, 5.9, 500, "ortho-unwrapped"))
    out.append(_frame(rng.uniform(0, 10, size=(2100, 3)), [2100], workloads.BOX_ORTHO,
                      workloads.ortho_box(10.0, 10.0, 10.0), 8.0, 333, "ortho-beyond-half"))
    out.append(workloads.random_frame(13, [2600, 900], workloads.BOX_TRICLINIC, n_bins=777))
    out[-1].name = "tric-2species"
    w = workloads.min_width(SKEW)
    out.append(workloads.random_frame(14, [1500, 700], workloads.BOX_TRICLINIC, box=SKEW,
                                      r_max=0.8 * w, n_bins=300))
    out[-1].name = "tric-search"
    x = rng.uniform(-1.5, 2.5, size=(1800, 3)) @ SKEW
    out.append(_frame(x, [1000, 800], workloads.BOX_TRICLINIC, SKEW, 0.45 * w, 256,
                      "tric-unwrapped"))
    c3 = workloads.triclinic(n=6000)
    c3.name = "tric-clustered-6k"
    out.append(c3)
    out.append(workloads.random_frame(15, [2000, 1000], workloads.BOX_ORTHO, n_bins=50_000))
    out[-1].name = "ortho-50k-bins-sweeps"
    out.append(workloads.random_frame(16, [1700], workloads.BOX_NONE, r_max=17.3,
                                      n_bins=90_001))
    out[-1].name = "none-90001-bins-sweeps"
    out.append(_frame(np.tile([[1.5, 2.5, 3.5]], (3000, 1)), [3000], workloads.BOX_NONE, None,
                      1.0, 64, "coincident"))
    out.append(workloads.random_frame(17, [1200, 800], workloads.BOX_NONE, r_max=1e-3,
                                      n_bins=10))
    out[-1].name = "all-out-of-range"
    out.append(workloads.random_frame(18, [900, 1100], workloads.BOX_ORTHO, n_bins=1))
    out[-1].name = "one-bin"
    tr = workloads.trajectory_frame(7)
    out.append(tr.subset([4000] * tr.n_species))
    # image search: nearly every pair needs it (r_max close to the longest
    # reduced vector of a strongly skewed cell)
    sheared = np.array([[9.0, 0, 0], [4.4, 8.0, 0], [-4.3, 3.9, 7.5]])
    out.append(workloads.random_frame(19, [1400, 900], workloads.BOX_TRICLINIC, box=sheared,
                                      r_max=0.98 * workloads.min_width(sheared) * 1.2,
                                      n_bins=400))
    out[-1].name = "tric-search-sheared"
    # an orthogonal cell given as triclinic, beyond half its width: every
    # image lies on a tie boundary of the reduced cube
    out.append(workloads.random_frame(20, [1600], workloads.BOX_TRICLINIC,
                                      box=workloads.ortho_box(9.0, 10.0, 11.0), r_max=7.0,
                                      n_bins=350))
    out[-1].name = "tric-search-orthogonal"
    # a dyadic lattice of points in a dyadic cell: many fractional
    # differences are exactly +-1/2, and many distances repeat exactly
    cell = np.array([[8.0, 0, 0], [2.0, 8.0, 0], [-2.0, 2.0, 8.0]])
    grid = np.stack(np.meshgrid(*[np.arange(8) / 8.0] * 3, indexing="ij"), -1).reshape(-1, 3)
    out.append(_frame(grid @ cell, [300, len(grid) - 300], workloads.BOX_TRICLINIC, cell,
                      0.75 * workloads.min_width(cell), 97, "tric-search-lattice-ties"))
    # triclinic frames of at least 65,536 points are staged in spatial order
    # and take the group-shift path: a clustered frame, and unwrapped uniform
    # points with a one-point species
    c3s = workloads.triclinic(n=70_000)
    c3s.name = "tric-clustered-70k-sorted"
    out.append(c3s)
    xs = rng.uniform(-1.0, 2.0, size=(66_001, 3)) @ SKEW
    out.append(_frame(xs, [40_000, 1, 26_000], workloads.BOX_TRICLINIC, SKEW, 0.49 * w, 600,
                      "tric-unwrapped-66k-sorted"))
    # no box, coordinates over 800 binary orders of magnitude: squared
    # distances from zero and subnormals to overflow, so the short root's
    # guard (tiny q, t near bin edges, t far out of range) runs in every wave
    mant = rng.uniform(1.0, 2.0, size=(3000, 3)) * rng.choice([-1.0, 1.0], size=(3000, 3))
    xw = np.ldexp(mant, rng.integers(-400, 400, size=(3000, 1)))
    xw[rng.random(3000) < 0.02] = 0.0
    out.append(_frame(xw, [1700, 1300], workloads.BOX_NONE, None, 1.0, 4096,
                      "none-wide-magnitudes"))
    # binary64 orthorhombic frames of at least 65,536 points take the sorted
    # kernel with a diagonal cell matrix: unwrapped points (shifts beyond one
    # cell), three species with a one-point species, r_max beyond half the
    # shortest edge
    xo = rng.uniform(-25.0, 45.0, size=(67_001, 3))
    out.append(_frame(xo, [30_000, 1, 37_000], workloads.BOX_ORTHO,
                      workloads.ortho_box(20.0, 23.0, 26.0), 11.0, 800,
                      "ortho-unwrapped-67k-sorted"))
    return out
