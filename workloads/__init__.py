"""Seeded synthetic inputs for the pair-distance histogram.

This module only draws coordinates, boxes and job parameters. It holds none of
the histogram arithmetic, so both the CPU oracle and the HIP path can consume
exactly the same bytes from it.

The benchmark inputs follow the paper's practice of pseudo-random particle
coordinates in a box (Sec. 4, opening paragraphs), scaled to these workloads:

* ``tiny``      1 frame, N=5,000 uniform in [0,10)^3, 1 species, no box,
                r_max = 10*sqrt(3), 1,000 bins.
* ``ortho``     1 frame, N=100,000 uniform in a 40^3 periodic box, species
                60,000/40,000, r_max = 20, 10,000 bins.
* ``triclinic`` 1 frame, N=1,000,000 in the cell a=(50,0,0), b=(15,48,0),
                c=(10,12,45): 70% from 64 Gaussian clusters (sigma=2),
                30% uniform; species 50/30/20 %; r_max = 22; 20,000 bins.
* ``trajectory`` 512 orthorhombic frames with N log-uniform in [1e4, 2e5],
                1-4 species, density 1.5625, r_max = half the shortest edge,
                4,096 bins.
* ``serving``   a Poisson stream of jobs with N log-uniform in [1e3, 2e6],
                box none/ortho/triclinic, 1-3 species, 1k/10k/50k bins.

Every generator uses numpy's PCG64 with the seed stated in its docstring.
Coordinates are C-contiguous float64 arrays of shape (N, 3), species are
contiguous blocks described by an int64 offsets array of length k+1, and a
box is a (3, 3) float64 array whose rows are the cell vectors a, b, c.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BOX_NONE = 0
BOX_ORTHO = 1
BOX_TRICLINIC = 2

FP32 = 0
FP64 = 1

# particle density shared by the trajectory and serving workloads (N / V of the
# 100,000-particle 40^3 frame)
DENSITY = 100_000 / 40.0**3


@dataclasses.dataclass
class Frame:
    """One histogram job: coordinates, species blocks, box and binning."""

    coords: np.ndarray          # (N, 3) float64, C-contiguous
    offsets: np.ndarray         # (k+1,) int64, offsets[0] = 0, offsets[k] = N
    box_type: int
    box: Optional[np.ndarray]   # (3, 3) float64 rows a, b, c, or None
    r_max: float
    n_bins: int
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_species(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_hist(self) -> int:
        k = self.n_species
        return k * (k + 1) // 2

    def species_sizes(self) -> List[int]:
        return [int(self.offsets[s + 1] - self.offsets[s]) for s in range(self.n_species)]

    def hist_pairs(self) -> List[int]:
        """Pairs per histogram in the library order: (0,0),(1,1),...,(k-1,k-1)
        first, then (s,t) with s<t lexicographically."""
        n = self.species_sizes()
        k = len(n)
        out = [n[s] * (n[s] - 1) // 2 for s in range(k)]
        for s in range(k):
            for t in range(s + 1, k):
                out.append(n[s] * n[t])
        return out

    def total_pairs(self) -> int:
        return sum(self.hist_pairs())

    def subset(self, per_species: List[int]) -> "Frame":
        """The first ``per_species[s]`` points of every species block."""
        parts, offs = [], [0]
        for s, m in enumerate(per_species):
            lo = int(self.offsets[s])
            m = min(m, int(self.offsets[s + 1]) - lo)
            parts.append(self.coords[lo:lo + m])
            offs.append(offs[-1] + m)
        return Frame(np.ascontiguousarray(np.concatenate(parts)), np.asarray(offs, np.int64),
                     self.box_type, self.box, self.r_max, self.n_bins, self.name + "-subset")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _offsets(sizes) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, np.int64))]).astype(np.int64)


def ortho_box(lx: float, ly: float, lz: float) -> np.ndarray:
    return np.array([[lx, 0.0, 0.0], [0.0, ly, 0.0], [0.0, 0.0, lz]], np.float64)


def rows_combine(u: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """u @ rows for (n, 3) @ (3, 3), written as elementwise products and sums
    (u0*r0 + u1*r1) + u2*r2 so that the bytes do not depend on which BLAS
    kernel the host CPU selects: stored expected values made on one machine
    must be reproducible on another."""
    u = np.asarray(u, np.float64)
    r = np.asarray(rows, np.float64)
    return (u[:, 0:1] * r[0] + u[:, 1:2] * r[1]) + u[:, 2:3] * r[2]


def min_width(box: np.ndarray) -> float:
    """Smallest distance between opposite faces of the cell (geometry of the
    input, used to pick workload cut-offs). Written with scalar arithmetic,
    not BLAS, so it is the same on every host."""
    a, b, c = ([float(t) for t in v] for v in np.asarray(box, np.float64))

    def cross(u, v):
        return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])

    def norm(u):
        return math.sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])

    bc, ca, ab = cross(b, c), cross(c, a), cross(a, b)
    vol = abs(a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2])
    return min(vol / norm(bc), vol / norm(ca), vol / norm(ab))


# --------------------------------------------------------------------------- #
# single-frame workloads
# --------------------------------------------------------------------------- #

def tiny(seed: int = 1, n: int = 5000) -> Frame:
    """N uniform points in [0,10)^3, one species, no box, r_max = 10*sqrt(3)
    (every pair in range), 1,000 bins. Seed 1."""
    x = _rng(seed).uniform(0.0, 10.0, size=(n, 3))
    return Frame(np.ascontiguousarray(x), _offsets([n]), BOX_NONE, None,
                 10.0 * math.sqrt(3.0), 1000, "tiny")


def ortho(seed: int = 2, n: int = 100_000, frac_a: float = 0.6,
          length: float = 40.0, r_max: float = 20.0, n_bins: int = 10_000) -> Frame:
    """N uniform points in a periodic cube of edge 40; species A = first 60 %,
    B = the rest (iid, so contiguous blocks are fine); r_max = 20; 10,000
    bins. Seed 2."""
    x = _rng(seed).uniform(0.0, length, size=(n, 3))
    na = int(round(n * frac_a))
    return Frame(np.ascontiguousarray(x), _offsets([na, n - na]), BOX_ORTHO,
                 ortho_box(length, length, length), r_max, n_bins, "ortho")


TRICLINIC_BOX = np.array([[50.0, 0.0, 0.0], [15.0, 48.0, 0.0], [10.0, 12.0, 45.0]], np.float64)


def triclinic(seed: int = 3, n: int = 1_000_000, n_centres: int = 64, sigma: float = 2.0,
              frac_background: float = 0.3, species=(0.5, 0.3, 0.2),
              r_max: float = 22.0, n_bins: int = 20_000) -> Frame:
    """Clustered points in the triclinic cell a=(50,0,0), b=(15,48,0),
    c=(10,12,45). 64 centres uniform in fractional coordinates; 70 % of the
    points are centre + N(0, sigma^2 I) (Cartesian), wrapped into the cell
    through fractional mod 1; 30 % are uniform in fractional coordinates.
    Species are drawn by a seeded permutation (50/30/20 %) and stably sorted
    into blocks. r_max = 22 < w_min/2 = 22.5; 20,000 bins. Seed 3."""
    rng = _rng(seed)
    rows = TRICLINIC_BOX                       # rows a, b, c (lower triangular)
    # inverse of the lower-triangular row matrix, written out: x = u @ rows
    # gives u = x @ inv
    (ax, _, _), (bx, by, _), (cx, cy, cz) = rows
    inv = np.array([[1.0 / ax, 0.0, 0.0],
                    [-bx / (ax * by), 1.0 / by, 0.0],
                    [(bx * cy - by * cx) / (ax * by * cz), -cy / (by * cz), 1.0 / cz]])
    n_bg = int(round(n * frac_background))
    n_cl = n - n_bg
    centres = rows_combine(rng.uniform(0.0, 1.0, size=(n_centres, 3)), rows)
    which = rng.integers(0, n_centres, size=n_cl)
    pts = centres[which] + rng.normal(0.0, sigma, size=(n_cl, 3))
    frac = rows_combine(pts, inv) % 1.0
    frac = np.concatenate([frac, rng.uniform(0.0, 1.0, size=(n_bg, 3))])
    frac = frac[rng.permutation(n)]
    x = rows_combine(frac, rows)
    counts = [int(round(n * f)) for f in species[:-1]]
    counts.append(n - sum(counts))
    labels = rng.permutation(np.repeat(np.arange(len(counts)), counts))
    order = np.argsort(labels, kind="stable")
    return Frame(np.ascontiguousarray(x[order]), _offsets(counts), BOX_TRICLINIC,
                 TRICLINIC_BOX.copy(), r_max, n_bins, "triclinic")


# --------------------------------------------------------------------------- #
# many-frame workloads
# --------------------------------------------------------------------------- #

def _species_split(rng: np.random.Generator, n: int, k: int) -> List[int]:
    w = rng.dirichlet(np.ones(k))
    sizes = np.maximum(1, np.floor(w * (n - k)).astype(np.int64) + 1)
    sizes[-1] = n - int(sizes[:-1].sum())
    if sizes[-1] < 1:                     # pragma: no cover - guarded by the +1 above
        sizes = np.full(k, n // k)
        sizes[-1] = n - sizes[:-1].sum()
    return [int(v) for v in sizes]


def _aspect(rng: np.random.Generator) -> np.ndarray:
    f = rng.uniform(0.8, 1.25, size=3)
    return f / np.cbrt(np.prod(f))


def trajectory_frame(f: int, n_bins: int = 4096) -> Frame:
    """Frame f of the trajectory workload (seed 4000+f): N = floor(exp U(ln 1e4,
    ln 2e5)), 1-4 species with Dirichlet(1) fractions, orthorhombic box of
    volume N/1.5625 with aspect factors U[0.8,1.25], uniform coordinates,
    r_max = half the shortest edge, 4,096 bins."""
    rng = _rng(4000 + f)
    n = int(math.floor(math.exp(rng.uniform(math.log(1e4), math.log(2e5)))))
    k = int(rng.integers(1, 5))
    sizes = _species_split(rng, n, k)
    edge = (n / DENSITY) ** (1.0 / 3.0) * _aspect(rng)
    x = rng.uniform(0.0, 1.0, size=(n, 3)) * edge
    return Frame(np.ascontiguousarray(x), _offsets(sizes), BOX_ORTHO,
                 ortho_box(*edge), 0.5 * float(edge.min()), n_bins, f"traj{f}")


def trajectory(n_frames: int = 512, n_bins: int = 4096) -> List[Frame]:
    return [trajectory_frame(f, n_bins) for f in range(n_frames)]


def random_triclinic_cell(rng: np.random.Generator, volume: float) -> np.ndarray:
    """A reduced lower-triangular cell: diagonal from the cube edge times
    U[0.8,1.25] factors (renormalised to the volume), b_x, c_x ~ U(-a_x/2, a_x/2),
    c_y ~ U(-b_y/2, b_y/2)."""
    edge = volume ** (1.0 / 3.0) * _aspect(rng)
    ax, by, cz = (float(v) for v in edge)
    bx = float(rng.uniform(-ax / 2, ax / 2))
    cx = float(rng.uniform(-ax / 2, ax / 2))
    cy = float(rng.uniform(-by / 2, by / 2))
    return np.array([[ax, 0.0, 0.0], [bx, by, 0.0], [cx, cy, cz]], np.float64)


@dataclasses.dataclass
class Job:
    arrival_s: float
    frame: Frame
    job_id: int


def image_search(n: int = 200_000, seed: int = 31) -> Frame:
    """n uniform points (the bench density) in a skewed triclinic cell, the
    first 60 % one species and the rest another, r_max = 0.8 of the smallest
    cell width (so the 27-image search runs), 4,000 bins."""
    rng = _rng(seed)
    shape = np.array([[10.0, 0, 0], [3.0, 9.5, 0], [-2.0, 3.5, 9.0]])
    # lower triangular: the determinant is the product of the diagonal
    box = shape * (n / DENSITY / (shape[0, 0] * shape[1, 1] * shape[2, 2])) ** (1.0 / 3.0)
    x = rows_combine(rng.uniform(0.0, 1.0, size=(n, 3)), box)
    na = (n * 3) // 5
    return Frame(np.ascontiguousarray(x), _offsets([na, n - na]), BOX_TRICLINIC, box,
                 0.8 * min_width(box), 4000, f"image-search-{n}")


def serving_job(rng: np.random.Generator, job_id: int, arrival: float,
                n_lo: float = 1e3, n_hi: float = 2e6,
                bins=(1000, 10_000, 50_000)) -> Job:
    n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    box_type = int(rng.integers(0, 3))
    k = int(rng.integers(1, 4))
    k = min(k, n)
    sizes = _species_split(rng, n, k)
    n_bins = int(bins[int(rng.integers(0, len(bins)))])
    vol = n / DENSITY
    if box_type == BOX_NONE:
        edge = vol ** (1.0 / 3.0)
        x = rng.uniform(0.0, edge, size=(n, 3))
        box, r_max = None, edge * math.sqrt(3.0)
    elif box_type == BOX_ORTHO:
        edge = vol ** (1.0 / 3.0) * _aspect(rng)
        x = rng.uniform(0.0, 1.0, size=(n, 3)) * edge
        box, r_max = ortho_box(*edge), 0.5 * float(edge.min())
    else:
        box = random_triclinic_cell(rng, vol)
        x = rows_combine(rng.uniform(0.0, 1.0, size=(n, 3)), box)
        r_max = 0.49 * min_width(box)
    fr = Frame(np.ascontiguousarray(x), _offsets(sizes), box_type, box, float(r_max),
               n_bins, f"job{job_id}")
    return Job(arrival, fr, job_id)


def serving_trace(n_jobs: int, rate_hz: float, seed: int = 5, **kw) -> List[Job]:
    """Poisson arrivals at ``rate_hz`` (seed 5); see :func:`serving_job`."""
    rng = _rng(seed)
    t, jobs = 0.0, []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_hz))
        jobs.append(serving_job(rng, j, t, **kw))
    return jobs


# --------------------------------------------------------------------------- #
# small random frames for parity tests
# --------------------------------------------------------------------------- #

def random_frame(seed: int, sizes, box_type: int, r_max: Optional[float] = None,
                 n_bins: int = 64, box: Optional[np.ndarray] = None,
                 extent: float = 10.0) -> Frame:
    """Uniform points in the cell (or in [0, extent)^3 without a box)."""
    rng = _rng(seed)
    n = int(sum(sizes))
    if box_type == BOX_NONE:
        x = rng.uniform(0.0, extent, size=(n, 3))
        rm = extent * math.sqrt(3.0) if r_max is None else r_max
        bx = None
    else:
        if box is None:
            if box_type == BOX_ORTHO:
                box = ortho_box(extent, extent * 0.9, extent * 1.1)
            else:
                box = np.array([[extent, 0, 0], [0.3 * extent, 0.95 * extent, 0],
                                [-0.2 * extent, 0.35 * extent, 0.9 * extent]], np.float64)
        bx = np.asarray(box, np.float64)
        x = rows_combine(rng.uniform(0.0, 1.0, size=(n, 3)), bx)
        rm = 0.45 * min_width(bx) if r_max is None else r_max
    return Frame(np.ascontiguousarray(x), _offsets(sizes), box_type, bx, float(rm),
                 int(n_bins), f"rand{seed}")
