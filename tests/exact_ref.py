"""Exact-arithmetic brute force for tiny frames (test helper).

Every binary64 input is a dyadic rational, so after scaling all coordinates
and cell vectors by one common power of two they become Python integers and
squared distances are exact. The minimum image is found by plain enumeration
of lattice shifts n_a*a + n_b*b + n_c*c with |n| <= reach (the textbook
definition of the nearest image, not the reduction formula), and the bin is

    kappa = max{ k : (k * r_max / n_bins)^2 <= q }     (half-open bins)

decided exactly; the pair is in range iff kappa < n_bins. Pairs whose scaled
distance lies within ``edge_tol`` (relative) of a bin edge are reported
separately, because a correctly rounded FP64 evaluation may put them on
either side.

This module shares nothing with the oracle or the library: it is the
independent definition the oracle is pinned to.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from typing import List, Optional, Tuple

import numpy as np


def _common_scale(values) -> int:
    den = 1
    for v in values:
        d = Fraction(float(v)).denominator
        if d > den:
            den = d
    return den


def exact_histogram(coords, offsets, box: Optional[np.ndarray], r_max: float, n_bins: int,
                    reach: int = 3, edge_tol: float = 1e-9) -> Tuple[np.ndarray, np.ndarray, int]:
    """Returns (hist[H][n_bins], out_of_range[H], n_near_edge)."""
    coords = np.asarray(coords, np.float64)
    offsets = [int(v) for v in offsets]
    vals = list(coords.ravel())
    if box is not None:
        vals += list(np.asarray(box, np.float64).ravel())
    den = _common_scale(vals)
    X = [[int(Fraction(float(v)) * den) for v in row] for row in coords]
    shifts: List[Tuple[int, int, int]] = [(0, 0, 0)]
    if box is not None:
        B = [[int(Fraction(float(v)) * den) for v in row] for row in np.asarray(box, np.float64)]
        shifts = []
        for na, nb, nc in itertools.product(range(-reach, reach + 1), repeat=3):
            shifts.append(tuple(na * B[0][c] + nb * B[1][c] + nc * B[2][c] for c in range(3)))
    rm = Fraction(float(r_max))
    # t^2 = q/den^2 * n_bins^2 / r_max^2 = q * C, C = n_bins^2 * rm.den^2 / (den^2 * rm.num^2)
    c_num = n_bins * n_bins * rm.denominator * rm.denominator
    c_den = den * den * rm.numerator * rm.numerator

    k = len(offsets) - 1
    pairs = [(s, s) for s in range(k)] + [(s, t) for s in range(k) for t in range(s + 1, k)]
    hist = np.zeros((len(pairs), n_bins), np.uint64)
    oor = np.zeros(len(pairs), np.uint64)
    near = 0
    for h, (s, t) in enumerate(pairs):
        for i in range(offsets[s], offsets[s + 1]):
            j0 = i + 1 if s == t else offsets[t]
            xi = X[i]
            for j in range(j0, offsets[t + 1]):
                xj = X[j]
                d0, d1, d2 = xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]
                q = min((d0 + S[0]) ** 2 + (d1 + S[1]) ** 2 + (d2 + S[2]) ** 2 for S in shifts)
                num = q * c_num
                kk = math.isqrt(num // c_den)          # floor(t)
                tf = math.sqrt(num / c_den) if num else 0.0
                if kk > 0 or tf > 0:
                    frac_lo = tf - kk
                    if (kk >= 1 and frac_lo <= edge_tol * max(tf, 1.0)) or \
                            (kk + 1 - tf) <= edge_tol * max(tf, 1.0):
                        near += 1
                if kk < n_bins:
                    hist[h, kk] += 1
                else:
                    oor[h] += 1
    return hist, oor, near
