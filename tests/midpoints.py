"""Frames whose binary64 squared distances sit next to the squares of rounding
midpoints: the arguments where a square root that is not correctly rounded
returns the neighbouring double.

For a double y with ulp u, the midpoint m = y + u/2 is not a double, and the
doubles q nearest to m*m have sqrt(q) within a tiny fraction of an ulp of m.
``hard_q`` returns such q (the nearest double to m*m and its neighbours).
``edge_q`` does the same for midpoints just below and above integers n, so
that with s = n_bins / r_max = 1 a root one ulp off would move the pair into
the neighbouring bin.

``pair_coords`` turns each q into a pair of points whose canonical binary64
arithmetic (d = x_j - x_i, q = fma(dz, dz, fma(dy, dy, dx*dx))) gives exactly
that q: dx just below sqrt(q), dy = sqrt(q - dx*dx) rounded, dz = 0. Each pair
is translated 10^4 further along z, so pairs of different pairs are far out of
range (r_max is at most 5,000 here). Everything is checked in exact rational
arithmetic (``canonical_q``).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def rn(x: Fraction) -> float:
    """Round a rational to the nearest double (ties to even)."""
    return float(x)  # int / int true division in CPython rounds correctly


def ulp(x: float) -> float:
    return math.ulp(x)


def hard_q(rng: np.random.Generator, n: int, e_lo: int = -30, e_hi: int = 40, k: int = 2):
    """q next to (y + ulp(y)/2)^2 for n random doubles y in [2^e_lo, 2^e_hi)."""
    out = []
    for _ in range(n):
        e = int(rng.integers(e_lo, e_hi))
        y = math.ldexp(1.0 + float(rng.random()), e)
        m = Fraction(y) + Fraction(ulp(y)) / 2
        q0 = rn(m * m)
        out.extend(_around(q0, k))
    return out


def _hensel_root(c: int, k: int, start: int) -> int:
    """M with M*M + M + c = 0 (mod 2^k), lifted bit by bit from M = start
    (mod 2); the derivative 2M + 1 is odd, so each bit is forced."""
    m = start
    for i in range(1, k):
        if (m * m + m + c) % (1 << (i + 1)) != 0:
            m += 1 << i
    return m


def hardest_q(cs=range(-40, 41, 2), exps=(-3, 0, 7, 30)):
    """q = u^2 (M^2 + M + c) for 53-bit M with M^2 + M + c divisible by the
    spacing of doubles at q: q is then a double whose root lies only about
    |c|/(8M) of an ulp from the midpoint M*u + u/2, the closest a root of a
    double can come to a midpoint (Q - M^2 - M - 1/4 is never 0). Found by
    Hensel lifting the congruence, for small even c."""
    out = []
    for c in cs:
        for k in (52, 53):
            for start in (0, 1):
                m = _hensel_root(c, k, start) + (1 << 52)
                while m < (1 << 53):
                    qq = m * m + m + c
                    if qq.bit_length() - 53 <= k and qq % (1 << (qq.bit_length() - 53)) == 0:
                        for e in exps:
                            u = Fraction(2) ** (e - 52)
                            q = u * u * qq
                            if rn(q) == q:
                                out.append(float(q))
                    m += 1 << k
    return sorted(set(out))


def edge_q(integers, k: int = 2):
    """q next to the squares of the midpoints just below and just above each
    integer n: (n - ulp(pred(n))/2)^2 and (n + ulp(n)/2)^2."""
    out = []
    for n in integers:
        n = float(n)
        below = Fraction(n) - Fraction(ulp(math.nextafter(n, 0.0))) / 2
        above = Fraction(n) + Fraction(ulp(n)) / 2
        for m in (below, above):
            out.extend(_around(rn(m * m), k))
    return out


def _around(q0: float, k: int):
    vals = [q0]
    a = b = q0
    for _ in range(k):
        a = math.nextafter(a, 0.0)
        b = math.nextafter(b, math.inf)
        vals += [a, b]
    return vals


def canonical_q(dx: float, dy: float, dz: float = 0.0) -> float:
    """fma(dz, dz, fma(dy, dy, dx*dx)) in binary64, evaluated exactly."""
    xx = rn(Fraction(dx) * Fraction(dx))
    inner = rn(Fraction(dy) * Fraction(dy) + Fraction(xx))
    return rn(Fraction(dz) * Fraction(dz) + Fraction(inner))


def pair_offsets(q: float):
    """(dx, dy) with canonical_q(dx, dy) == q."""
    r = math.sqrt(q)
    dx = r * (1.0 - 2.0 ** -20)
    delta = Fraction(q) - Fraction(rn(Fraction(dx) * Fraction(dx)))
    dy = math.sqrt(float(delta))
    if canonical_q(dx, dy) != q:
        # one step of dy either way always lands on q: dy^2 moves q by far
        # less than an ulp of q
        for cand in (math.nextafter(dy, 0.0), math.nextafter(dy, math.inf)):
            if canonical_q(dx, cand) == q:
                return dx, cand
        raise AssertionError(f"no pair for q={q!r}")
    return dx, dy


def pair_coords(qs):
    """(coords [2K, 3], pi, pj): pair k is points 2k (origin + shift) and
    2k + 1, its canonical q is qs[k]."""
    xs = np.zeros((2 * len(qs), 3))
    for k, q in enumerate(qs):
        dx, dy = pair_offsets(q)
        z = 1.0e4 * k
        xs[2 * k] = (0.0, 0.0, z)
        xs[2 * k + 1] = (dx, dy, z)
    pi = np.arange(0, 2 * len(qs), 2)
    return np.ascontiguousarray(xs), pi, pi + 1
