"""The binary64 root of the pair kernel, step by step in exact rational
arithmetic (every operation rounded once to the nearest double, as the device
executes it), with the v_rsq_f64 seed perturbed to the worst relative error
the ISA states for it (2^-23) in both directions.

* sqrt_cr (iteration + Tuckerman's rounding test) must equal IEEE sqrt
  (Python's math.sqrt) on the arguments whose roots come closest to rounding
  midpoints (down to about 3e-17 of an ulp; with the seed at its worst the
  iteration alone returns the wrong neighbour for half of them), on those
  nearest to squared midpoints, at powers of two, at the edge of the scaled
  range (2^-767) and on subnormals.
* t_fast64 (seed + one Goldschmidt step, the scale folded into its last
  fma) must stay within 2^13 ulps of the canonical t, and whenever its guard
  (low 32 bits of t at least 2^16 from a multiple of 2^32, t < 2^20) lets it
  through, its floor must equal the canonical floor.

This checks the method the kernel implements; the GPU tests check the kernel
itself against the oracle on the same arguments (tests/test_gpu_sqrt.py)."""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import midpoints

F = Fraction


def rn(x):
    return float(x)


def mul(a, b):
    return rn(F(a) * F(b))


def fma(a, b, c):
    return rn(F(a) * F(b) + F(c))


def bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def from_bits(b):
    return struct.unpack("<d", struct.pack("<Q", b & (2**64 - 1)))[0]


def seed(q, rel):
    """A v_rsq_f64 result with relative error rel (|rel| <= 2^-23)."""
    return rn(F(1.0 / math.sqrt(q)) * (1 + F(rel)))


def sqrt_cr(q, rel):
    tiny = q < 2.0 ** -767
    qs = math.ldexp(q, 1024) if tiny else q
    if not (qs > 0.0 and qs <= 1.7976931348623157e308):
        return q if q >= 0.0 or q != q else math.nan
    y0 = seed(qs, rel)
    g = mul(qs, y0)
    h = mul(0.5, y0)
    e = fma(-h, g, 0.5)
    h = fma(h, e, h)
    g = fma(g, e, g)
    d = fma(-g, g, qs)
    g = fma(d, h, g)
    d = fma(-g, g, qs)
    y = fma(d, h, g)
    r = fma(-y, y, qs)
    yb = bits(y)
    ex = ((yb >> 52) & 0x7FF) - 1022
    uy = math.ldexp(y, ex - 53)
    pow2 = (yb & ((1 << 52) - 1)) == 0
    low = -0.5 * uy if pow2 else -uy
    step = 1 if r > uy else (-1 if r <= low else 0)
    y = from_bits(yb + step)
    return math.ldexp(y, -512) if tiny else y


def t_fast(q, s, rel):
    y = seed(q, rel)
    g = mul(q, y)
    h = mul(0.5, y)
    e = fma(-h, g, 0.5)
    gs = mul(g, s)
    t = fma(gs, e, gs)
    lo = (bits(t) + 0x10000) & 0xFFFFFFFF
    near = lo < 0x20000
    return t, near


RELS = [-(2.0 ** -23), -(2.0 ** -24), 0.0, 2.0 ** -24, 2.0 ** -23]


def hard_args():
    rng = np.random.Generator(np.random.PCG64(2024))
    qs = midpoints.hardest_q()
    qs += midpoints.hard_q(rng, 150, -40, 60, k=2)
    qs += midpoints.edge_q([1, 2, 3, 7, 64, 999, 1000, 1024, 4095, 65536, 1048575], k=2)
    # powers of two and their neighbours, the scaled range's edge, subnormals
    for e in (-1070, -1000, -800, -768, -767, -766, -100, -1, 0, 1, 2, 51, 52, 53, 1000, 1023):
        p = math.ldexp(1.0, e)
        qs += [p, math.nextafter(p, 0.0), math.nextafter(p, math.inf)]
    qs += [5e-324, 1e-320, 2.2250738585072014e-308, 1.7976931348623157e308]
    return [q for q in qs if q > 0.0]


@pytest.mark.parametrize("rel", RELS)
def test_sqrt_cr_is_correctly_rounded(rel):
    for q in hard_args():
        got = sqrt_cr(q, rel)
        assert got == math.sqrt(q), (q, rel, got, math.sqrt(q))


def test_hardest_arguments_need_the_rounding_test():
    """Without the rounding test the iteration returns the neighbouring
    double on some of the hardest arguments (so the test above has teeth)."""
    def iteration_only(q, rel):
        y0 = seed(q, rel)
        g, h = mul(q, y0), mul(0.5, y0)
        e = fma(-h, g, 0.5)
        h, g = fma(h, e, h), fma(g, e, g)
        g = fma(fma(-g, g, q), h, g)
        return fma(fma(-g, g, q), h, g)
    qs = midpoints.hardest_q()
    assert sum(iteration_only(q, 2.0 ** -23) != math.sqrt(q) for q in qs) > 10


def test_sqrt_cr_special_values():
    assert sqrt_cr(0.0, 0.0) == 0.0
    assert sqrt_cr(math.inf, 0.0) == math.inf
    assert math.isnan(sqrt_cr(math.nan, 0.0))


@pytest.mark.parametrize("rel", RELS)
def test_fast_t_and_guard(rel):
    qs = midpoints.edge_q([1, 2, 3, 5, 99, 100, 1024, 4095, 20000, 1048575], k=3)
    rng = np.random.Generator(np.random.PCG64(7))
    qs += list(rng.uniform(1e-6, 4e10, size=400))
    for s in (1.0, 0.5, 3.0, 1.0 / 3.0, 512.0 / 22.0):
        for q in qs:
            t_canon = mul(math.sqrt(q), s)
            t, near = t_fast(q, s, rel)
            assert abs(t - t_canon) <= 2 ** 13 * math.ulp(t_canon), (q, s, rel)
            if not near and t < 2.0 ** 20:
                assert math.floor(t) == math.floor(t_canon), (q, s, rel, t, t_canon)
