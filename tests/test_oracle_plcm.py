"""Pins of the oracle's PLCM and byte generator (Sec. 3, Eq. (5) and the
PLCM byte generator).  Nothing here calls the GPU library."""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

from golden_io import records

HALF = Fraction(1, 2)


def rn(q: Fraction) -> float:
    """Round an exact rational to the nearest binary64 (ties to even):
    CPython's int/int true division is correctly rounded."""
    return q.numerator / q.denominator


def plcm_exact_ieee(x: float, p: float) -> float:
    """Eq. (5) evaluated with exact rationals, each IEEE operation rounded
    once to binary64.  An independent route to the same value the oracle
    must give when every C operator is one correctly rounded operation."""
    X, P = Fraction(x), Fraction(p)
    if X > HALF:
        X = Fraction(rn(1 - X))
    if X < P:
        return rn(X / P)
    num = Fraction(rn(X - P))
    den = Fraction(rn(HALF - P))
    return rn(num / den)


def quarter_map_exact(X: Fraction) -> Fraction:
    """Eq. (5) with p = 1/4 in exact arithmetic: 4x on [0,1/4),
    4x-1 on [1/4,1/2], F(1-x) on (1/2,1].  Every step is exact in binary64
    (multiplying by 4, Sterbenz subtraction), so no rounding enters."""
    if X > HALF:
        X = 1 - X
    if X < Fraction(1, 4):
        return 4 * X
    return 4 * X - 1


def test_special_orbits(orc):
    for (x0, p), orbit in records("plcm_orbits.txt"):
        x, p = float(x0), float(p)
        for want in orbit:
            x = orc.plcm(x, p)
            assert x == float(want), (x0, p, orbit)


def test_fixed_point_zero_and_p(orc):
    rng = np.random.default_rng(5)
    for p in rng.uniform(1e-3, 0.5 - 1e-3, 200):
        assert orc.plcm(0.0, p) == 0.0
        assert orc.plcm(float(p), p) == 0.0          # x = p starts the second piece at 0
        assert orc.plcm(0.5, p) == 1.0               # (1/2-p)/(1/2-p)
        assert orc.plcm(1.0, p) == 0.0               # F(1-1) = F(0)


def test_quarter_orbit_is_exact(orc):
    """p = 1/4: the binary64 orbit equals the exact rational orbit."""
    rng = np.random.default_rng(11)
    for x0 in rng.uniform(0, 1, 50):
        x, X = float(x0), Fraction(float(x0))
        for _ in range(60):
            x = orc.plcm(x, 0.25)
            X = quarter_map_exact(X)
            assert Fraction(x) == X


def test_correct_rounding_of_every_operation(orc):
    """General p: each step is RN of the exact quotient of RN operands."""
    rng = np.random.default_rng(12)
    xs = np.concatenate([rng.uniform(0, 1, 3000), rng.uniform(0.49, 0.51, 500),
                         rng.uniform(0, 1e-6, 200), 1 - rng.uniform(0, 1e-6, 200)])
    ps = np.concatenate([rng.uniform(0, 0.5, 3500), rng.uniform(0.4999, 0.5, 200),
                         rng.uniform(1e-12, 1e-6, 200)])
    for x, p in zip(xs, ps):
        if not 0 < p < 0.5:
            continue
        assert orc.plcm(float(x), float(p)) == plcm_exact_ieee(float(x), float(p)), (x, p)


def test_branch_boundaries(orc):
    """x just below / at / above p and 1/2 pick the piece Eq. (5) names."""
    p = 0.3
    below = np.nextafter(p, 0)
    assert orc.plcm(below, p) == plcm_exact_ieee(below, p)
    assert orc.plcm(below, p) <= 1.0 and orc.plcm(below, p) > 0.99
    assert orc.plcm(p, p) == 0.0
    above_half = np.nextafter(0.5, 1)
    assert orc.plcm(above_half, p) == plcm_exact_ieee(above_half, p)
    assert orc.plcm(0.5, p) == 1.0


def _bytes6(x: float) -> bytes:
    return struct.pack("<d", x)[:6]


@pytest.mark.parametrize("nbytes", [1, 5, 6, 7, 12, 13, 600, 601])
def test_byte_generator_exact_orbit(orc, nbytes):
    """Bytes 0..5 of each iterate (little-endian), XOR of the two maps,
    starting at the first iterate; only the first nbytes are kept and the
    state advances ceil(nbytes/6) steps."""
    rng = np.random.default_rng(nbytes)
    x1, x2 = float(rng.uniform(0, 1)), float(rng.uniform(0, 1))
    X1, X2 = Fraction(x1), Fraction(x2)
    want = bytearray()
    steps = -(-nbytes // 6)
    for _ in range(steps):
        X1, X2 = quarter_map_exact(X1), quarter_map_exact(X2)
        a, b = _bytes6(float(X1)), _bytes6(float(X2))
        want += bytes(u ^ v for u, v in zip(a, b))
    got, y1, y2 = orc.plcm_bytes(x1, 0.25, x2, 0.25, nbytes)
    assert bytes(got) == bytes(want[:nbytes])
    assert y1 == float(X1) and y2 == float(X2)


def test_byte_generator_general_p(orc):
    rng = np.random.default_rng(3)
    x1, p1, x2, p2 = (float(v) for v in (rng.uniform(0, 1), rng.uniform(0, .5),
                                          rng.uniform(0, 1), rng.uniform(0, .5)))
    got, _, _ = orc.plcm_bytes(x1, p1, x2, p2, 6 * 200)
    a, b = x1, x2
    want = bytearray()
    for _ in range(200):
        a, b = plcm_exact_ieee(a, p1), plcm_exact_ieee(b, p2)
        want += bytes(u ^ v for u, v in zip(_bytes6(a), _bytes6(b)))
    assert bytes(got) == bytes(want)


def test_keystream_layout_and_continuation(orc):
    """Per frame, band i gets r*S_i bytes (Algorithm 2 iterates each band's
    generator until its bytes for the frame exist), bands in order; the
    chains carry across frames."""
    from paper_2302_07411_amd.inputs import plcm_key
    H, W, C, n, r = 10, 6, 3, 3, 2          # bands of 3, 3, 4 rows
    pm = plcm_key(n, 77)
    k_all = orc.PlcmKey(H, W, C, n, r, pm).keystream(3)
    k_split = orc.PlcmKey(H, W, C, n, r, pm)
    parts = [k_split.keystream(1), k_split.keystream(2)]
    assert np.array_equal(k_all, np.concatenate(parts))
    # frame 0 band by band from the byte generator
    x = pm.copy()
    row = W * C
    for i in range(n):
        lo, hi = orc.band_lo(H, n, i), orc.band_lo(H, n, i + 1)
        S = (hi - lo) * row
        got = k_all[0, r * lo * row: r * lo * row + r * S]
        want, _, _ = orc.plcm_bytes(x[i, 0], x[i, 1], x[i, 2], x[i, 3], r * S)
        assert np.array_equal(got, want)


def test_keystream_bytes_are_uniform(orc):
    """Statistical sanity: chi-square of 2^20 keystream bytes against the
    uniform histogram stays below 293.25 (the 5% critical value the paper
    uses in Sec. 4)."""
    out, _, _ = orc.plcm_bytes(0.1234567, 0.3141592, 0.7654321, 0.2718281, 1 << 20)
    hist = np.bincount(out, minlength=256).astype(np.float64)
    e = out.size / 256
    chi2 = float(((hist - e) ** 2 / e).sum())
    assert chi2 < 293.25
    assert not math.isnan(chi2)
