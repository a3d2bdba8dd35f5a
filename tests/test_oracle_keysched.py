"""Oracle pins for the key schedule of the main thread (Algorithm 1, the
reading CV_KEY_SCHEDULE_VERSION 1 of the library's header): exact rational
PLCM orbits, the 2DLASM master stepped through the separately pinned
one-step map, resumption at any frame, ranges, degenerate keys."""
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle


PLCM_DEGENERATE = ([0.25, 0.25, 0.3, 0.2],    # map 1 starts at x0 = p: F(p) = 0
                   [0.3, 0.2, 0.25, 0.25],    # map 2 likewise
                   [0.3, 0.2, 0.375, 0.25])   # map 2: 0.375 -> 1/2 -> 1 -> 0


def _bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def _plcm_exact(x: Fraction, p: Fraction) -> Fraction:
    if x > Fraction(1, 2):
        x = 1 - x
    return x / p if x < p else (x - p) / (Fraction(1, 2) - p)


def test_plcm_master_exact_orbit():
    """p = 1/4 for both maps: every PLCM step (a fold 1 - x, a product by 4,
    x - 1/4 for x in [1/4, 1/2]) is exact in binary64, so the draws can be
    computed with rationals and the parameters and seeds follow from the
    stated rule.  Each step drops two bits of the start's binary expansion,
    which leaves about 25 draws before an orbit reaches 0."""
    K = [0.3, 0.25, 0.6, 0.25]
    n, T = 2, 6
    xs = [Fraction(K[0]), Fraction(K[2])]
    draws = []
    while len(draws) < 20:
        xs = [_plcm_exact(xs[0], Fraction(1, 4)), _plcm_exact(xs[1], Fraction(1, 4))]
        draws.append((float(xs[0]), float(xs[1])))
        assert all(Fraction(float(x)) == x for x in xs)  # exactly representable
    want_pm, k = [], 0
    for _ in range(2 * n):
        while not (0 < draws[k][0] < 1 and 0 < draws[k][1] < 1):
            k += 1
        u, v = draws[k]
        want_pm += [u, v / 2]
        k += 1
    want_sc = [1 + ((_bits(u) ^ _bits(v)) & 0xFFFF) for u, v in draws[k:k + T]]
    pm, sc = oracle.key_schedule(False, K, n, 0, T)
    assert list(pm.reshape(-1)) == want_pm
    assert list(sc) == want_sc


def test_lasm_master_follows_the_map():
    K = [0.3, 0.6, 0.9]
    pm, sc = oracle.key_schedule(True, K, 1, 0, 3)
    x, y, draws = K[0], K[1], []
    for _ in range(7):
        x, y = oracle.lasm(x, y, K[2])
        draws.append((x, y))
    (u0, v0), (u1, _), (u2, v2), (u3, _) = draws[:4]
    assert list(pm[0]) == [u0, v0, 0.44 + 0.49 * u1, u2, v2, 0.44 + 0.49 * u3]
    assert list(sc) == [1 + ((_bits(u) ^ _bits(v)) & 0xFFFF) for u, v in draws[4:7]]


@pytest.mark.parametrize("is_lasm", [False, True])
def test_resume_and_ranges(is_lasm):
    K = [0.41, 0.63, 0.77] if is_lasm else [0.41, 0.13, 0.77, 0.29]
    pm, sc = oracle.key_schedule(is_lasm, K, 5, 0, 50)
    pm2, sc2 = oracle.key_schedule(is_lasm, K, 5, 20, 30)
    assert np.array_equal(pm, pm2) and np.array_equal(sc[20:], sc2)
    assert sc.min() >= 1 and sc.max() <= 65536
    if is_lasm:
        assert ((pm[:, [0, 1, 3, 4]] > 0) & (pm[:, [0, 1, 3, 4]] < 1)).all()
        assert ((pm[:, [2, 5]] >= 0.44) & (pm[:, [2, 5]] <= 0.93)).all()
    else:
        assert ((pm[:, [0, 2]] > 0) & (pm[:, [0, 2]] < 1)).all()
        assert ((pm[:, [1, 3]] > 0) & (pm[:, [1, 3]] < 0.5)).all()


def test_degenerate_master_keys():
    """A draw with a component outside (0,1) is skipped; since 0 is a fixed
    point of both maps (and 1 maps to 0), such a master orbit never yields a
    usable draw again, and the schedule must report the key as degenerate
    whichever component collapsed."""
    for K in PLCM_DEGENERATE:
        with pytest.raises(ValueError):
            oracle.key_schedule(False, K, 1, 0, 1)
    for K in ([0.3, 1.0, 0.9], [1.0, 0.3, 0.9]):  # y or x pinned at 0 after one step
        with pytest.raises(ValueError):
            oracle.key_schedule(True, K, 1, 0, 1)
