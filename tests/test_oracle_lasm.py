"""Pins of the oracle's 2DLASM generator (Sec. 3, Eq. (6)) and of its
correctly rounded sine, against things other than the oracle itself:

  - the sine against mpmath at 200 bits rounded to binary64 (an independent
    arbitrary-precision library; the oracle uses libquadmath);
  - closed forms: x = 1/2, y = 1, mu = 1 makes the first argument exactly
    RN(pi), whose sine is known, and y(1-y) = 0 pins y' = 0;
  - the two one-dimensional reductions of Eq. (6): with y = 0 the x update
    and with x = 0 the y update are the same map, bit for bit -- which fails
    if either update used the wrong coupling term;
  - the byte layout: with map 2 parked at its fixed point (0, 0) the
    keystream is the little-endian bytes 0..5 of map 1's x, then y;
  - range and round-trip invariants of the whole cipher with 2DLASM keys.
"""
import struct

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, lasm_key, uniform_frames

PI = 3.141592653589793  # RN(pi)


def rn_sin(t: float) -> float:
    """RN(sin(t)) via mpmath: 200-bit sine, one rounding to 53 bits."""
    with mp.workprec(200):
        s = mp.sin(mp.mpf(t))
    with mp.workprec(53):
        return float(+s)


def test_cr_sin_matches_mpmath():
    r = np.random.default_rng(11)
    ts = list(r.uniform(0.0, PI, 20000))
    ts += list(np.exp(r.uniform(np.log(2.0 ** -60), 0.0, 4000)))
    hp = PI / 2
    ts += [0.0, 1e-300, 2.0 ** -30, 0.5, 1.0, 2.0, 3.0, hp, np.nextafter(hp, 0), np.nextafter(hp, 4),
           PI, np.nextafter(PI, 0), 1.5707963267948966, 0.7853981633974483]
    bad = [t for t in ts if oracle.cr_sin(float(t)) != rn_sin(float(t))]
    assert not bad, f"{len(bad)} arguments differ, e.g. {bad[:3]}"


def test_near_midpoint_detection():
    """With the margin widened to 2^-60 (1/128 of the gap between binary64
    midpoints at the same scale) about 1 argument in 64 is flagged; the flag
    must agree with the distance to the nearest midpoint that mpmath finds."""
    import ctypes as ct
    r = np.random.default_rng(5)
    flagged = 0
    for t in r.uniform(0.01, PI, 4000):
        out = ct.c_double()
        got = oracle.lib().oracle_cr_sin_margin(float(t), ct.byref(out), -60)
        with mp.workprec(200):
            s = mp.sin(mp.mpf(float(t)))
            d = rn_sin(float(t))
            ulp = mp.mpf(np.nextafter(d, 4.0)) - mp.mpf(d)
            dist = min(abs(s - (mp.mpf(d) + ulp / 2)), abs(s - (mp.mpf(d) - ulp / 2)))
            rel = dist / abs(s)
        if abs(rel - mp.mpf(2) ** -60) < mp.mpf(2) ** -90:
            continue  # too close to the margin itself to judge
        assert got == (1 if rel <= mp.mpf(2) ** -60 else 0), t
        flagged += got
    assert 10 < flagged < 400


def test_cr_sin_closed_forms():
    assert oracle.cr_sin(0.0) == 0.0
    # sin(RN(pi)) = pi - RN(pi) + O(1e-48): the binary64 nearest to 1.2246467991473532e-16
    assert oracle.cr_sin(PI) == float.fromhex("0x1.1a62633145c07p-53")
    assert oracle.cr_sin(1e-300) == 1e-300  # sin(t) = t(1 - t^2/6): rounds to t


def test_first_step_closed_form():
    # x = 1/2, y = 1, mu = 1: ((pi*1)*(1+3))*(1/2)*(1/2) = RN(pi) exactly
    x1, y1 = oracle.lasm(0.5, 1.0, 1.0)
    assert x1 == float.fromhex("0x1.1a62633145c07p-53")
    assert y1 == 0.0  # y(1-y) = 0


def test_one_dimensional_reductions_coincide():
    for mu in (0.375, 0.41, 0.5, 0.93, 1.0):
        for s in (0.1, 0.3, 0.77):
            ax, ay = s, 0.0   # y parked at 0: only x moves
            bx, by = 0.0, s   # x parked at 0: only y moves
            for _ in range(200):
                ax, ay = oracle.lasm(ax, ay, mu)
                bx, by = oracle.lasm(bx, by, mu)
                assert ay == 0.0 and bx == 0.0
                assert ax == by, (mu, s)


def test_new_x_enters_the_y_update():
    # with x0 = y0 the y update would repeat the x update if it used x0
    x1, y1 = oracle.lasm(0.5, 0.5, 1.0)
    assert x1 != y1
    # the same step through mpmath with binary64 rounding after every operation
    with mp.workprec(53):
        pi, mu = mp.mpf(PI), mp.mpf(1)
        ax = ((pi * mu) * (mp.mpf(0.5) + 3)) * mp.mpf(0.5) * (1 - mp.mpf(0.5))
        want_x = rn_sin(float(ax))
        ay = ((pi * mu) * (mp.mpf(want_x) + 3)) * mp.mpf(0.5) * (1 - mp.mpf(0.5))
        want_y = rn_sin(float(ay))
    assert (x1, y1) == (want_x, want_y)


def test_byte_layout():
    m1 = (0.3, 0.6, 0.9)
    got, _, (x2, y2) = oracle.lasm_bytes(m1, (0.0, 0.0, 0.9), 12 * 5 + 7)
    assert (x2, y2) == (0.0, 0.0)
    want = []
    x, y = m1[0], m1[1]
    for _ in range(6):
        x, y = oracle.lasm(x, y, m1[2])
        want += list(struct.pack("<d", x)[:6]) + list(struct.pack("<d", y)[:6])
    assert list(got) == want[:67]


def test_orbits_stay_in_the_unit_interval():
    r = np.random.default_rng(3)
    for _ in range(200):
        x, y = r.uniform(0, 1, 2)
        mu = float(r.choice([0.375, 0.41, 0.6, 0.93, 1.0]))
        for _ in range(50):
            x, y = oracle.lasm(float(x), float(y), mu)
            assert 0.0 <= x <= 1.0 and 0.0 <= y <= 1.0


@pytest.mark.parametrize("H,W,C,n,r,T", [(24, 20, 3, 4, 5, 2), (9, 9, 1, 9, 3, 2), (17, 3, 1, 1, 5, 2)])
def test_cipher_round_trip(H, W, C, n, r, T):
    pm = lasm_key(n, 40 + H)
    frames = uniform_frames(H, W, C, T, 41 + W)
    s_c = confusion_seeds(T, 42)
    enc = oracle.LasmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    assert not np.array_equal(enc, frames)
    dec = oracle.LasmKey(H, W, C, n, r, pm).decrypt(enc, s_c)
    assert np.array_equal(dec, frames)


def test_keystream_continues_across_frames():
    H, W, C, n, r = 12, 8, 3, 3, 2
    pm = lasm_key(n, 9)
    two = oracle.LasmKey(H, W, C, n, r, pm).keystream(2)
    k = oracle.LasmKey(H, W, C, n, r, pm)
    a, b = k.keystream(1), k.keystream(1)
    assert np.array_equal(two, np.concatenate([a, b]))
