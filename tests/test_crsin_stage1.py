"""The first stage of the 2DLASM generator's sine (cv_sin_stage1, host):
its double-double value against mpmath at 250 bits stays inside the stated
relative error bound 2^-69.2 on random arguments, small arguments,
arguments next to its table points and cell boundaries, and next to pi/2
and pi; whenever its rounding test decides, the result is RN(sin t)."""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_2302_07411_amd import binding as B

PI_HI = 3.141592653589793
HALF_PI = 1.5707963267948966


def _args():
    r = np.random.default_rng(2026)
    ts = [r.uniform(0.0, PI_HI, 20000),
          np.exp(r.uniform(math.log(2.0 ** -60), 0.0, 4000))]
    j = r.integers(1, 403, 1500)
    for base in (j / 256.0, (j + 0.5) / 256.0):        # table points and cell edges
        for k in (-3, -1, 0, 1, 3):
            ts.append(base + k * np.spacing(base))
    for x in (HALF_PI, PI_HI, 1.0, 0.5, 2.0 ** -9, 2.0 ** -8):
        v = x
        near = [v]
        for _ in range(8):
            v = np.nextafter(v, 0.0)
            near.append(v)
        v = x
        for _ in range(8):
            v = np.nextafter(v, 4.0)
            near.append(v)
        ts.append(np.array(near))
    ts.append(np.array([0.0, 5e-324, 1e-300, 2.0 ** -1000, 1e-20]))
    t = np.concatenate(ts)
    return t[(t >= 0.0) & (t <= PI_HI)]


def test_stage1_error_bound_and_rounding():
    B.load()
    t = _args()
    hi, lo, dec = B.sin_stage1(t)
    mp.mp.prec = 250
    worst = 0.0
    for x, h, l, d in zip(t, hi, lo, dec):
        exact = mp.sin(mp.mpf(float(x)))
        if exact == 0:
            assert h == 0.0 and l == 0.0
            continue
        rel = abs((mp.mpf(float(h)) + mp.mpf(float(l)) - exact) / exact)
        worst = max(worst, float(rel))
        if d:
            with mp.workprec(53):
                rn = float(+exact)
            assert h == rn, f"t={float(x).hex()}: stage 1 decided {h!r}, RN(sin t) = {rn!r}"
    assert worst < 2.0 ** -69.2, f"max relative error 2^{math.log2(worst):.2f}"
    assert dec.mean() > 0.999


def test_stage1_rejects_arguments_outside_the_range():
    B.load()
    for bad in ([-1e-300], [3.1415926535897936], [float("nan")]):
        with pytest.raises(B.CvError):
            B.sin_stage1(bad)
