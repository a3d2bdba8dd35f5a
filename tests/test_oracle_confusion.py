"""Pins of the oracle's row-shift table and confusion (Sec. 2, Eq. (1),
Eq. (2), Algorithm 2)."""
import math

import mpmath
import numpy as np
import pytest

from golden_io import fields, records


def test_gtables_golden(orc):
    for lhs, g in records("gtables.txt"):
        if len(lhs) == 2:
            H, s_c = (int(v) for v in lhs)
            assert list(orc.gtable(H, s_c)) == [int(v) for v in g]
        else:
            H, s_c, alpha = (int(v) for v in lhs)
            assert orc.gtable(H, s_c)[alpha] == int(g[0]), lhs


def _g_high_precision(H, s_c):
    """floor(s_c * RN(sin(theta))) with theta = RN(RN(2*pi*alpha)/H) formed
    by the same binary64 operations, and sin evaluated with 80 significant
    digits then rounded once to binary64 (a correctly rounded sine)."""
    mpmath.mp.dps = 80
    out = []
    for alpha in range(H):
        theta = ((2.0 * math.pi) * float(alpha)) / float(H)
        s = float(mpmath.sin(mpmath.mpf(theta)))       # mpf(float) is exact
        out.append(math.floor(float(s_c) * s))
    return out


@pytest.mark.parametrize("H,s_c", [(256, 1), (256, 40000), (480, 777), (768, 65535),
                                   (1080, 12345), (97, 3), (2160, 65535)])
def test_gtable_high_precision(orc, H, s_c):
    assert list(orc.gtable(H, s_c)) == _g_high_precision(H, s_c)


@pytest.mark.parametrize("H", [4, 8, 256, 480, 768, 1080])
def test_gtable_quadrants(orc, H):
    """sin(0)=0, sin(pi/2) and sin(3pi/2) round to +-1 exactly, and the
    binary64 pi lies below pi so sin of it is a tiny positive number."""
    for s_c in (1, 2, 999, 65535):
        g = orc.gtable(H, s_c)
        assert g[0] == 0
        assert g[H // 4] == s_c and g[H // 2] == 0 and g[3 * H // 4] == -s_c
        assert np.all(np.abs(g) <= s_c)


def _skew_then_rotate(X, g):
    """Eq. (1) factored: alpha=(a+o) mod H moves column o down by o (a
    column roll); beta=(o+g[alpha]) mod W then rolls row alpha right by
    g[alpha].  Built from numpy.roll only."""
    H, W, C = X.shape
    Y1 = np.empty_like(X)
    for o in range(W):
        Y1[:, o] = np.roll(X[:, o], o % H, axis=0)
    Y = np.empty_like(X)
    for alpha in range(H):
        Y[alpha] = np.roll(Y1[alpha], int(g[alpha]) % W, axis=0)
    return Y


def test_confusion_golden(orc):
    f = fields("confusion_4x4.txt")
    H, W = int(f["H"][0]), int(f["W"][0])
    X = np.array([int(v) for v in f["X"]], np.uint8).reshape(H, W, 1)
    Y = np.array([int(v) for v in f["Y"]], np.uint8).reshape(H, W, 1)
    g = orc.gtable(H, int(f["s_c"][0]))
    assert np.array_equal(orc.confuse(X, g), Y)
    assert np.array_equal(orc.unconfuse(Y, g), X)


SHAPES = [(4, 4, 1), (8, 8, 3), (7, 5, 3), (5, 9, 1), (12, 30, 2), (31, 17, 3), (64, 64, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_confusion_factorisation(orc, shape):
    H, W, C = shape
    rng = np.random.default_rng(H * 100 + W)
    X = rng.integers(0, 256, (H, W, C), dtype=np.uint8)
    for g in (np.zeros(H, np.int64), orc.gtable(H, int(rng.integers(1, 65536))),
              rng.integers(-10 ** 6, 10 ** 6, H)):
        assert np.array_equal(orc.confuse(X, g), _skew_then_rotate(X, g))


@pytest.mark.parametrize("shape", SHAPES)
def test_confusion_is_a_pixel_permutation(orc, shape):
    """An iota frame (pixel index spread over 3 bytes) maps to a permutation
    of the indices, every pixel moving as a whole; histograms are kept; and
    Eq. (2) inverts Eq. (1) in both orders."""
    H, W, _ = shape
    N = H * W
    idx = np.arange(N, dtype=np.uint32)
    X = np.stack([(idx >> 16) & 255, (idx >> 8) & 255, idx & 255], -1).astype(np.uint8)
    X = X.reshape(H, W, 3)
    g = orc.gtable(H, 1 + (H * 7919) % 65535)
    Y = orc.confuse(X, g)
    back = (Y[..., 0].astype(np.uint32) << 16) | (Y[..., 1].astype(np.uint32) << 8) | Y[..., 2]
    assert np.array_equal(np.sort(back.ravel()), idx)
    assert np.array_equal(orc.unconfuse(Y, g), X)
    assert np.array_equal(orc.confuse(orc.unconfuse(X, g), g), X)
    for c in range(3):
        assert np.array_equal(np.bincount(X[..., c].ravel(), minlength=256),
                              np.bincount(Y[..., c].ravel(), minlength=256))
