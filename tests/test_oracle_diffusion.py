"""Pins of the oracle's diffusion and its inverse (Sec. 2, Eq. (3),
Eq. (4), Algorithm 2)."""
import numpy as np
import pytest

from golden_io import fields


def _ints(tokens):
    return np.array([int(v) for v in tokens], np.uint8)


def _band_bounds(orc, H, W, C, n):
    """Byte ranges of the n bands, from the definition of the split
    (Algorithm 2's band bounds i*H/n, extended as floor(i*H/n) so that every
    row is covered when n does not divide H), not from the oracle."""
    row = W * C
    return [((i * H // n) * row, ((i + 1) * H // n) * row) for i in range(n)]


def test_band_split(orc):
    """Hand-listed splits: n | H gives Algorithm 2's equal bands of H/n
    rows; otherwise floor(i*H/n) boundaries."""
    cases = {(10, 3): [0, 3, 6, 10], (256, 4): [0, 64, 128, 192, 256],
             (1080, 16): [0, 67, 135, 202, 270, 337, 405, 472, 540, 607, 675, 742,
                          810, 877, 945, 1012, 1080],
             (9, 9): list(range(10)), (7, 1): [0, 7]}
    for (H, n), want in cases.items():
        assert [orc.band_lo(H, n, i) for i in range(n + 1)] == want


def test_golden_band(orc):
    """4x4 frame, 2 bands, r=1: band 0 chained to the pre-diffusion last
    byte of band 1."""
    f = fields("diffusion.txt")
    Y = np.concatenate([_ints(f["band_Y"]), _ints(f["band_next_Y"])]).reshape(4, 4, 1)
    ks = np.zeros(16, np.uint8)
    ks[:8] = _ints(f["b"])
    ks[8:] = np.arange(8, 16, dtype=np.uint8) * 29
    Z = orc.diffuse(Y, 2, 1, 0, ks)
    assert np.array_equal(Z.ravel()[:8], _ints(f["band_Z"]))
    assert np.array_equal(orc.undiffuse(Z, 2, 1, 0, ks), Y)


def test_golden_wrap(orc):
    """mod-256 addition and subtraction: a 2x3 gray frame, 2 bands of 3."""
    f = fields("diffusion.txt")
    Y = np.zeros((2, 3, 1), np.uint8)
    Y[0, :, 0] = _ints(f["wrap_Y"])
    Y[1, 2, 0] = int(f["wrap_next_last"][0])
    ks = np.zeros(6, np.uint8)
    ks[:3] = _ints(f["wrap_b"])
    Z = orc.diffuse(Y, 2, 1, 0, ks)
    assert np.array_equal(Z[0, :, 0], _ints(f["wrap_Z"]))
    assert np.array_equal(orc.undiffuse(Z, 2, 1, 0, ks), Y)


CASES = [(4, 4, 1, 2, 1), (16, 8, 3, 4, 5), (10, 6, 3, 3, 2), (9, 7, 1, 9, 3),
         (13, 5, 3, 1, 5), (30, 11, 2, 7, 4)]


@pytest.mark.parametrize("H,W,C,n,r", CASES)
def test_zero_keystream_is_a_prefix_xor(orc, H, W, C, n, r):
    """With b = 0, Eq. (3) is C_k = P_k xor C_{k-1}: a textbook inclusive
    XOR scan of each band, seeded with the next band's last byte."""
    rng = np.random.default_rng(H * W + n)
    Y = rng.integers(0, 256, (H, W, C), dtype=np.uint8)
    ks = np.zeros(r * Y.size, np.uint8)
    flat = Y.ravel()
    bounds = _band_bounds(orc, H, W, C, n)
    for j in range(r):
        Z = orc.diffuse(Y, n, r, j, ks).ravel()
        for i, (lo, hi) in enumerate(bounds):
            seed = flat[bounds[(i + 1) % n][1] - 1]
            want = np.bitwise_xor.accumulate(flat[lo:hi]) ^ seed
            assert np.array_equal(Z[lo:hi], want)


@pytest.mark.parametrize("H,W,C,n,r", CASES)
def test_closed_form_prefix_xor(orc, H, W, C, n, r):
    """Unrolling Eq. (3): C_k = s_d xor D_0 xor ... xor D_k with
    D_k = b_k xor ((P_k + b_k) mod 256); round j reads the band's keystream
    bytes [j*S_i, (j+1)*S_i) from its block of r*S_i bytes."""
    rng = np.random.default_rng(H * 31 + r)
    Y = rng.integers(0, 256, (H, W, C), dtype=np.uint8)
    ks = rng.integers(0, 256, r * Y.size, dtype=np.uint8)
    flat = Y.ravel()
    bounds = _band_bounds(orc, H, W, C, n)
    for j in range(r):
        Z = orc.diffuse(Y, n, r, j, ks).ravel()
        for i, (lo, hi) in enumerate(bounds):
            S = hi - lo
            b = ks[r * lo + j * S: r * lo + (j + 1) * S]
            D = b ^ ((flat[lo:hi].astype(np.uint16) + b) & 255).astype(np.uint8)
            seed = flat[bounds[(i + 1) % n][1] - 1]
            assert np.array_equal(Z[lo:hi], np.bitwise_xor.accumulate(D) ^ seed)
        assert np.array_equal(orc.undiffuse(orc.diffuse(Y, n, r, j, ks), n, r, j, ks), Y)


def test_single_band_seeds_itself(orc):
    """n = 1: the next band of band 0 is band 0, so s_d is its own last
    (pre-diffusion) byte."""
    Y = np.arange(12, dtype=np.uint8).reshape(3, 4, 1)
    ks = np.zeros(12, np.uint8)
    Z = orc.diffuse(Y, 1, 1, 0, ks).ravel()
    assert Z[0] == 0 ^ 11


def test_inverse_is_elementwise(orc):
    """Eq. (4) needs no scan: changing one cipher byte changes at most that
    plain byte, its successor, and (for the last two bytes of a band) the
    first byte of the previous band."""
    H, W, C, n, r = 12, 5, 3, 4, 1
    rng = np.random.default_rng(1)
    Z = rng.integers(0, 256, (H, W, C), dtype=np.uint8)
    ks = rng.integers(0, 256, Z.size, dtype=np.uint8)
    Y = orc.undiffuse(Z, n, r, 0, ks).ravel()
    for pos in range(Z.size):
        Z2 = Z.copy().ravel()
        Z2[pos] ^= 0x5A
        Y2 = orc.undiffuse(Z2.reshape(Z.shape), n, r, 0, ks).ravel()
        assert 1 <= np.count_nonzero(Y2 != Y) <= 3
