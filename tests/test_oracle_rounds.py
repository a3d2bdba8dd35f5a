"""Pins of the oracle's keystream-driven rounds (`oracle_rounds`) and of the
2DLASM keystream's frame/band layout (`oracle_lasm_keystream`), each against
separately pinned pieces rather than against itself:

  - the rounds of T frames with an arbitrary keystream (random bytes, not a
    generator's) equal a per-frame composition of the pinned primitives
    (Eq. (1) + Eq. (3) per round, Eq. (4) + Eq. (2) in reverse; Algorithm 2's
    round loop), frame t using bytes [t*r*F, (t+1)*r*F) of the keystream;
  - with a PLCM keystream they equal the PLCM cipher (Algorithms 1-2), which
    is pinned by composition in test_oracle_cipher.py;
  - frame t, band i of the 2DLASM keystream is the slice
    [t*r*F + r*lo_i*W*C, +r*S_i) and equals the pinned byte generator
    (Sec. 3, Eq. (6) and the byte extraction) run on band i's record,
    continued from frame to frame.

Shapes have r >= 2, T >= 2 and bands of unequal height, so that an offset of
t*F instead of t*r*F, or lo*W*C instead of r*lo*W*C, changes the result.
"""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import (confusion_seeds, lasm_key, plcm_key,
                                         uniform_frames)

SHAPES = [
    (10, 6, 3, 3, 2, 3),     # bands of 3, 3, 4 rows
    (20, 36, 3, 3, 5, 2),    # non-square, n does not divide H
    (9, 9, 1, 9, 3, 2),      # one row per band
    (17, 3, 1, 1, 4, 2),     # one band, seeds itself
]


def _compose(H, W, C, n, r, decrypt, ks, frames, s_c):
    F = H * W * C
    out = []
    for t, f in enumerate(frames):
        k = ks[t * r * F:(t + 1) * r * F]
        g = oracle.gtable(H, int(s_c[t]))
        A = f
        if not decrypt:
            for j in range(r):
                A = oracle.diffuse(oracle.confuse(A, g), n, r, j, k)
        else:
            for j in reversed(range(r)):
                A = oracle.unconfuse(oracle.undiffuse(A, n, r, j, k), g)
        out.append(A)
    return np.stack(out)


@pytest.mark.parametrize("H,W,C,n,r,T", SHAPES)
def test_rounds_equal_composed_primitives(H, W, C, n, r, T):
    ks = np.random.default_rng(H * 7 + W).integers(0, 256, T * r * H * W * C, dtype=np.uint8)
    frames = uniform_frames(H, W, C, T, seed=3 + H)
    s_c = confusion_seeds(T, 5 + W)
    enc = oracle.rounds(H, W, C, n, r, False, ks, frames, s_c)
    assert np.array_equal(enc, _compose(H, W, C, n, r, False, ks, frames, s_c))
    dec = oracle.rounds(H, W, C, n, r, True, ks, enc, s_c)
    assert np.array_equal(dec, _compose(H, W, C, n, r, True, ks, enc, s_c))
    assert np.array_equal(dec, frames)


@pytest.mark.parametrize("H,W,C,n,r,T", SHAPES)
def test_rounds_with_plcm_keystream_equal_the_plcm_cipher(H, W, C, n, r, T):
    pm = plcm_key(n, 100 + H)
    frames = uniform_frames(H, W, C, T, seed=7 + W)
    s_c = confusion_seeds(T, 11 + H)
    ks = oracle.PlcmKey(H, W, C, n, r, pm).keystream(T)
    cipher = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    assert np.array_equal(oracle.rounds(H, W, C, n, r, False, ks, frames, s_c), cipher)
    assert np.array_equal(oracle.rounds(H, W, C, n, r, True, ks, cipher, s_c),
                          oracle.PlcmKey(H, W, C, n, r, pm).decrypt(cipher, s_c))


@pytest.mark.parametrize("H,W,C,n,r,T", [(10, 6, 3, 3, 2, 3), (7, 4, 1, 2, 3, 2)])
def test_lasm_keystream_layout_by_band_and_frame(H, W, C, n, r, T):
    pm = lasm_key(n, 60 + H)
    ks = oracle.LasmKey(H, W, C, n, r, pm).keystream(T)
    row, F = W * C, H * W * C
    assert ks.shape == (T, r * F)
    maps = [[tuple(pm[i, 0:3]), tuple(pm[i, 3:6])] for i in range(n)]
    for t in range(T):
        for i in range(n):
            lo, hi = oracle.band_lo(H, n, i), oracle.band_lo(H, n, i + 1)
            S = (hi - lo) * row
            want, s1, s2 = oracle.lasm_bytes(maps[i][0], maps[i][1], r * S)
            maps[i] = [(s1[0], s1[1], maps[i][0][2]), (s2[0], s2[1], maps[i][1][2])]
            flat = ks.reshape(-1)
            got = flat[t * r * F + r * lo * row: t * r * F + r * lo * row + r * S]
            assert np.array_equal(got, want), (t, i)
