"""Whole-cipher pins of the oracle: Algorithms 1-2 with r rounds of
Eq. (1) + Eq. (3), decryption by Eq. (4) + Eq. (2), PRBG state across
frames, and the differential / error-propagation behaviour the paper reports
(Sec. 4-5)."""
import numpy as np
import pytest

from paper_2302_07411_amd.inputs import (CorrelatedVideo, confusion_seeds, plcm_key,
                                         uniform_frames)

SHAPES = [
    (256, 256, 1, 4, 5, 1),     # the paper-literal gray case
    (48, 48, 3, 8, 5, 3),
    (20, 36, 3, 3, 5, 2),       # non-square, n does not divide H
    (36, 20, 3, 5, 2, 2),
    (9, 9, 1, 9, 3, 2),         # one row per band
    (17, 3, 1, 1, 5, 2),        # one band, seeds itself
    (30, 30, 3, 7, 1, 2),       # a single round
]


@pytest.mark.parametrize("H,W,C,n,r,T", SHAPES)
def test_round_trip(orc, H, W, C, n, r, T):
    pm = plcm_key(n, H * 1000 + W)
    frames = uniform_frames(H, W, C, T, seed=H + W)
    s_c = confusion_seeds(T, H)
    enc = orc.PlcmKey(H, W, C, n, r, pm)
    dec = orc.PlcmKey(H, W, C, n, r, pm)
    cipher = enc.encrypt(frames, s_c)
    assert not np.array_equal(cipher, frames)
    assert np.array_equal(dec.decrypt(cipher, s_c), frames)
    # both keys advanced identically
    assert np.array_equal(enc.x1, dec.x1) and np.array_equal(enc.x2, dec.x2)


def test_state_continues_across_calls(orc):
    H, W, C, n, r = 24, 24, 3, 4, 5
    pm = plcm_key(n, 5)
    frames = CorrelatedVideo(H, W, C, 9).frames(0, 5)
    s_c = confusion_seeds(5, 9)
    whole = orc.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    k = orc.PlcmKey(H, W, C, n, r, pm)
    parts = np.concatenate([k.encrypt(frames[:2], s_c[:2]), k.encrypt(frames[2:], s_c[2:])])
    assert np.array_equal(whole, parts)
    # the same frame twice gives different cipher frames (fresh keystream)
    twice = orc.PlcmKey(H, W, C, n, r, pm).encrypt(np.stack([frames[0]] * 2), [s_c[0]] * 2)
    assert not np.array_equal(twice[0], twice[1])


def test_encrypt_matches_composed_steps(orc):
    """The whole-frame routine equals keystream, g table, then r x (Eq. (1),
    Eq. (3)) composed from the separately pinned steps."""
    H, W, C, n, r = 20, 12, 3, 3, 5
    pm = plcm_key(n, 21)
    f = uniform_frames(H, W, C, 1, 4)[0]
    s_c = 4321
    ks = orc.PlcmKey(H, W, C, n, r, pm).keystream(1)[0]
    g = orc.gtable(H, s_c)
    A = f
    for j in range(r):
        A = orc.diffuse(orc.confuse(A, g), n, r, j, ks)
    got = orc.PlcmKey(H, W, C, n, r, pm).encrypt(f[None], [s_c])[0]
    assert np.array_equal(got, A)


def _encrypt_with_fixed_keystream(orc, frame, n, r, ks, g):
    A = frame
    for j in range(r):
        A = orc.diffuse(orc.confuse(A, g), n, r, j, ks)
    return A


def test_npcr_uaci_sec5(orc):
    """Sec. 5 differential test at 512x512: change one pixel's value by one
    (its least significant bit flips), encrypt with the same byte sequences;
    NPCR must exceed 99.5893% and UACI fall in [33.3730%, 33.5541%] (the
    paper's 5% thresholds)."""
    H = W = 512
    n, r = 8, 5
    rng = np.random.default_rng(2024)
    frame = CorrelatedVideo(H, W, 1, 3).frame(0)
    ks = orc.PlcmKey(H, W, 1, n, r, plcm_key(n, 8)).keystream(1)[0]
    g = orc.gtable(H, 1234)
    c1 = _encrypt_with_fixed_keystream(orc, frame, n, r, ks, g)
    for _ in range(3):
        f2 = frame.copy()
        a, o = rng.integers(0, H), rng.integers(0, W)
        f2[a, o, 0] ^= 1
        c2 = _encrypt_with_fixed_keystream(orc, f2, n, r, ks, g)
        npcr = 100.0 * np.count_nonzero(c1 != c2) / c1.size
        uaci = 100.0 * np.abs(c1.astype(np.int32) - c2).sum() / (255.0 * c1.size)
        assert npcr > 99.5893
        assert 33.3730 <= uaci <= 33.5541


def test_cipher_histogram_sec4(orc):
    """Sec. 4: chi-square of the cipher histogram below 293.25 and entropy
    close to 8 bits, on a strongly correlated frame."""
    H = W = 256
    frame = CorrelatedVideo(H, W, 3, 17).frame(0)
    c = orc.PlcmKey(H, W, 3, 8, 5, plcm_key(8, 17)).encrypt(frame[None], [777])[0]
    for ch in range(3):
        hist = np.bincount(c[..., ch].ravel(), minlength=256).astype(np.float64)
        e = H * W / 256
        assert ((hist - e) ** 2 / e).sum() < 293.25
        p = hist / hist.sum()
        assert -(p[p > 0] * np.log2(p[p > 0])).sum() > 7.99


@pytest.mark.parametrize("r", [1, 2, 3, 5])
def test_error_propagation_bound(orc, r):
    """Decryption of a cipher frame with one corrupted byte: Eq. (4) makes
    each plain byte depend on two cipher bytes (or the next band's last two
    for a band's first byte), and Eq. (2) only moves bytes, so at most 3^r
    bytes come out wrong and every other byte is exact (the mechanism behind
    the noise and data-loss experiments of Sec. 5)."""
    H, W, C, n = 32, 32, 3, 4
    pm = plcm_key(n, 99)
    frame = uniform_frames(H, W, C, 1, 3)
    cipher = orc.PlcmKey(H, W, C, n, r, pm).encrypt(frame, [55])
    rng = np.random.default_rng(r)
    for _ in range(20):
        bad = cipher.copy().reshape(-1)
        bad[rng.integers(0, bad.size)] ^= 0xFF
        plain = orc.PlcmKey(H, W, C, n, r, pm).decrypt(bad.reshape(cipher.shape), [55])
        wrong = np.count_nonzero(plain != frame)
        assert 1 <= wrong <= 3 ** r


@pytest.mark.parametrize("bit", [7, 6, 4])
def test_high_bit_differences_stay_high(orc, bit):
    """Structure of Eq. (3): modular addition carries only upwards, XOR and
    the permutation of Eq. (1) act bitwise, so a plaintext difference
    confined to bits >= k stays confined to bits >= k through every round.
    A flip of bit 7 alone changes only bit 7 of any cipher byte."""
    H, W, C, n, r = 64, 64, 3, 4, 5
    pm = plcm_key(n, 1)
    frame = uniform_frames(H, W, C, 1, 8)
    f2 = frame.copy()
    f2[0, 13, 1, 2] ^= 1 << bit
    c1 = orc.PlcmKey(H, W, C, n, r, pm).encrypt(frame, [321])
    c2 = orc.PlcmKey(H, W, C, n, r, pm).encrypt(f2, [321])
    diff = c1 ^ c2
    low_mask = (1 << bit) - 1
    assert np.count_nonzero(diff & low_mask) == 0
    assert np.count_nonzero(diff) > 0.4 * diff.size
