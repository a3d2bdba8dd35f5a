"""The statistical harness (paper_2302_07411_amd.analysis) pinned to closed
forms of the paper's definitions (Sec. 4 and 5): histograms with known
variance and chi-square, distributions with known entropy, exactly
correlated and anti-correlated samples, the exact NPCR/UACI of all 65,536
byte pairs (the expected values for independent uniform ciphers)."""
import numpy as np
import pytest

from paper_2302_07411_amd import analysis as A

N = 256 * 64  # pixels in the synthetic histograms


def _img(values):
    return np.asarray(values, np.uint8).reshape(128, -1)


def test_uniform_histogram():
    u = _img(np.tile(np.arange(256), N // 256))
    assert A.histogram_variance(u) == 0.0
    assert A.chi_square(u) == 0.0
    assert A.entropy(u) == 8.0


def test_single_value_histogram():
    s = _img(np.full(N, 17))
    # z = (0, ..., N, ..., 0): 255 ordered pairs each way with (N - 0)^2 / 2
    assert A.histogram_variance(s) == pytest.approx(255 * N ** 2 / 256 ** 2, rel=1e-12)
    # (N - N/256)^2/(N/256) + 255 * N/256 = 255 N
    assert A.chi_square(s) == pytest.approx(255 * N, rel=1e-12)
    assert A.entropy(s) == 0.0


def test_two_value_histogram():
    t = _img(np.repeat([3, 200], N // 2))
    # equal counts N/2 at two values: only the 2 * 2 * 254 ordered pairs with an
    # empty bin contribute, each (N/2)^2 / 2
    assert A.histogram_variance(t) == pytest.approx(127 * N ** 2 / 256 ** 2, rel=1e-12)
    assert A.chi_square(t) == pytest.approx(127 * N, rel=1e-12)
    assert A.entropy(t) == 1.0
    q = _img(np.concatenate([np.full(N // 2, 1), np.full(N // 4, 2), np.full(N // 4, 3)]))
    assert A.entropy(q) == 1.5


def test_correlation():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, 5000)
    assert A.correlation(x, x) == pytest.approx(1.0, abs=1e-12)
    assert A.correlation(x, 255 - x) == pytest.approx(-1.0, abs=1e-12)
    ramp = np.tile(np.arange(200, dtype=np.uint8), (150, 1))  # c[i, j] = j
    r = A.adjacent_correlation(ramp, 3000, rng)
    assert r["h"] == pytest.approx(1.0, abs=1e-12)   # (j, j+1)
    assert r["v"] == pytest.approx(1.0, abs=1e-12)   # (j, j)
    assert r["d"] == pytest.approx(1.0, abs=1e-12)


def test_local_entropy():
    rng = np.random.default_rng(2)
    i, j = np.indices((44 * 6, 44 * 6))
    checker = np.where((i + j) % 2 == 0, 10, 250).astype(np.uint8)  # every 44x44 block half/half
    assert A.local_entropy(checker, rng) == 1.0
    assert A.local_entropy(np.zeros((300, 300), np.uint8), rng) == 0.0
    # with k equal to the number of grid cells every cell is used once
    img = rng.integers(0, 256, (88, 132), dtype=np.uint8)
    cells = [A.entropy(img[a:a + 44, b:b + 44]) for a in (0, 44) for b in (0, 44, 88)]
    assert A.local_entropy(img, rng, k=6) == pytest.approx(np.mean(cells), abs=1e-12)


def test_npcr_uaci_exact():
    a, b = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    a, b = a.astype(np.uint8), b.astype(np.uint8)
    # all 65,536 pairs once: the expected values for independent uniform bytes
    assert A.npcr(a, b) == pytest.approx(100.0 * (1 - 1 / 256), abs=1e-12)
    d = np.arange(1, 256)
    want_uaci = 100.0 * 2 * (d * (256 - d)).sum() / (256 ** 2 * 255)
    assert A.uaci(a, b) == pytest.approx(want_uaci, abs=1e-12)
    assert round(want_uaci, 4) == 33.4635          # the value the paper quotes
    c = np.arange(256, dtype=np.uint8)
    assert A.npcr(c, c) == 0.0 and A.uaci(c, c) == 0.0
    assert A.uaci(c, 255 - c) == pytest.approx(100.0 * 128 / 255, abs=1e-12)  # mean |2c - 255| = 128


def test_psnr_noise_and_loss():
    rng = np.random.default_rng(3)
    f = rng.integers(1, 255, (400, 300, 3), dtype=np.uint8)
    assert A.psnr(f, f) == float("inf")
    assert A.psnr(f, f + 1) == pytest.approx(10 * np.log10(255.0 ** 2), abs=1e-9)
    g = A.salt_and_pepper(f, 0.03, rng)
    hit = np.any(g != f, axis=2)
    assert abs(hit.mean() - 0.03) < 0.003
    assert np.isin(g[hit], [0, 255]).all()
    assert (g[hit] == g[hit][:, :1]).all()          # the whole pixel takes one value
    h = A.block_loss(f, 64, 255, rng)
    assert np.count_nonzero(np.any(h != f, axis=2)) == 64 * 64
