"""Statistical and security measures of cipher frames (Sec. 4 and 5 of the
paper), computed on the host from frames the GPU library produced.

Each function follows the paper's definition:
  - histogram variance and chi-square (Sec. 4, uniformity);
  - correlation of adjacent pixels, horizontal / vertical / diagonal, over
    randomly chosen pairs (Sec. 4);
  - information entropy and the (k, T_B) local Shannon entropy (Sec. 4);
  - NPCR and UACI between two cipher frames (Sec. 5, differential attacks);
  - PSNR, salt-and-pepper noise and block loss for the robustness tests
    (Sec. 5, noise and data loss).
Frames are uint8 arrays of shape (H, W) or (H, W, C); the statistics are
taken per channel where the paper tabulates them per channel.
"""
from __future__ import annotations

import numpy as np

CHI2_CRITICAL_005 = 293.25         # chi-square(0.05, 255), Sec. 4
NPCR_MIN_512 = 99.5893             # expected NPCR at 512x512, significance 0.05, Sec. 5
UACI_RANGE_512 = (33.3730, 33.5541)
LOCAL_ENTROPY_K, LOCAL_ENTROPY_TB = 30, 1936


def _channels(frame: np.ndarray):
    f = np.asarray(frame)
    return [f] if f.ndim == 2 else [f[..., c] for c in range(f.shape[-1])]


def histogram(channel: np.ndarray) -> np.ndarray:
    return np.bincount(np.asarray(channel, np.uint8).reshape(-1), minlength=256).astype(np.float64)


def histogram_variance(channel: np.ndarray) -> float:
    """var(Z) = (1/256^2) sum_i sum_j (z_i - z_j)^2 / 2 over the histogram Z."""
    z = histogram(channel)
    return float(((z[:, None] - z[None, :]) ** 2).sum() / 2.0 / 256.0 ** 2)


def chi_square(channel: np.ndarray) -> float:
    """sum_i (z_i - N/256)^2 / (N/256)."""
    z = histogram(channel)
    e = z.sum() / 256.0
    return float(((z - e) ** 2 / e).sum())


def correlation(x: np.ndarray, y: np.ndarray) -> float:
    """r = cov(x, y) / sqrt(D(x) D(y)) with the 1/N moments of the paper."""
    x = np.asarray(x, np.float64).reshape(-1)
    y = np.asarray(y, np.float64).reshape(-1)
    dx, dy = x - x.mean(), y - y.mean()
    den = np.sqrt((dx * dx).mean() * (dy * dy).mean())
    return float((dx * dy).mean() / den) if den > 0 else float("nan")


def adjacent_correlation(channel: np.ndarray, pairs: int, rng: np.random.Generator) -> dict:
    """Correlation of `pairs` randomly chosen horizontally, vertically and
    diagonally adjacent pixel pairs."""
    c = np.asarray(channel)
    H, W = c.shape
    out = {}
    for name, (di, dj) in (("h", (0, 1)), ("v", (1, 0)), ("d", (1, 1))):
        i = rng.integers(0, H - di, pairs)
        j = rng.integers(0, W - dj, pairs)
        out[name] = correlation(c[i, j], c[i + di, j + dj])
    return out


def entropy(values: np.ndarray) -> float:
    """H = sum_i p_i log2(1 / p_i) over the byte values present."""
    z = histogram(values)
    p = z[z > 0] / z.sum()
    return float(-(p * np.log2(p)).sum())


def local_entropy(channel: np.ndarray, rng: np.random.Generator, k: int = LOCAL_ENTROPY_K,
                  tb: int = LOCAL_ENTROPY_TB) -> float:
    """Mean entropy of k randomly chosen non-overlapping square blocks of
    tb pixels (tb a perfect square; 1936 = 44 x 44)."""
    side = int(round(np.sqrt(tb)))
    assert side * side == tb
    c = np.asarray(channel)
    gh, gw = c.shape[0] // side, c.shape[1] // side
    assert gh * gw >= k, "frame too small for k blocks"
    cells = rng.choice(gh * gw, size=k, replace=False)
    hs = [entropy(c[(q // gw) * side:(q // gw + 1) * side, (q % gw) * side:(q % gw + 1) * side])
          for q in cells]
    return float(np.mean(hs))


def npcr(c1: np.ndarray, c2: np.ndarray) -> float:
    """Percentage of positions whose values differ (per byte of a channel)."""
    a, b = np.asarray(c1), np.asarray(c2)
    return float(np.count_nonzero(a != b) * 100.0 / a.size)


def uaci(c1: np.ndarray, c2: np.ndarray) -> float:
    """Mean |c1 - c2| / 255, in percent."""
    a, b = np.asarray(c1, np.int16), np.asarray(c2, np.int16)
    return float(np.abs(a - b).sum() * 100.0 / (255.0 * a.size))


def psnr(ref: np.ndarray, test: np.ndarray) -> float:
    d = np.asarray(ref, np.float64) - np.asarray(test, np.float64)
    mse = float((d * d).mean())
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def salt_and_pepper(frame: np.ndarray, fraction: float, rng: np.random.Generator) -> np.ndarray:
    """Set `fraction` of the pixels (all channels of a pixel) to 0 or 255."""
    f = np.array(frame, copy=True)
    H, W = f.shape[:2]
    m = rng.random((H, W)) < fraction
    v = np.where(rng.random((H, W)) < 0.5, 0, 255).astype(np.uint8)
    f[m] = v[m][:, None] if f.ndim == 3 else v[m]
    return f


def block_loss(frame: np.ndarray, size: int, value: int, rng: np.random.Generator) -> np.ndarray:
    """Replace one randomly placed size x size block with `value`."""
    f = np.array(frame, copy=True)
    H, W = f.shape[:2]
    i = int(rng.integers(0, H - size + 1))
    j = int(rng.integers(0, W - size + 1))
    f[i:i + size, j:j + size] = value
    return f


def frame_summary(plain: np.ndarray, cipher: np.ndarray, rng: np.random.Generator,
                  pairs: int = 20000) -> dict:
    """The Sec. 4 table entries for one plain/cipher frame pair, per channel."""
    out = {"chi2": [], "variance_plain": [], "variance_cipher": [], "entropy": [],
           "local_entropy": [], "corr_plain": [], "corr_cipher": []}
    for p, c in zip(_channels(plain), _channels(cipher)):
        out["chi2"].append(chi_square(c))
        out["variance_plain"].append(histogram_variance(p))
        out["variance_cipher"].append(histogram_variance(c))
        out["entropy"].append(entropy(c))
        out["local_entropy"].append(local_entropy(c, rng))
        out["corr_plain"].append(adjacent_correlation(p, pairs, rng))
        out["corr_cipher"].append(adjacent_correlation(c, pairs, rng))
    return out
