"""Seeded synthetic inputs: video frames, PLCM keys and confusion seeds.

This module holds none of the cipher's arithmetic.  It is the only code the
GPU path and the CPU oracle share: both are fed the same frames and keys.

The paper encrypts videos from a public video trace library, resized to
96^2 ... 960^2 RGB (Sec. 3, Tab. 2), and standard 512x512 test images
(Sec. 4).  Neither is available here; the correlated generator below stands
in for them: two moving 2-D sinusoidal gradients plus Gaussian noise
(sigma=8), clipped to 0..255, which gives the strong adjacent-pixel
correlation (>0.9) of natural frames that Sec. 4 measures.

Keys follow the ranges of Sec. 3, Eq. (5): initial values x0 in (0,1) and
control parameters p in (0,1/2), both open; one record (x0_1, p_1, x0_2,
p_2) per subframe.  Confusion seeds s_c are positive integers (Sec. 2,
Eq. 1), drawn uniformly from 1..65535.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


class CorrelatedVideo:
    """Moving-gradient video generator.

    I(t,y,x,c) = clip(round(128 + 60 sin(2pi(f1x x + f1y y - v1 t) + phi_c)
                                + 40 sin(2pi(f2x x - f2y y + v2 t) + psi_c)
                                + N(0, 8^2)), 0, 255)
    with frequencies f ~ U[1/256, 1/32] cycles/pixel, speeds v ~ U[0.01,
    0.05] cycles/frame and one phase pair per channel.  Frame t is a pure
    function of (seed, t), so any subset of frames can be regenerated.
    """

    def __init__(self, H: int, W: int, C: int, seed: int):
        self.H, self.W, self.C, self.seed = H, W, C, seed
        r = _rng(seed)
        self.f1x, self.f1y, self.f2x, self.f2y = r.uniform(1 / 256, 1 / 32, 4)
        self.v1, self.v2 = r.uniform(0.01, 0.05, 2)
        self.phi = r.uniform(0, TWO_PI, C)
        self.psi = r.uniform(0, TWO_PI, C)
        self._y = np.arange(H, dtype=np.float64)[:, None]
        self._x = np.arange(W, dtype=np.float64)[None, :]

    def frame(self, t: int) -> np.ndarray:
        H, W, C = self.H, self.W, self.C
        out = np.empty((H, W, C), np.uint8)
        base1 = TWO_PI * (self.f1x * self._x + self.f1y * self._y - self.v1 * t)
        base2 = TWO_PI * (self.f2x * self._x - self.f2y * self._y + self.v2 * t)
        noise = _rng((self.seed << 20) + t).standard_normal((H, W, C), np.float32) * 8.0
        for c in range(C):
            v = 128.0 + 60.0 * np.sin(base1 + self.phi[c]) + 40.0 * np.sin(base2 + self.psi[c])
            v = v.astype(np.float32) + noise[:, :, c]
            out[:, :, c] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
        return out

    def frames(self, t0: int, T: int) -> np.ndarray:
        return np.stack([self.frame(t0 + k) for k in range(T)])

    def frames_torch(self, t0: int, T: int, device):
        """The same recipe evaluated with torch on `device` (float32, torch's
        own seeded normal noise), for workloads too large to generate on the
        host.  Returns a contiguous uint8 tensor (T, H, W, C).  The values
        differ from frames() (another noise source); each consumer uses one
        of the two consistently."""
        import torch
        H, W, C = self.H, self.W, self.C
        g = torch.Generator(device=device)
        g.manual_seed((self.seed << 20) + t0)
        y = torch.arange(H, device=device, dtype=torch.float32).view(1, H, 1)
        x = torch.arange(W, device=device, dtype=torch.float32).view(1, 1, W)
        t = torch.arange(t0, t0 + T, device=device, dtype=torch.float32).view(T, 1, 1)
        base1 = TWO_PI * (self.f1x * x + self.f1y * y - self.v1 * t)
        base2 = TWO_PI * (self.f2x * x - self.f2y * y + self.v2 * t)
        out = torch.empty((T, H, W, C), dtype=torch.uint8, device=device)
        for c in range(C):
            v = 128.0 + 60.0 * torch.sin(base1 + float(self.phi[c])) \
                + 40.0 * torch.sin(base2 + float(self.psi[c]))
            v = v + 8.0 * torch.randn((T, H, W), generator=g, device=device, dtype=torch.float32)
            out[..., c] = v.round_().clamp_(0, 255).to(torch.uint8)
        return out


def uniform_frames(H: int, W: int, C: int, T: int, seed: int) -> np.ndarray:
    """Independent uniform bytes (the 256x256 grayscale single-frame case)."""
    return _rng(seed).integers(0, 256, size=(T, H, W, C), dtype=np.uint8)


def _open_uniform(r: np.random.Generator, lo: float, hi: float, size: int) -> np.ndarray:
    v = r.uniform(lo, hi, size)
    bad = (v <= lo) | (v >= hi)
    while bad.any():
        v[bad] = r.uniform(lo, hi, int(bad.sum()))
        bad = (v <= lo) | (v >= hi)
    return v


def plcm_key(n: int, seed: int) -> np.ndarray:
    """n PLCM key records (x0_1, p_1, x0_2, p_2) as an (n, 4) float64 array."""
    r = _rng(seed)
    pm = np.empty((n, 4), np.float64)
    pm[:, 0] = _open_uniform(r, 0.0, 1.0, n)
    pm[:, 1] = _open_uniform(r, 0.0, 0.5, n)
    pm[:, 2] = _open_uniform(r, 0.0, 1.0, n)
    pm[:, 3] = _open_uniform(r, 0.0, 0.5, n)
    return pm


# Admissible control parameters of the 2DLASM (Sec. 3, Eq. (6)).
LASM_MU_RANGES = [(0.37, 0.38), (0.4, 0.42), (0.44, 0.93)]


def lasm_key(n: int, seed: int) -> np.ndarray:
    """n 2DLASM key records (x0_1, y0_1, mu_1, x0_2, y0_2, mu_2) as an (n, 6)
    float64 array: initial values in (0,1), mu uniform over the admissible
    intervals (weighted by length)."""
    r = _rng(seed)
    pm = np.empty((n, 6), np.float64)
    lens = np.array([b - a for a, b in LASM_MU_RANGES])
    for m in range(2):
        pm[:, 3 * m] = _open_uniform(r, 0.0, 1.0, n)
        pm[:, 3 * m + 1] = _open_uniform(r, 0.0, 1.0, n)
        k = r.choice(len(LASM_MU_RANGES), size=n, p=lens / lens.sum())
        pm[:, 3 * m + 2] = [r.uniform(*LASM_MU_RANGES[i]) for i in k]
    return pm


def confusion_seeds(T: int, seed: int) -> np.ndarray:
    """One confusion seed per frame, uniform on 1..65535."""
    return _rng(seed + 7919).integers(1, 65536, size=T, dtype=np.uint32)


# The five workloads of the benchmark suite (sizes, subframe counts, rounds).
WORKLOADS = {
    "gray256": dict(H=256, W=256, C=1, n=4, r=5, T=1, kind="uniform", seed=1000),
    "rgb480": dict(H=480, W=480, C=3, n=8, r=5, T=240, kind="correlated", seed=1001),
    "rgb768": dict(H=768, W=768, C=3, n=16, r=5, T=1440, kind="correlated", seed=1002),
}


def batched_streams(count: int, seed: int):
    """Multi-stream tick workload: per stream (H, W, C, n), resolution uniform
    over 480^2, 576^2, 768^2 and 1920x1080 (3 channels), n uniform over
    8/16/32."""
    r = _rng(seed)
    sizes = [(480, 480), (576, 576), (768, 768), (1080, 1920)]
    out = []
    for _ in range(count):
        H, W = sizes[int(r.integers(0, len(sizes)))]
        out.append((H, W, 3, int((8, 16, 32)[int(r.integers(0, 3))])))
    return out


SERVED_SIZES = [(480, 480), (576, 576), (768, 768), (720, 1280), (1080, 1920), (2160, 3840)]


def served_streams(count: int, seed: int, decrypt_share: float = 0.2):
    """Serving workload: per stream (H, W, C, n, decrypt), resolution uniform
    over SERVED_SIZES (3 channels), n the smallest of 8/16/32/64 whose
    tallest band holds at most 800 KB, and a decrypt_share of the streams
    decrypting."""
    r = _rng(seed)
    out = []
    for _ in range(count):
        H, W = SERVED_SIZES[int(r.integers(0, len(SERVED_SIZES)))]
        n = next(n for n in (8, 16, 32, 64) if -(-H // n) * W * 3 <= 800_000)
        out.append((H, W, 3, n, bool(r.random() < decrypt_share)))
    return out


def poisson_arrivals(count: int, rate: float, seconds: float, seed: int):
    """Arrival times of `count` independent Poisson streams of `rate` frames
    per second over `seconds`: a list of (time, stream) sorted by time."""
    r = _rng(seed)
    ev = []
    for s in range(count):
        t = r.exponential(1.0 / rate)
        while t < seconds:
            ev.append((t, s))
            t += r.exponential(1.0 / rate)
    ev.sort()
    return ev


def adjacent_correlation(frame: np.ndarray, axis: int) -> float:
    """Pearson correlation of horizontally (axis=1) or vertically (axis=0)
    adjacent pixel values over all channels; used to validate the generator."""
    f = frame.astype(np.float64)
    if axis == 1:
        a, b = f[:, :-1], f[:, 1:]
    else:
        a, b = f[:-1], f[1:]
    return float(np.corrcoef(a.ravel(), b.ravel())[0, 1])
