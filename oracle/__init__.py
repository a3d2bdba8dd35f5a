"""CPU oracle of the chaotic video cipher -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper over ``oracle.c``: plain, slow, single-threaded C written
step by step from the paper (Jiang, Yuan, Li, Lu, arXiv 2302.07411; Sec. 2
Eqs. (1)-(4) and Algorithms 1-2, Sec. 3 Eq. (5) and the PLCM byte
generator).  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
loads it, and the two share no code.

Pins (tests/test_oracle_*.py): exact-rational PLCM orbits, the special
orbits of Eq. (5), the 2DLASM sine against mpmath and the special orbits
and reductions of Eq. (6), hand-traced confusion and diffusion fixtures
(tests/golden/), the skew/row-rotation factorisation of Eq. (1), the
prefix-XOR closed form of Eq. (3), high-precision g tables, round trips,
bijection/histogram invariants, and the NPCR/UACI and error-propagation
bounds the construction implies.

``paper_mt.c`` (same library) is the paper's multithreaded CPU design (one
thread per subframe, two barriers per round), built on the oracle's
primitives and checked against it; ``bench.py`` times it on the GPU
machine's host as the paper-design CPU baseline.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_MT = os.path.join(_HERE, "paper_mt.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# binary64 throughout, one IEEE operation per C operator: no FMA contraction,
# no fast-math, SSE2 (the x86-64 default), no flush-to-zero.
CFLAGS = ["-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-fno-unsafe-math-optimizations"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc and return its path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-pthread", "-o", tmp, _SRC, _SRC_MT,
                               "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ct.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_SRC_MT)):
            build()
        L = ct.CDLL(_LIB)
        u8p = ct.POINTER(ct.c_uint8)
        dp = ct.POINTER(ct.c_double)
        u32 = ct.c_uint32
        L.oracle_plcm.restype = ct.c_double
        L.oracle_plcm.argtypes = [ct.c_double, ct.c_double]
        L.oracle_plcm_bytes.restype = None
        L.oracle_plcm_bytes.argtypes = [dp, ct.c_double, dp, ct.c_double, ct.c_uint64, u8p]
        L.oracle_band_lo.restype = u32
        L.oracle_band_lo.argtypes = [u32, u32, u32]
        L.oracle_gtable.restype = None
        L.oracle_gtable.argtypes = [u32, u32, ct.POINTER(ct.c_int64)]
        for name in ("oracle_confuse", "oracle_unconfuse"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [u8p, u8p, u32, u32, u32, ct.POINTER(ct.c_int64)]
        for name in ("oracle_diffuse", "oracle_undiffuse"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [u8p, u8p, u32, u32, u32, u32, u32, u32, u8p]
        L.oracle_plcm_keystream.restype = None
        L.oracle_plcm_keystream.argtypes = [u32, u32, u32, u32, u32, dp, dp, dp, dp,
                                            ct.c_uint64, u8p]
        for name in ("oracle_encrypt", "oracle_decrypt"):
            f = getattr(L, name)
            f.restype = ct.c_int
            f.argtypes = [u32, u32, u32, u32, u32, dp, dp, dp, dp, u8p, u8p,
                          ct.POINTER(ct.c_uint32), ct.c_uint64]
        L.oracle_cr_sin_margin.restype = ct.c_int
        L.oracle_cr_sin_margin.argtypes = [ct.c_double, dp, ct.c_int]
        L.oracle_key_schedule.restype = ct.c_int
        L.oracle_key_schedule.argtypes = [ct.c_int, dp, u32, dp, ct.c_uint64,
                                          ct.POINTER(ct.c_uint32), ct.c_uint64]
        L.paper_mt_encrypt.restype = ct.c_int
        L.paper_mt_encrypt.argtypes = [u32, u32, u32, u32, u32, dp, dp, u8p, u8p,
                                       ct.POINTER(ct.c_uint32), ct.c_uint64]
        L.oracle_cr_sin_array.restype = ct.c_uint64
        L.oracle_cr_sin_array.argtypes = [dp, dp, ct.c_uint64]
        L.oracle_cr_sin.restype = ct.c_int
        L.oracle_cr_sin.argtypes = [ct.c_double, dp]
        L.oracle_lasm.restype = ct.c_int
        L.oracle_lasm.argtypes = [dp, dp, ct.c_double]
        L.oracle_lasm_bytes.restype = ct.c_int
        L.oracle_lasm_bytes.argtypes = [dp, dp, ct.c_double, dp, dp, ct.c_double, ct.c_uint64, u8p]
        L.oracle_lasm_keystream.restype = ct.c_int
        L.oracle_lasm_keystream.argtypes = [u32, u32, u32, u32, u32, dp, dp, dp, dp, dp, dp,
                                            ct.c_uint64, u8p]
        L.oracle_rounds.restype = ct.c_int
        L.oracle_rounds.argtypes = [u32, u32, u32, u32, u32, ct.c_int, u8p, u8p, u8p,
                                    ct.POINTER(ct.c_uint32), ct.c_uint64]
        _lib = L
    return _lib


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_uint8))


def _f64(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


# ------------------------------------------------------------ primitives ---

def plcm(x: float, p: float) -> float:
    """Eq. (5), one step."""
    return lib().oracle_plcm(x, p)


def plcm_bytes(x1: float, p1: float, x2: float, p2: float, nbytes: int):
    """PLCM byte generator (Sec. 3).  Returns (bytes, x1', x2')."""
    a = ct.c_double(x1)
    b = ct.c_double(x2)
    out = np.zeros(nbytes, np.uint8)
    lib().oracle_plcm_bytes(ct.byref(a), p1, ct.byref(b), p2, nbytes, _u8(out))
    return out, a.value, b.value


class Undecided(ArithmeticError):
    """A sine value too close to a binary64 rounding boundary to round."""


def cr_sin(t: float) -> float:
    """RN(sin(t)), binary128 evaluation rounded once (Sec. 3, Eq. (6)'s sine)."""
    out = ct.c_double()
    if lib().oracle_cr_sin(t, ct.byref(out)):
        raise Undecided(t)
    return out.value


def cr_sin_array(t: np.ndarray) -> np.ndarray:
    """cr_sin over a float64 array."""
    t = np.ascontiguousarray(t, np.float64)
    out = np.empty_like(t)
    if lib().oracle_cr_sin_array(_f64(t), _f64(out), t.size):
        raise Undecided("array")
    return out


def lasm(x: float, y: float, mu: float):
    """Eq. (6), one step of one map: returns (x', y')."""
    a, b = ct.c_double(x), ct.c_double(y)
    if lib().oracle_lasm(ct.byref(a), ct.byref(b), mu):
        raise Undecided((x, y, mu))
    return a.value, b.value


def lasm_bytes(m1, m2, nbytes: int):
    """2DLASM byte generator (Sec. 3) for maps m1, m2 = (x, y, mu).  Returns
    (bytes, (x1', y1'), (x2', y2'))."""
    x1, y1, x2, y2 = (ct.c_double(v) for v in (m1[0], m1[1], m2[0], m2[1]))
    out = np.zeros(nbytes, np.uint8)
    if lib().oracle_lasm_bytes(ct.byref(x1), ct.byref(y1), m1[2], ct.byref(x2), ct.byref(y2),
                               m2[2], nbytes, _u8(out)):
        raise Undecided((m1, m2))
    return out, (x1.value, y1.value), (x2.value, y2.value)


def key_schedule(is_lasm: bool, K, n: int, first_frame: int, T: int):
    """Algorithm 1's key schedule (reading 1): returns (P_m as (n, 4) or (n, 6),
    s_c for frames first_frame .. first_frame+T-1)."""
    K = np.ascontiguousarray(np.asarray(K, np.float64))
    pm = np.zeros(n * (6 if is_lasm else 4), np.float64)
    sc = np.zeros(max(T, 1), np.uint32)
    rc = lib().oracle_key_schedule(int(is_lasm), _f64(K), n, _f64(pm), first_frame,
                                   sc.ctypes.data_as(ct.POINTER(ct.c_uint32)), T)
    if rc == 1:
        raise Undecided("key schedule")
    if rc:
        raise ValueError("degenerate master key")
    return pm.reshape(n, -1), sc[:T]


def band_lo(H: int, n: int, i: int) -> int:
    return lib().oracle_band_lo(H, n, i)


def gtable(H: int, s_c: int) -> np.ndarray:
    g = np.zeros(H, np.int64)
    lib().oracle_gtable(H, s_c, g.ctypes.data_as(ct.POINTER(ct.c_int64)))
    return g


def confuse(frame: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Eq. (1) on one HWC frame (H, W, C) with an explicit shift table g."""
    H, W, C = frame.shape
    frame = np.ascontiguousarray(frame)
    g = np.ascontiguousarray(g, np.int64)
    out = np.zeros_like(frame)
    lib().oracle_confuse(_u8(frame), _u8(out), H, W, C,
                         g.ctypes.data_as(ct.POINTER(ct.c_int64)))
    return out


def unconfuse(frame: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Eq. (2)."""
    H, W, C = frame.shape
    frame = np.ascontiguousarray(frame)
    g = np.ascontiguousarray(g, np.int64)
    out = np.zeros_like(frame)
    lib().oracle_unconfuse(_u8(frame), _u8(out), H, W, C,
                           g.ctypes.data_as(ct.POINTER(ct.c_int64)))
    return out


def diffuse(Y: np.ndarray, n: int, r: int, j: int, ks: np.ndarray) -> np.ndarray:
    """Eq. (3) on every band, round j; ks is the frame's r*F keystream."""
    H, W, C = Y.shape
    Y = np.ascontiguousarray(Y)
    ks = np.ascontiguousarray(ks, np.uint8)
    assert ks.size == r * Y.size
    Z = np.zeros_like(Y)
    lib().oracle_diffuse(_u8(Y), _u8(Z), H, W, C, n, r, j, _u8(ks))
    return Z


def undiffuse(Z: np.ndarray, n: int, r: int, j: int, ks: np.ndarray) -> np.ndarray:
    """Eq. (4) on every band, round j."""
    H, W, C = Z.shape
    Z = np.ascontiguousarray(Z)
    ks = np.ascontiguousarray(ks, np.uint8)
    assert ks.size == r * Z.size
    Y = np.zeros_like(Z)
    lib().oracle_undiffuse(_u8(Z), _u8(Y), H, W, C, n, r, j, _u8(ks))
    return Y


def rounds(H: int, W: int, C: int, n: int, r: int, decrypt: bool, ks: np.ndarray,
           frames: np.ndarray, s_c) -> np.ndarray:
    """The r rounds of T frames with a given keystream (T*r*F bytes, frame
    after frame): Eq. (1) then Eq. (3) per round, or Eq. (4) then Eq. (2) in
    reverse round order (Algorithm 2's round loop)."""
    frames = np.ascontiguousarray(frames, np.uint8).reshape(-1, H, W, C)
    T = frames.shape[0]
    ks = np.ascontiguousarray(np.asarray(ks, np.uint8).reshape(-1))
    assert ks.size == T * r * H * W * C
    s_c = np.ascontiguousarray(np.asarray(s_c, np.uint32).reshape(-1))
    assert s_c.size == T
    out = np.zeros_like(frames)
    if lib().oracle_rounds(H, W, C, n, r, int(decrypt), _u8(ks), _u8(frames), _u8(out),
                           s_c.ctypes.data_as(ct.POINTER(ct.c_uint32)), T):
        raise MemoryError("oracle allocation failed")
    return out


# ---------------------------------------------------------- stateful key ---

class PlcmKey:
    """PLCM key state of one stream: per band (x1, p1, x2, p2); the chain
    states x1, x2 advance with every frame (Algorithm 2: the PRBG is
    initialised once, before the frame loop)."""

    def __init__(self, H, W, C, n, r, pm):
        pm = np.asarray(pm, np.float64).reshape(n, 4)
        self.geom = (H, W, C, n, r)
        self.x1 = np.ascontiguousarray(pm[:, 0].copy())
        self.p1 = np.ascontiguousarray(pm[:, 1].copy())
        self.x2 = np.ascontiguousarray(pm[:, 2].copy())
        self.p2 = np.ascontiguousarray(pm[:, 3].copy())

    def keystream(self, T: int) -> np.ndarray:
        H, W, C, n, r = self.geom
        ks = np.zeros(T * r * H * W * C, np.uint8)
        lib().oracle_plcm_keystream(H, W, C, n, r, _f64(self.x1), _f64(self.p1),
                                    _f64(self.x2), _f64(self.p2), T, _u8(ks))
        return ks.reshape(T, r * H * W * C)

    def _run(self, fn, frames, s_c):
        H, W, C, n, r = self.geom
        frames = np.ascontiguousarray(frames, np.uint8).reshape(-1, H, W, C)
        T = frames.shape[0]
        s_c = np.ascontiguousarray(np.asarray(s_c, np.uint32).reshape(-1))
        assert s_c.size == T
        out = np.zeros_like(frames)
        rc = fn(H, W, C, n, r, _f64(self.x1), _f64(self.p1), _f64(self.x2),
                _f64(self.p2), _u8(frames), _u8(out),
                s_c.ctypes.data_as(ct.POINTER(ct.c_uint32)), T)
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        return out

    def encrypt(self, frames, s_c) -> np.ndarray:
        return self._run(lib().oracle_encrypt, frames, s_c)

    def decrypt(self, frames, s_c) -> np.ndarray:
        return self._run(lib().oracle_decrypt, frames, s_c)


class LasmKey:
    """2DLASM key state of one stream: per band two maps (x, y, mu); the
    states advance with every frame.  `pm` is (n, 6): x0_1, y0_1, mu_1,
    x0_2, y0_2, mu_2."""

    def __init__(self, H, W, C, n, r, pm):
        pm = np.asarray(pm, np.float64).reshape(n, 6)
        self.geom = (H, W, C, n, r)
        self.x1 = np.ascontiguousarray(pm[:, 0].copy())
        self.y1 = np.ascontiguousarray(pm[:, 1].copy())
        self.mu1 = np.ascontiguousarray(pm[:, 2].copy())
        self.x2 = np.ascontiguousarray(pm[:, 3].copy())
        self.y2 = np.ascontiguousarray(pm[:, 4].copy())
        self.mu2 = np.ascontiguousarray(pm[:, 5].copy())

    def state(self) -> np.ndarray:
        """(n, 4): x_1, y_1, x_2, y_2 per band."""
        return np.stack([self.x1, self.y1, self.x2, self.y2], axis=1)

    def keystream(self, T: int) -> np.ndarray:
        H, W, C, n, r = self.geom
        ks = np.zeros(T * r * H * W * C, np.uint8)
        if lib().oracle_lasm_keystream(H, W, C, n, r, _f64(self.x1), _f64(self.y1),
                                       _f64(self.mu1), _f64(self.x2), _f64(self.y2),
                                       _f64(self.mu2), T, _u8(ks)):
            raise Undecided("keystream")
        return ks.reshape(T, r * H * W * C)

    def _rounds(self, decrypt, frames, s_c):
        H, W, C, n, r = self.geom
        frames = np.ascontiguousarray(frames, np.uint8).reshape(-1, H, W, C)
        T = frames.shape[0]
        s_c = np.ascontiguousarray(np.asarray(s_c, np.uint32).reshape(-1))
        assert s_c.size == T
        return rounds(H, W, C, n, r, decrypt, self.keystream(T), frames, s_c)

    def encrypt(self, frames, s_c) -> np.ndarray:
        return self._rounds(False, frames, s_c)

    def decrypt(self, frames, s_c) -> np.ndarray:
        return self._rounds(True, frames, s_c)


def paper_mt_encrypt(H, W, C, n, r, pm, state, frames, s_c) -> np.ndarray:
    """The paper's multithreaded design (paper_mt.c): n threads, one per
    subframe.  `state` is an (n, 2) float64 array of the current x of both
    maps of every band (advanced in place); returns the cipher frames."""
    frames = np.ascontiguousarray(frames, dtype=np.uint8)
    T = frames.shape[0]
    pm = np.ascontiguousarray(np.asarray(pm, np.float64).reshape(n, 4))
    assert state.dtype == np.float64 and state.flags.c_contiguous and state.shape == (n, 2)
    sc = np.ascontiguousarray(np.asarray(s_c, np.uint32).reshape(-1))
    assert sc.size == T
    out = np.empty_like(frames)
    if lib().paper_mt_encrypt(H, W, C, n, r, _f64(pm), _f64(state), _u8(frames), _u8(out),
                              sc.ctypes.data_as(ct.POINTER(ct.c_uint32)), T):
        raise MemoryError("paper_mt_encrypt: buffers or threads")
    return out
