"""Thin ctypes binding of libchaosvid (include/chaosvid.h).

Argument marshalling only: every step of the cipher runs in the library's
HIP kernels.  PyTorch provides device memory (uint8 CUDA tensors) and the
current HIP stream.  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libchaosvid.so")

CV_OK, CV_E_INVAL, CV_E_NOMEM, CV_E_HIP, CV_E_AGAIN, CV_E_STATE = range(6)
CV_MAP_PLCM = 0
CV_MAP_2DLASM = 1
CV_PATH_PLAIN = 0
CV_PATH_FUSED = 1

# every symbol include/chaosvid.h declares
EXPORTS = (
    "cv_spec_version", "cv_last_error", "cv_keysetup", "cv_key_free", "cv_key_get_state",
    "cv_key_set_state", "cv_key_set_path", "cv_encrypt_frames", "cv_decrypt_frames",
    "cv_keystream_frames", "cv_apply_rounds", "cv_key_get_launch", "cv_key_set_launch",
    "cv_key_set_profiling", "cv_key_get_profile", "cv_batch_create", "cv_batch_free",
    "cv_batch_get_shape", "cv_batch_set_shape", "cv_batch_run", "cv_batch_sync",
    "cv_batch_get_info", "cv_batch_autotune", "cv_batch_set_profiling", "cv_batch_get_profile",
    "cv_server_create", "cv_server_tune", "cv_server_free", "cv_server_drain",
    "cv_server_get_stats", "cv_stream_open", "cv_stream_submit", "cv_stream_poll",
    "cv_stream_close", "cv_cr_sin", "cv_key_schedule", "cv_sin_stage1", "cv_key_sync",
    "cv_key_set_spin_limit", "cv_apply_rounds_noalloc", "cv_key_graph_counts",
    "cv_key_autotune", "cv_key_lookahead_counts",
)


class CvGeom(ct.Structure):
    _fields_ = [("height", ct.c_uint32), ("width", ct.c_uint32), ("channels", ct.c_uint32),
                ("n_sub", ct.c_uint32), ("rounds", ct.c_uint32)]


class CvLaunch(ct.Structure):
    _fields_ = [("batch_frames", ct.c_uint32), ("threads", ct.c_uint32),
                ("tile_rows_enc", ct.c_uint32), ("tile_rows_dec", ct.c_uint32),
                ("prbg_variant", ct.c_uint32), ("round_variant", ct.c_uint32),
                ("tile_rows_pw", ct.c_uint32), ("fused_groups", ct.c_uint32),
                ("use_graph", ct.c_uint32), ("lookahead", ct.c_uint32)]


class CvProfile(ct.Structure):
    _fields_ = [("prbg_ms", ct.c_double), ("prbg_launches", ct.c_uint64),
                ("prbg_steps", ct.c_uint64), ("round_ms", ct.c_double),
                ("round_launches", ct.c_uint64), ("round_frames", ct.c_uint64)]


class CvBatchItem(ct.Structure):
    _fields_ = [("key", ct.c_void_p), ("in_", ct.c_void_p), ("out", ct.c_void_p),
                ("s_c", ct.POINTER(ct.c_uint32)), ("n_frames", ct.c_uint32),
                ("decrypt", ct.c_int32)]


class CvBatchShape(ct.Structure):
    _fields_ = [("threads", ct.c_uint32), ("group_wgs", ct.c_uint32),
                ("max_groups", ct.c_uint32), ("use_graph", ct.c_uint32),
                ("tile_rows_max", ct.c_uint32), ("prefetch", ct.c_uint32)]


class CvBatchInfo(ct.Structure):
    _fields_ = [("ticks", ct.c_uint64), ("graph_captures", ct.c_uint64),
                ("graph_replays", ct.c_uint64), ("last_jobs", ct.c_uint32),
                ("last_groups", ct.c_uint32), ("last_chains", ct.c_uint32),
                ("last_fallback_items", ct.c_uint32), ("tune_cache_hits", ct.c_uint32),
                ("tune_shapes_timed", ct.c_uint32), ("prefetch_hits", ct.c_uint32),
                ("prefetch_misses", ct.c_uint32), ("last_wide_groups", ct.c_uint32)]


class CvServerStats(ct.Structure):
    _fields_ = [("frames_done", ct.c_uint64), ("rounds_ticks", ct.c_uint64),
                ("keystream_launches", ct.c_uint64), ("keystream_frames", ct.c_uint64),
                ("open_streams", ct.c_uint32), ("split_cus", ct.c_uint32),
                ("hbm_used", ct.c_uint64), ("hbm_budget", ct.c_uint64),
                ("keystream_ms", ct.c_double), ("rounds_ms", ct.c_double),
                ("starved_frames", ct.c_uint64)]


class CvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libchaosvid status {status}: {msg}")
        self.status = status


_lib = None


def load() -> ct.CDLL:
    """Load the in-tree libchaosvid.so (built by `python -m
    paper_2302_07411_amd.build` or __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2302_07411_amd.build")
    L = ct.CDLL(LIB_PATH)
    vp, sz, u8p = ct.c_void_p, ct.c_size_t, ct.c_void_p
    L.cv_spec_version.restype = ct.c_int
    L.cv_spec_version.argtypes = []
    L.cv_last_error.restype = ct.c_char_p
    L.cv_last_error.argtypes = []
    L.cv_keysetup.restype = ct.c_int
    L.cv_keysetup.argtypes = [ct.POINTER(CvGeom), ct.c_int, ct.POINTER(ct.c_double), sz, ct.c_int,
                              ct.POINTER(vp)]
    L.cv_key_free.restype = None
    L.cv_key_free.argtypes = [vp]
    L.cv_key_get_state.restype = ct.c_int
    L.cv_key_get_state.argtypes = [vp, ct.POINTER(ct.c_double), sz, ct.POINTER(ct.c_uint64)]
    L.cv_key_set_state.restype = ct.c_int
    L.cv_key_set_state.argtypes = [vp, ct.POINTER(ct.c_double), sz, ct.c_uint64]
    L.cv_key_sync.restype = ct.c_int
    L.cv_key_sync.argtypes = [vp]
    L.cv_key_set_spin_limit.restype = ct.c_int
    L.cv_key_set_spin_limit.argtypes = [vp, ct.c_uint32]
    L.cv_key_set_path.restype = ct.c_int
    L.cv_key_set_path.argtypes = [vp, ct.c_int]
    L.cv_key_graph_counts.restype = ct.c_int
    L.cv_key_autotune.restype = ct.c_int
    L.cv_key_autotune.argtypes = [vp, ct.c_int, ct.c_uint32, vp, ct.POINTER(CvLaunch),
                                  ct.POINTER(ct.c_int)]
    L.cv_key_graph_counts.argtypes = [vp, ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_uint64)]
    L.cv_key_lookahead_counts.restype = ct.c_int
    L.cv_key_lookahead_counts.argtypes = [vp, ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_uint64)]
    for name in ("cv_encrypt_frames", "cv_decrypt_frames"):
        f = getattr(L, name)
        f.restype = ct.c_int
        f.argtypes = [vp, u8p, u8p, ct.POINTER(ct.c_uint32), sz, vp]
    L.cv_key_get_launch.restype = ct.c_int
    L.cv_key_get_launch.argtypes = [vp, ct.POINTER(CvLaunch)]
    L.cv_key_set_launch.restype = ct.c_int
    L.cv_key_set_launch.argtypes = [vp, ct.POINTER(CvLaunch)]
    L.cv_key_set_profiling.restype = ct.c_int
    L.cv_key_set_profiling.argtypes = [vp, ct.c_int]
    L.cv_key_get_profile.restype = ct.c_int
    L.cv_key_get_profile.argtypes = [vp, ct.POINTER(CvProfile)]
    L.cv_keystream_frames.restype = ct.c_int
    L.cv_keystream_frames.argtypes = [vp, u8p, sz, vp]
    L.cv_apply_rounds.restype = ct.c_int
    L.cv_apply_rounds.argtypes = [vp, ct.c_int, u8p, u8p, u8p, ct.POINTER(ct.c_uint32), sz, vp]
    L.cv_apply_rounds_noalloc.restype = ct.c_int
    L.cv_apply_rounds_noalloc.argtypes = [vp, ct.c_int, u8p, u8p, u8p, ct.POINTER(ct.c_uint32), sz,
                                          vp]
    L.cv_batch_create.restype = ct.c_int
    L.cv_batch_create.argtypes = [ct.c_int, ct.POINTER(vp)]
    L.cv_batch_free.restype = None
    L.cv_batch_free.argtypes = [vp]
    L.cv_batch_get_shape.restype = ct.c_int
    L.cv_batch_get_shape.argtypes = [vp, ct.POINTER(CvBatchShape)]
    L.cv_batch_set_shape.restype = ct.c_int
    L.cv_batch_set_shape.argtypes = [vp, ct.POINTER(CvBatchShape)]
    L.cv_batch_run.restype = ct.c_int
    L.cv_batch_run.argtypes = [vp, ct.POINTER(CvBatchItem), sz, vp]
    L.cv_batch_sync.restype = ct.c_int
    L.cv_batch_sync.argtypes = [vp]
    L.cv_batch_get_info.restype = ct.c_int
    L.cv_batch_get_info.argtypes = [vp, ct.POINTER(CvBatchInfo)]
    L.cv_batch_autotune.restype = ct.c_int
    L.cv_batch_autotune.argtypes = [vp, ct.POINTER(CvBatchItem), sz, vp, ct.POINTER(CvBatchShape)]
    L.cv_batch_set_profiling.restype = ct.c_int
    L.cv_batch_set_profiling.argtypes = [vp, ct.c_int]
    L.cv_batch_get_profile.restype = ct.c_int
    L.cv_batch_get_profile.argtypes = [vp, ct.POINTER(CvProfile)]
    L.cv_sin_stage1.restype = ct.c_int
    L.cv_sin_stage1.argtypes = [ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                                ct.POINTER(ct.c_double), ct.POINTER(ct.c_int), sz]
    L.cv_key_schedule.restype = ct.c_int
    L.cv_key_schedule.argtypes = [ct.c_int, ct.POINTER(ct.c_double), sz, ct.c_uint32,
                                  ct.POINTER(ct.c_double), sz, ct.c_uint64,
                                  ct.POINTER(ct.c_uint32), sz]
    L.cv_cr_sin.restype = ct.c_int
    L.cv_cr_sin.argtypes = [vp, vp, sz, ct.c_int, vp, vp]
    L.cv_server_create.restype = ct.c_int
    L.cv_server_create.argtypes = [ct.c_int, sz, ct.POINTER(vp)]
    L.cv_server_tune.restype = ct.c_int
    L.cv_server_tune.argtypes = [vp, ct.c_uint32, ct.c_uint32, ct.c_int]
    L.cv_server_free.restype = None
    L.cv_server_free.argtypes = [vp]
    L.cv_server_drain.restype = ct.c_int
    L.cv_server_drain.argtypes = [vp]
    L.cv_server_get_stats.restype = ct.c_int
    L.cv_server_get_stats.argtypes = [vp, ct.POINTER(CvServerStats)]
    L.cv_stream_open.restype = ct.c_int
    L.cv_stream_open.argtypes = [vp, ct.POINTER(CvGeom), ct.c_int, ct.POINTER(ct.c_double), sz,
                                 ct.c_int, ct.POINTER(vp)]
    L.cv_stream_submit.restype = ct.c_int
    L.cv_stream_submit.argtypes = [vp, u8p, u8p, ct.c_uint32, ct.POINTER(ct.c_uint64)]
    L.cv_stream_poll.restype = ct.c_int
    L.cv_stream_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double)]
    L.cv_stream_close.restype = ct.c_int
    L.cv_stream_close.argtypes = [vp]
    _lib = L
    return L


def _check(status: int):
    if status != CV_OK:
        raise CvError(status, load().cv_last_error().decode())


def _ptr(t) -> int:
    """Device address of a contiguous uint8 CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError("expected a torch.uint8 tensor on a HIP device")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _seeds(s_c, n: int):
    arr = np.ascontiguousarray(np.asarray(s_c, dtype=np.uint32).reshape(-1))
    if arr.size != n:
        raise ValueError(f"need {n} confusion seeds, got {arr.size}")
    return arr, arr.ctypes.data_as(ct.POINTER(ct.c_uint32))


class Key:
    """One stream's key: per-band chaotic generators on the device
    (cv_keysetup).  `pm` is an (n, 4) array of (x0_1, p_1, x0_2, p_2) for
    PLCM or an (n, 6) array of (x0_1, y0_1, mu_1, x0_2, y0_2, mu_2) for
    2DLASM."""

    def __init__(self, H, W, C, n, r, pm, device: int = 0, map: int = CV_MAP_PLCM):
        L = load()
        self.geom = (H, W, C, n, r)
        self.map = map
        self.frame_bytes = H * W * C
        pm = np.ascontiguousarray(np.asarray(pm, np.float64).reshape(-1))
        g = CvGeom(H, W, C, n, r)
        h = ct.c_void_p()
        _check(L.cv_keysetup(ct.byref(g), map, pm.ctypes.data_as(ct.POINTER(ct.c_double)),
                             pm.size, device, ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().cv_key_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _nframes(self, t) -> int:
        if t.numel() % self.frame_bytes:
            raise ValueError("tensor size is not a whole number of frames")
        return t.numel() // self.frame_bytes

    def encrypt(self, src, dst, s_c, stream=None):
        n = self._nframes(src)
        if dst.numel() != src.numel():
            raise ValueError("dst size differs from src")
        arr, p = _seeds(s_c, n)
        _check(load().cv_encrypt_frames(self._h, _ptr(src), _ptr(dst), p, n, _stream(stream)))

    def decrypt(self, src, dst, s_c, stream=None):
        n = self._nframes(src)
        if dst.numel() != src.numel():
            raise ValueError("dst size differs from src")
        arr, p = _seeds(s_c, n)
        _check(load().cv_decrypt_frames(self._h, _ptr(src), _ptr(dst), p, n, _stream(stream)))

    def keystream(self, dst, n_frames: int, stream=None):
        r = self.geom[4]
        if dst.numel() != n_frames * r * self.frame_bytes:
            raise ValueError("keystream buffer must hold n_frames*r*H*W*C bytes")
        _check(load().cv_keystream_frames(self._h, _ptr(dst), n_frames, _stream(stream)))

    def apply_rounds(self, decrypt: bool, src, dst, ks, s_c, stream=None):
        n = self._nframes(src)
        r = self.geom[4]
        if ks.numel() != n * r * self.frame_bytes or dst.numel() != src.numel():
            raise ValueError("buffer sizes do not match")
        arr, p = _seeds(s_c, n)
        _check(load().cv_apply_rounds(self._h, int(bool(decrypt)), _ptr(src), _ptr(dst), _ptr(ks),
                                      p, n, _stream(stream)))

    def apply_rounds_noalloc(self, decrypt: bool, src, dst, ks, s_c, stream=None):
        """cv_apply_rounds_noalloc: as apply_rounds, with the library's static
        device scratch instead of allocated workspace (synchronous)."""
        n = self._nframes(src)
        r = self.geom[4]
        if ks.numel() != n * r * self.frame_bytes or dst.numel() != src.numel():
            raise ValueError("buffer sizes do not match")
        arr, p = _seeds(s_c, n)
        _check(load().cv_apply_rounds_noalloc(self._h, int(bool(decrypt)), _ptr(src), _ptr(dst),
                                              _ptr(ks), p, n, _stream(stream)))

    def get_state(self):
        """(state, frame_index): state is (n, 2) {x_1, x_2} for PLCM, (n, 4)
        {x_1, y_1, x_2, y_2} for 2DLASM."""
        n = self.geom[3]
        per = 2 if self.map == CV_MAP_PLCM else 4
        x = np.zeros(per * n, np.float64)
        fi = ct.c_uint64()
        _check(load().cv_key_get_state(self._h, x.ctypes.data_as(ct.POINTER(ct.c_double)), x.size,
                                       ct.byref(fi)))
        return x.reshape(n, per), fi.value

    def set_state(self, x, frame_index: int):
        x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1))
        _check(load().cv_key_set_state(self._h, x.ctypes.data_as(ct.POINTER(ct.c_double)), x.size,
                                       frame_index))

    def sync(self):
        """cv_key_sync: wait for the key's work; raises CvError on a device error."""
        _check(load().cv_key_sync(self._h))

    def set_spin_limit(self, polls: int):
        """Testing hook (cv_key_set_spin_limit)."""
        _check(load().cv_key_set_spin_limit(self._h, polls))

    def autotune(self, decrypt: bool, n_frames: int, stream=None):
        """cv_key_autotune: (launch shape dict, taken from the cache?)."""
        l, c = CvLaunch(), ct.c_int()
        _check(load().cv_key_autotune(self._h, int(bool(decrypt)), n_frames, _stream(stream),
                                      ct.byref(l), ct.byref(c)))
        return {f: getattr(l, f) for f, _ in CvLaunch._fields_}, bool(c.value)

    def graph_counts(self):
        """(captures, replays) of the key's graphs (cv_launch.use_graph)."""
        c, r = ct.c_uint64(), ct.c_uint64()
        _check(load().cv_key_graph_counts(self._h, ct.byref(c), ct.byref(r)))
        return c.value, r.value

    def lookahead_counts(self):
        """(hits, misses) of the key's keystream lookahead (cv_launch.lookahead)."""
        h, m = ct.c_uint64(), ct.c_uint64()
        _check(load().cv_key_lookahead_counts(self._h, ct.byref(h), ct.byref(m)))
        return h.value, m.value

    def set_path(self, path: int):
        _check(load().cv_key_set_path(self._h, path))

    def get_launch(self) -> dict:
        l = CvLaunch()
        _check(load().cv_key_get_launch(self._h, ct.byref(l)))
        return {f: getattr(l, f) for f, _ in CvLaunch._fields_}

    def set_launch(self, **kw):
        cur = self.get_launch()
        cur.update(kw)
        l = CvLaunch(**cur)
        _check(load().cv_key_set_launch(self._h, ct.byref(l)))

    def set_profiling(self, on: bool):
        _check(load().cv_key_set_profiling(self._h, int(bool(on))))

    def get_profile(self) -> dict:
        p = CvProfile()
        _check(load().cv_key_get_profile(self._h, ct.byref(p)))
        return {f: getattr(p, f) for f, _ in CvProfile._fields_}


class Batch:
    """Many streams per tick (cv_batch_*).  An item is a tuple
    (key, src, dst, s_c) or (key, src, dst, s_c, decrypt)."""

    def __init__(self, device: int = 0):
        h = ct.c_void_p()
        _check(load().cv_batch_create(device, ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().cv_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _items(items):
        arr = (CvBatchItem * max(1, len(items)))()
        keep = []
        for i, it in enumerate(items):
            key, src, dst, s_c = it[:4]
            dec = int(bool(it[4])) if len(it) > 4 else 0
            n = key._nframes(src)
            if dst.numel() != src.numel():
                raise ValueError("dst size differs from src")
            seeds, p = _seeds(s_c, n)
            keep.append(seeds)
            arr[i] = CvBatchItem(key._h.value, _ptr(src) if n else None, _ptr(dst) if n else None,
                                 p, n, dec)
        return arr, keep

    def run(self, items, stream=None):
        arr, keep = self._items(items)
        _check(load().cv_batch_run(self._h, arr, len(items), _stream(stream)))

    def sync(self):
        _check(load().cv_batch_sync(self._h))

    def autotune(self, items, stream=None) -> dict:
        arr, keep = self._items(items)
        best = CvBatchShape()
        _check(load().cv_batch_autotune(self._h, arr, len(items), _stream(stream), ct.byref(best)))
        return {f: getattr(best, f) for f, _ in CvBatchShape._fields_}

    def get_shape(self) -> dict:
        s = CvBatchShape()
        _check(load().cv_batch_get_shape(self._h, ct.byref(s)))
        return {f: getattr(s, f) for f, _ in CvBatchShape._fields_}

    def set_shape(self, **kw):
        cur = self.get_shape()
        cur.update(kw)
        _check(load().cv_batch_set_shape(self._h, ct.byref(CvBatchShape(**cur))))

    def info(self) -> dict:
        i = CvBatchInfo()
        _check(load().cv_batch_get_info(self._h, ct.byref(i)))
        return {f: getattr(i, f) for f, _ in CvBatchInfo._fields_}

    def set_profiling(self, on: bool):
        _check(load().cv_batch_set_profiling(self._h, int(bool(on))))

    def get_profile(self) -> dict:
        p = CvProfile()
        _check(load().cv_batch_get_profile(self._h, ct.byref(p)))
        return {f: getattr(p, f) for f, _ in CvProfile._fields_}


class Server:
    """Serving loop (cv_server_*): live streams whose frames are batched into
    rounds ticks by a worker thread, keystream generated ahead."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, ring_frames: int = None,
                 queue_frames: int = None, split_cus: int = 1):
        h = ct.c_void_p()
        _check(load().cv_server_create(device, hbm_budget, ct.byref(h)))
        self._h = h
        self._streams = []
        _check(load().cv_server_tune(self._h, ring_frames or 3, queue_frames or 8,
                                     int(split_cus)))

    def open(self, H, W, C, n, r, pm, decrypt: bool = False,
             map: int = CV_MAP_PLCM) -> "ServerStream":
        pm = np.ascontiguousarray(np.asarray(pm, np.float64).reshape(-1))
        g = CvGeom(H, W, C, n, r)
        h = ct.c_void_p()
        _check(load().cv_stream_open(self._h, ct.byref(g), map,
                                     pm.ctypes.data_as(ct.POINTER(ct.c_double)), pm.size,
                                     int(bool(decrypt)), ct.byref(h)))
        st = ServerStream(self, h, H * W * C)
        self._streams.append(st)
        return st

    def drain(self):
        _check(load().cv_server_drain(self._h))

    def stats(self) -> dict:
        st = CvServerStats()
        _check(load().cv_server_get_stats(self._h, ct.byref(st)))
        return {f: getattr(st, f) for f, _ in CvServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().cv_server_free(self._h)
            self._h = None
            for st in self._streams:
                st._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerStream:
    def __init__(self, server, h, frame_bytes):
        self.server, self._h, self.frame_bytes = server, h, frame_bytes

    def submit(self, frame, out, s_c: int) -> int:
        """Queue one frame; returns its ticket.  Raises CvError with status
        CV_E_AGAIN when the stream's queue is full."""
        if frame.numel() != self.frame_bytes or out.numel() != self.frame_bytes:
            raise ValueError("frame and out must hold one frame")
        t = ct.c_uint64()
        _check(load().cv_stream_submit(self._h, _ptr(frame), _ptr(out), int(s_c), ct.byref(t)))
        return t.value

    def try_submit(self, frame, out, s_c: int):
        """As submit, but returns None instead of raising when the queue is full."""
        t = ct.c_uint64()
        st = load().cv_stream_submit(self._h, _ptr(frame), _ptr(out), int(s_c), ct.byref(t))
        if st == CV_E_AGAIN:
            return None
        _check(st)
        return t.value

    def poll(self, ticket: int):
        """(done, latency_ms) of a submitted frame."""
        d, lat = ct.c_int(), ct.c_double()
        _check(load().cv_stream_poll(self._h, ticket, ct.byref(d), ct.byref(lat)))
        return bool(d.value), lat.value

    def close(self):
        if self._h is not None:
            _check(load().cv_stream_close(self._h))
            self._h = None
            try:
                self.server._streams.remove(self)
            except ValueError:
                pass


def cr_sin(t, out, force_exact: bool = False, stream=None) -> bool:
    """RN(sin(t)) on the device for a float64 CUDA tensor t with values in
    [0, RN(pi)] into `out`; returns True if every value was rounded with
    certainty (cv_cr_sin)."""
    import torch
    for x in (t, out):
        if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_cuda \
                or not x.is_contiguous():
            raise TypeError("expected contiguous float64 tensors on a HIP device")
    if out.numel() != t.numel():
        raise ValueError("out size differs from t")
    flag = torch.zeros(1, dtype=torch.int32, device=t.device)
    _check(load().cv_cr_sin(t.data_ptr(), out.data_ptr(), t.numel(), int(bool(force_exact)),
                            flag.data_ptr(), _stream(stream)))
    return int(flag.item()) == 0


def key_schedule(K, n_sub: int, first_frame: int = 0, n_frames: int = 0,
                 map: int = CV_MAP_PLCM):
    """Algorithm 1's key schedule (cv_key_schedule): the subframe parameters
    P_m ((n_sub, 4) for PLCM, (n_sub, 6) for 2DLASM) and the confusion seeds
    of frames first_frame .. first_frame + n_frames - 1, from the key K."""
    K = np.ascontiguousarray(np.asarray(K, np.float64).reshape(-1))
    per = 4 if map == CV_MAP_PLCM else 6
    pm = np.zeros(per * n_sub, np.float64)
    sc = np.zeros(max(1, n_frames), np.uint32)
    _check(load().cv_key_schedule(map, K.ctypes.data_as(ct.POINTER(ct.c_double)), K.size, n_sub,
                                  pm.ctypes.data_as(ct.POINTER(ct.c_double)), pm.size,
                                  first_frame, sc.ctypes.data_as(ct.POINTER(ct.c_uint32)),
                                  n_frames))
    return pm.reshape(n_sub, per), sc[:n_frames]


def sin_stage1(t):
    """cv_sin_stage1 (host): (hi, lo, decided) of the sine's first stage."""
    t = np.ascontiguousarray(np.asarray(t, np.float64).reshape(-1))
    hi, lo = np.empty_like(t), np.empty_like(t)
    dec = np.empty(t.size, np.int32)
    dp = ct.POINTER(ct.c_double)
    _check(load().cv_sin_stage1(t.ctypes.data_as(dp), hi.ctypes.data_as(dp), lo.ctypes.data_as(dp),
                                dec.ctypes.data_as(ct.POINTER(ct.c_int)), t.size))
    return hi, lo, dec.astype(bool)
