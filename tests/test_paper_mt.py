"""The paper's multithreaded CPU design (oracle/paper_mt.c: one thread per
subframe, confusion and diffusion separated by barriers) gives the
single-threaded oracle's bytes and generator state, frame after frame."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, plcm_key, uniform_frames


@pytest.mark.parametrize("H,W,C,n,r,T", [
    (48, 48, 3, 8, 5, 3),
    (50, 44, 3, 6, 5, 2),     # n does not divide H
    (33, 16, 4, 4, 3, 2),
    (20, 36, 1, 1, 5, 2),     # one band: the seed is its own last byte
    (12, 16, 3, 12, 2, 2),    # one row per band
    (96, 128, 3, 16, 1, 2),   # one round
])
def test_matches_oracle(H, W, C, n, r, T):
    pm = plcm_key(n, 40 + H + n)
    frames = uniform_frames(H, W, C, T, 41 + W)
    s_c = confusion_seeds(T, 42 + C)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.encrypt(frames, s_c)
    state = np.ascontiguousarray(pm[:, [0, 2]])
    got = oracle.paper_mt_encrypt(H, W, C, n, r, pm, state, frames, s_c)
    assert np.array_equal(got, want)
    assert np.array_equal(state[:, 0], ref.x1) and np.array_equal(state[:, 1], ref.x2)
    # the state carries over: the next frames continue the same video
    more = uniform_frames(H, W, C, 2, 43 + W)
    s2 = confusion_seeds(2, 44 + C)
    assert np.array_equal(oracle.paper_mt_encrypt(H, W, C, n, r, pm, state, more, s2),
                          ref.encrypt(more, s2))
