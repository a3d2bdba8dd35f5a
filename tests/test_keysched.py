"""The library's key schedule (cv_key_schedule, host code) equals the
oracle's bit for bit, and rejects degenerate and invalid master keys.  No
GPU is used."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd import binding as B
from test_oracle_keysched import PLCM_DEGENERATE


@pytest.mark.parametrize("is_lasm", [False, True])
@pytest.mark.parametrize("n,first", [(1, 0), (3, 57), (16, 0)])
def test_library_matches_oracle(is_lasm, n, first):
    B.load()
    r = np.random.default_rng(n * 7 + first)
    for _ in range(5):
        if is_lasm:
            K = [r.uniform(0.01, 0.99), r.uniform(0.01, 0.99), r.choice([0.375, 0.41, r.uniform(0.44, 0.93), 1.0])]
            m = B.CV_MAP_2DLASM
        else:
            K = [r.uniform(0.01, 0.99), r.uniform(0.01, 0.49), r.uniform(0.01, 0.99), r.uniform(0.01, 0.49)]
            m = B.CV_MAP_PLCM
        want_pm, want_sc = oracle.key_schedule(is_lasm, K, n, first, 120)
        pm, sc = B.key_schedule(K, n, first, 120, map=m)
        assert np.array_equal(pm.view(np.uint64), want_pm.view(np.uint64))
        assert np.array_equal(sc, want_sc)


def test_degenerate_and_invalid_keys():
    B.load()
    for K in PLCM_DEGENERATE:
        with pytest.raises(B.CvError) as e:
            B.key_schedule(K, 1, 0, 1)
        assert e.value.status == B.CV_E_INVAL
    for bad in ([0.0, 0.2, 0.3, 0.2], [0.3, 0.5, 0.3, 0.2], [0.3, 0.2, 0.3]):
        with pytest.raises(B.CvError):
            B.key_schedule(bad, 2, 0, 1)
    with pytest.raises(B.CvError):
        B.key_schedule([0.3, 0.6, 0.39], 2, 0, 1, map=B.CV_MAP_2DLASM)  # mu not admissible
    with pytest.raises(B.CvError):
        B.key_schedule([0.3, 1.0, 0.9], 2, 0, 1, map=B.CV_MAP_2DLASM)  # y0 outside (0,1)
