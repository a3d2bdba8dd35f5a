"""The largest frame a key accepts: H*W*C at most (2^32 - 1)/8 bytes, here
10922x16384x3 (536,838,144 bytes; one row more is refused, see test_abi).
With 16 subframes every band is 682 or 683 rows of 49,152 bytes, 28 million
chain steps per band and frame, and the row-run rounds take bands of
hundreds of two-row LDS tiles chained by their carries (Sec. 2: the band
split of Algorithm 2, Eq. (1) and Eq. (3)).  One frame through the fused and
the plain per-round paths equals the oracle byte for byte, and decrypting
it gives the frame back."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H, W, C, N, R = 10922, 16384, 3, 16, 5
S_C = 31337


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def test_largest_accepted_frame(B):
    assert H * W * C <= (2**32 - 1) // 8 < (H + 1) * W * C
    pm = plcm_key(N, 8100)
    frame = uniform_frames(H, W, C, 1, 8101)
    print("[case] largest frame: oracle", flush=True)
    want = oracle.PlcmKey(H, W, C, N, R, pm).encrypt(frame, [S_C]).reshape(-1)
    src = torch.from_numpy(frame.reshape(-1)).to("cuda:0")
    cipher = torch.empty_like(src)
    back = torch.empty_like(src)
    for path in (B.CV_PATH_FUSED, B.CV_PATH_PLAIN):
        print(f"[case] largest frame: path {path}", flush=True)
        enc = B.Key(H, W, C, N, R, pm)
        enc.set_path(path)
        enc.encrypt(src, cipher, [S_C])
        torch.cuda.synchronize()
        got = cipher.cpu().numpy()
        assert np.array_equal(got, want), f"path {path}: {np.count_nonzero(got != want)} bytes differ"
        dec = B.Key(H, W, C, N, R, pm)
        dec.set_path(path)
        dec.decrypt(cipher, back, [S_C])
        torch.cuda.synchronize()
        assert torch.equal(back, src), f"path {path}: round trip differs"
        enc.close()
        dec.close()
