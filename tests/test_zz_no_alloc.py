"""cv_apply_rounds_noalloc (the allocation-free variant of cv_apply_rounds,
for callers that cannot allocate device memory) against cv_apply_rounds on
the same keystream and frames, bit for bit: two calls in a row, the second
with fewer frames, for the fused kernels (row-run encryption, pixel-word
decryption) and the byte kernels, with chunks of frames that fill the static
scratch; its size limit, its barrier error report, and that a call on a key
with no workspace allocates no device memory."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _case(B, geom, T, seed, decrypt):
    """Keystream of T frames from one key; rounds by cv_apply_rounds on a
    second key and by cv_apply_rounds_noalloc on a third (fresh) key."""
    H, W, C, n, r = geom
    pm = plcm_key(n, seed)
    F = H * W * C
    frames = uniform_frames(H, W, C, T, seed + 1)
    s_c = confusion_seeds(T, seed + 2)
    dev = torch.device("cuda:0")
    gen = B.Key(H, W, C, n, r, pm)
    ks = torch.empty(T * r * F, dtype=torch.uint8, device=dev)
    gen.keystream(ks, T)
    src = torch.from_numpy(frames.reshape(-1)).to(dev)
    want = torch.empty_like(src)
    got = torch.full_like(src, 0x5A)
    ref = B.Key(H, W, C, n, r, pm)
    ref.set_path(B.CV_PATH_FUSED)
    ref.apply_rounds(decrypt, src, want, ks, s_c)
    torch.cuda.synchronize()
    na = B.Key(H, W, C, n, r, pm)
    na.apply_rounds_noalloc(decrypt, src, got, ks, s_c)
    torch.cuda.synchronize()
    return frames, s_c, ks, want, got, na


GEOMS = [
    (768, 768, 3, 16, 5),   # fused: row-run encryption, pixel-word decryption
    (64, 48, 3, 4, 5),      # fused, small frame
    (40, 36, 1, 3, 5),      # byte kernels (one channel)
    (30, 20, 3, 4, 3),      # byte kernels (W % 16 != 0)
]


@pytest.mark.parametrize("decrypt", [False, True])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "x".join(map(str, g)))
def test_two_calls_second_smaller(B, geom, decrypt):
    """The same keys for both calls: 5 frames, then the next 2."""
    print(f"[case] noalloc two calls geom={geom} decrypt={decrypt}", flush=True)
    H, W, C, n, r = geom
    F = H * W * C
    pm = plcm_key(n, 300 + int(decrypt))
    gen, ref, na = (B.Key(H, W, C, n, r, pm) for _ in range(3))
    ref.set_path(B.CV_PATH_FUSED)
    dev = torch.device("cuda:0")
    for i, T in enumerate((5, 2)):
        frames = uniform_frames(H, W, C, T, 310 + i)
        s_c = confusion_seeds(T, 320 + i)
        ks = torch.empty(T * r * F, dtype=torch.uint8, device=dev)
        gen.keystream(ks, T)
        src = torch.from_numpy(frames.reshape(-1)).to(dev)
        want = torch.empty_like(src)
        got = torch.full_like(src, 0x5A)
        ref.apply_rounds(decrypt, src, want, ks, s_c)
        na.apply_rounds_noalloc(decrypt, src, got, ks, s_c)
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"call {i} ({T} frames) differs from cv_apply_rounds"


def test_small_case_equals_the_oracle(B):
    print("[case] noalloc vs oracle 64x48x3 n=4", flush=True)
    H, W, C, n, r = geom = (64, 48, 3, 4, 5)
    frames, s_c, ks, want, got, _ = _case(B, geom, 3, 400, False)
    ks_host = ks.cpu().numpy()
    exp = oracle.rounds(H, W, C, n, r, False, ks_host, frames, s_c)
    assert np.array_equal(got.cpu().numpy().reshape(frames.shape), exp)


@pytest.mark.parametrize("geom,T", [
    ((4096, 16, 3, 8, 5), 70),     # fused: 64 shift tables per chunk -> 2 chunks
    ((2000, 2000, 1, 8, 5), 17),   # byte kernels: 16 frames per chunk -> 2 chunks
], ids=["fused_chunks", "byte_chunks"])
def test_chunks_of_frames(B, geom, T):
    print(f"[case] noalloc chunks geom={geom} T={T}", flush=True)
    for decrypt in (False, True):
        frames, s_c, ks, want, got, _ = _case(B, geom, T, 500 + int(decrypt), decrypt)
        assert torch.equal(got, want), f"decrypt={decrypt}"


def test_frame_too_large_is_rejected(B):
    # 64 MiB frames: neither two pixel-word frames (fused) nor one frame
    # (byte kernels) fits beside the scratch header
    print("[case] noalloc 4096x4096x4 rejected", flush=True)
    H, W, C, n, r = 4096, 4096, 4, 16, 5
    k = B.Key(H, W, C, n, r, plcm_key(n, 600))
    F = H * W * C
    src = torch.zeros(F, dtype=torch.uint8, device="cuda:0")
    out = torch.empty_like(src)
    ks = torch.empty(r * F, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(B.CvError) as e:
        k.apply_rounds_noalloc(False, src, out, ks, [7])
    assert e.value.status == B.CV_E_INVAL and "allocation-free scratch (64 MiB)" in str(e.value)


def test_barrier_give_up_is_reported_and_the_next_call_is_clean(B):
    print("[case] noalloc barrier give-up", flush=True)
    geom = (48, 48, 3, 8, 5)
    frames, s_c, ks, want, got, na = _case(B, geom, 4, 700, False)
    assert torch.equal(got, want)
    src = torch.from_numpy(frames.reshape(-1)).to("cuda:0")
    na.set_spin_limit(0)
    with pytest.raises(B.CvError) as e:
        na.apply_rounds_noalloc(False, src, got, ks, s_c)
    assert e.value.status == B.CV_E_HIP and "group barrier" in str(e.value)
    na.set_spin_limit(1 << 21)
    got.fill_(0)
    na.apply_rounds_noalloc(False, src, got, ks, s_c)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_no_device_memory_is_allocated(B):
    print("[case] noalloc allocates nothing", flush=True)
    H, W, C, n, r = geom = (768, 768, 3, 16, 5)
    frames, s_c, ks, want, got, _ = _case(B, geom, 4, 800, False)   # warm: kernels loaded
    src = torch.from_numpy(frames.reshape(-1)).to("cuda:0")
    fresh = B.Key(H, W, C, n, r, plcm_key(n, 800))                  # no workspace yet
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    fresh.apply_rounds_noalloc(False, src, got, ks, s_c)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert torch.equal(got, want)
    # a key's own workspace at this size is hundreds of MB
    assert free0 - free1 < (1 << 20), f"device memory fell by {free0 - free1} bytes"
