"""Calls on one key queued without waiting on two HIP streams in turn: the
key's generator state and workspace are shared, so each call must start
after the key's last call on the other stream.  Every frame equals the
oracle's, on both round paths, with and without graph replay, for
encryption, decryption, and a keystream call followed by the rounds on the
other stream, and decryption calls that grow the key's workspace; and a
multi-stream tick waits for its keys' calls on another stream."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H, W, C, N, R, T = 96, 128, 3, 8, 5, 8
F = H * W * C


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda:0")


@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("decrypt", [False, True])
@pytest.mark.parametrize("path", ["fused", "plain"])
def test_calls_alternate_streams(B, path, decrypt, use_graph):
    print(f"[case] alternating streams path={path} decrypt={decrypt} graph={use_graph}", flush=True)
    pm = plcm_key(N, 8800)
    frames = uniform_frames(H, W, C, T, 8801)
    s_c = confusion_seeds(T, 8802)
    ref = oracle.PlcmKey(H, W, C, N, R, pm)
    want = ref.decrypt(frames, s_c) if decrypt else ref.encrypt(frames, s_c)
    k = B.Key(H, W, C, N, R, pm)
    k.set_path(B.CV_PATH_FUSED if path == "fused" else B.CV_PATH_PLAIN)
    k.set_launch(use_graph=use_graph)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    src = _dev(frames)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    call = k.decrypt if decrypt else k.encrypt
    for t in range(T):
        sl = slice(t * F, (t + 1) * F)
        call(src[sl], dst[sl], s_c[t:t + 1], stream=streams[t % 2])
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    k.close()


def test_keystream_then_rounds_on_the_other_stream(B):
    pm = plcm_key(N, 8900)
    frames = uniform_frames(H, W, C, T, 8901)
    s_c = confusion_seeds(T, 8902)
    want = oracle.PlcmKey(H, W, C, N, R, pm).encrypt(frames, s_c)
    k = B.Key(H, W, C, N, R, pm)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    src = _dev(frames)
    dst = torch.empty_like(src)
    ks = torch.empty(R * F, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    print("[case] keystream on one stream, rounds on the other", flush=True)
    for t in range(T):
        sl = slice(t * F, (t + 1) * F)
        k.keystream(ks, 1, stream=a)
        # the rounds wait for the key's keystream call; the next keystream
        # call waits for these rounds, which read the same buffer
        k.apply_rounds(False, src[sl], dst[sl], ks, s_c[t:t + 1], stream=b)
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    k.close()


def test_batch_tick_waits_for_the_keys_calls(B):
    pm = plcm_key(N, 9000)
    frames = uniform_frames(H, W, C, 2, 9001)
    s_c = confusion_seeds(2, 9002)
    want = oracle.PlcmKey(H, W, C, N, R, pm).encrypt(frames, s_c)
    k = B.Key(H, W, C, N, R, pm)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    src = _dev(frames)
    dst = torch.empty_like(src)
    bt = B.Batch()
    torch.cuda.synchronize()
    print("[case] direct call on one stream, batch tick on the other", flush=True)
    k.encrypt(src[:F], dst[:F], s_c[:1], stream=a)
    bt.run([(k, src[F:], dst[F:], s_c[1:])], stream=b)
    bt.sync()
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    bt.close()
    k.close()


def test_growing_calls_of_wide_decryption_on_two_streams(B):
    """Bands of 2048-pixel rows over one LDS tile: decryption by the row-run
    multi-stream kernel, whose tables grow with the frames of a call; calls
    of 1, then 4, then 2 frames on two streams in turn."""
    h, w, c, n, r = 64, 2048, 3, 2, 5
    f = h * w * c
    pm = plcm_key(n, 9100)
    counts = [1, 4, 2]
    total = sum(counts)
    frames = uniform_frames(h, w, c, total, 9101)
    s_c = confusion_seeds(total, 9102)
    want = oracle.PlcmKey(h, w, c, n, r, pm).decrypt(frames, s_c)
    k = B.Key(h, w, c, n, r, pm)
    k.set_path(B.CV_PATH_FUSED)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    src = _dev(frames)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    print("[case] wide decryption, growing calls on two streams", flush=True)
    t0 = 0
    for i, cnt in enumerate(counts):
        sl = slice(t0 * f, (t0 + cnt) * f)
        k.decrypt(src[sl], dst[sl], s_c[t0:t0 + cnt], stream=streams[i % 2])
        t0 += cnt
    k.sync()
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    k.close()
