"""Keystream lookahead of a key (cv_launch.lookahead = 1): after each
internal batch the next batch's keystream is generated on a private stream
from a copy of the generator states.  Frames encrypted or decrypted one call
at a time must equal the oracle frame by frame, whether a call takes the
lookahead or not: calls arriving after the lookahead finished, calls queued
back to back, calls that change the frame count, a keystream call or a state
set between calls, calls of several internal batches, calls on two streams
in turn, both round paths, and 2DLASM keys (their generator runs on the
private stream the same way)."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, lasm_key, plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda:0")


def _host(t, shape):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("decrypt", [False, True])
def test_lookahead_calls_match_oracle(B, path, decrypt):
    H, W, C, n, r = 96, 128, 3, 8, 5
    print(f"[case] lookahead path={path} decrypt={decrypt}", flush=True)
    pm = plcm_key(n, 7100)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    k = B.Key(H, W, C, n, r, pm)
    k.set_path(B.CV_PATH_FUSED if path == "fused" else B.CV_PATH_PLAIN)
    k.set_launch(lookahead=1, batch_frames=2)
    assert k.get_launch()["lookahead"] == 1
    op = ref.decrypt if decrypt else ref.encrypt
    call = k.decrypt if decrypt else k.encrypt
    # (frames in the call, wait for the device before the call, what happens first)
    plan = [(1, True, None), (1, True, None), (1, False, None), (1, False, None),
            (2, True, None), (2, False, None), (5, True, None), (1, True, "keystream"),
            (1, True, None), (1, True, "set_state"), (1, True, None), (3, False, None)]
    for i, (T, wait, event) in enumerate(plan):
        if event == "keystream":  # the key advances outside the calls: the lookahead is dropped
            ks = torch.empty(r * H * W * C, dtype=torch.uint8, device="cuda:0")
            k.keystream(ks, 1)
            want_ks = ref.keystream(1)
            assert np.array_equal(_host(ks, want_ks.shape), want_ks)
        if event == "set_state":  # state set from outside, to other values
            x, fi = k.get_state()
            xs = np.ascontiguousarray(x * np.array([0.5, 0.25]))
            k.set_state(xs, fi)
            ref.x1 = xs[:, 0].copy()
            ref.x2 = xs[:, 1].copy()
        if wait:
            torch.cuda.synchronize()
        frames = uniform_frames(H, W, C, T, 7200 + i)
        s_c = confusion_seeds(T, 7300 + i)
        want = op(frames, s_c)
        src = _dev(frames)
        dst = torch.empty_like(src)
        call(src, dst, s_c)
        got = _host(dst, want.shape)
        assert np.array_equal(got, want), f"call {i}: {np.count_nonzero(got != want)} bytes differ"
    hits, misses = k.lookahead_counts()
    # batches (of at most 2 frames) that found the lookahead of the batch before:
    # call 1, 2, 3 (T=1 after T=1); call 4's batch of 2 after T=1 misses; call 5 hits;
    # call 6 (5 frames: 2+2+1) hits, hits, misses; call 7 after a keystream call misses;
    # call 8 hits; call 9 after set_state misses; call 10 hits; call 11 (3 = 2+1):
    # misses (T=2 after T=1), misses (T=1 after T=2)
    assert (hits, misses) == (8, 6), (hits, misses)
    x, fi = k.get_state()
    assert np.array_equal(x[:, 0], ref.x1) and np.array_equal(x[:, 1], ref.x2)
    assert fi == sum(p[0] for p in plan) + 1  # the keystream call's frame
    k.close()


def test_lookahead_round_trip_and_off_equal(B):
    """The same frames through keys with the lookahead on and off give the
    same cipher, and decrypting with the lookahead gives the frames back."""
    H, W, C, n, r, T = 64, 80, 3, 4, 5, 6
    pm = plcm_key(n, 7400)
    frames = uniform_frames(H, W, C, T, 7401)
    s_c = confusion_seeds(T, 7402)
    on, off, dec = B.Key(H, W, C, n, r, pm), B.Key(H, W, C, n, r, pm), B.Key(H, W, C, n, r, pm)
    on.set_launch(lookahead=1)
    dec.set_launch(lookahead=1)
    src = _dev(frames)
    a, b_, back = torch.empty_like(src), torch.empty_like(src), torch.empty_like(src)
    F = H * W * C
    for t in range(T):
        sl = slice(t * F, (t + 1) * F)
        on.encrypt(src[sl], a[sl], s_c[t:t + 1])
        off.encrypt(src[sl], b_[sl], s_c[t:t + 1])
    for t in range(T):
        sl = slice(t * F, (t + 1) * F)
        dec.decrypt(a[sl], back[sl], s_c[t:t + 1])
    torch.cuda.synchronize()
    assert torch.equal(a, b_)
    assert torch.equal(back, src)
    assert on.lookahead_counts() == (T - 1, 0)
    for k in (on, off, dec):
        k.close()


def test_lookahead_calls_on_alternating_streams(B):
    """Calls queued without waiting on two streams in turn: each call starts
    after the last one's work, whatever stream it was on, and every frame
    equals the oracle's."""
    H, W, C, n, r, T = 64, 96, 3, 8, 5, 8
    pm = plcm_key(n, 7800)
    frames = uniform_frames(H, W, C, T, 7801)
    s_c = confusion_seeds(T, 7802)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    k = B.Key(H, W, C, n, r, pm)
    k.set_path(B.CV_PATH_FUSED)
    k.set_launch(lookahead=1)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    src = _dev(frames)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    F = H * W * C
    print("[case] lookahead alternating streams", flush=True)
    for t in range(T):
        sl = slice(t * F, (t + 1) * F)
        k.encrypt(src[sl], dst[sl], s_c[t:t + 1], stream=streams[t % 2])
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    assert k.lookahead_counts() == (T - 1, 0)
    k.close()


@pytest.mark.parametrize("decrypt", [False, True])
def test_lookahead_for_2dlasm(B, decrypt):
    """A 2DLASM key: one frame per call, waited for or queued, then a call of
    two frames (a miss) and a state set from outside (a miss); every frame
    equals the oracle's and the key's state follows the oracle's."""
    H, W, C, n, r = 48, 64, 3, 4, 3
    print(f"[case] 2DLASM lookahead decrypt={decrypt}", flush=True)
    pm = lasm_key(n, 7500)
    k = B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
    k.set_path(B.CV_PATH_FUSED)
    k.set_launch(lookahead=1)
    ref = oracle.LasmKey(H, W, C, n, r, pm)
    op = ref.decrypt if decrypt else ref.encrypt
    call = k.decrypt if decrypt else k.encrypt
    plan = [(1, True, None), (1, True, None), (1, False, None), (2, True, None),
            (1, True, "set_state"), (1, True, None)]
    for i, (T, wait, event) in enumerate(plan):
        if event == "set_state":
            x, fi = k.get_state()
            xs = np.ascontiguousarray(np.clip(x * 0.5 + 0.25, 0.0, 1.0))
            k.set_state(xs, fi)
            ref.x1, ref.y1, ref.x2, ref.y2 = (np.ascontiguousarray(xs[:, m]) for m in range(4))
        if wait:
            torch.cuda.synchronize()
        frames = uniform_frames(H, W, C, T, 7600 + i)
        s_c = confusion_seeds(T, 7700 + i)
        want = op(frames, s_c)
        src = _dev(frames)
        dst = torch.empty_like(src)
        call(src, dst, s_c)
        got = _host(dst, want.shape)
        assert np.array_equal(got, want), f"call {i}: {np.count_nonzero(got != want)} bytes differ"
    # hits: calls 1 and 2; misses: call 3 (two frames after one), call 4 (after set_state);
    # call 5 follows the set_state call's lookahead: a hit
    assert k.lookahead_counts() == (3, 2), k.lookahead_counts()
    x, _ = k.get_state()
    assert np.array_equal(x, ref.state())
    k.close()
