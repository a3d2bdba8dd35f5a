"""Graph replay of a key's per-call work (cv_launch.use_graph = 1): frames
encrypted or decrypted one call at a time from a ring of buffer slots, each
call replaying the graph captured for its slot, must equal the oracle frame
by frame -- with eager work of another key between the replays, for the
plain and the fused round paths (also bands over one LDS tile), the byte
kernels, calls of several internal batches, a 2DLASM key, and after the
launch shape changes (which drops the graphs)."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import (CorrelatedVideo, confusion_seeds, lasm_key, plcm_key,
                                         uniform_frames)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


CASES = [
    ("rgb768-fused", 768, 768, 3, 16, 5, "fused"),
    ("rgb768-plain", 768, 768, 3, 16, 5, "plain"),
    ("rgb48-fused", 48, 48, 3, 8, 5, "fused"),
    # bands of 32 rows of 2048 pixels exceed one LDS tile: decryption by the
    # row-run multi-stream kernel with device-written tables
    ("wide2048-fused", 64, 2048, 3, 2, 5, "fused"),
    ("odd-bytes", 31, 17, 3, 7, 4, "plain"),
]


@pytest.mark.parametrize("decrypt", [False, True])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_ring_of_slots_replays(B, case, decrypt):
    name, H, W, C, n, r, path = case
    T, SLOTS = 8, 3
    print(f"[case] graph ring {name} decrypt={decrypt}", flush=True)
    pm = plcm_key(n, 6100 + H)
    frames = (CorrelatedVideo(H, W, C, 6200 + H).frames(0, T) if H >= 256
              else uniform_frames(H, W, C, T, 6200 + H))
    s_c = confusion_seeds(T, 6300 + H)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.decrypt(frames, s_c) if decrypt else ref.encrypt(frames, s_c)
    F = H * W * C
    dev = torch.device("cuda:0")
    slots_in = [torch.empty(F, dtype=torch.uint8, device=dev) for _ in range(SLOTS)]
    slots_out = [torch.empty(F, dtype=torch.uint8, device=dev) for _ in range(SLOTS)]
    k = B.Key(H, W, C, n, r, pm)
    k.set_path(B.CV_PATH_FUSED if path == "fused" else B.CV_PATH_PLAIN)
    k.set_launch(use_graph=1)
    assert k.get_launch()["use_graph"] == 1
    other = B.Key(48, 48, 3, 8, 5, plcm_key(8, 6400))      # eager work between replays
    o_src = torch.from_numpy(uniform_frames(48, 48, 3, 1, 6401).reshape(-1)).to(dev)
    o_dst = torch.empty_like(o_src)
    for t in range(T):
        i = t % SLOTS
        slots_in[i].copy_(torch.from_numpy(np.ascontiguousarray(frames[t]).reshape(-1)))
        (k.decrypt if decrypt else k.encrypt)(slots_in[i], slots_out[i], s_c[t:t + 1])
        other.encrypt(o_src, o_dst, [t + 1])
        torch.cuda.synchronize()
        got = slots_out[i].cpu().numpy().reshape(want[t].shape)
        assert np.array_equal(got, want[t]), f"frame {t}: {np.count_nonzero(got != want[t])} bytes"
    assert k.graph_counts() == (SLOTS, T - SLOTS)
    k.sync()


def test_batches_per_call_and_shape_change(B):
    """Calls of 5 frames with batch_frames = 2 (graphs of 2 and 1 frames);
    a launch-shape change drops the graphs and later calls capture anew."""
    H, W, C, n, r = 64, 48, 3, 4, 5
    T = 15
    pm = plcm_key(n, 6500)
    frames = uniform_frames(H, W, C, T, 6501)
    s_c = confusion_seeds(T, 6502)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    F = H * W * C
    print("[case] graph batches per call", flush=True)
    src = torch.from_numpy(frames.reshape(-1)).to("cuda:0")
    inb = torch.empty(5 * F, dtype=torch.uint8, device="cuda:0")
    out = torch.empty(5 * F, dtype=torch.uint8, device="cuda:0")
    got = np.empty_like(want)
    k = B.Key(H, W, C, n, r, pm)
    k.set_path(B.CV_PATH_FUSED)
    k.set_launch(batch_frames=2, use_graph=1)
    for c in range(3):
        if c == 2:
            k.set_launch(threads=512)          # drops the graphs
        inb.copy_(src[c * 5 * F:(c + 1) * 5 * F])
        k.encrypt(inb, out, s_c[c * 5:(c + 1) * 5])
        torch.cuda.synchronize()
        got[c * 5:(c + 1) * 5] = out.cpu().numpy().reshape(5, H, W, C)
    assert np.array_equal(got, want)
    # call 0 captures the 2-frame batch at 0 and at 2 and the 1-frame one at
    # 4; call 1 replays all three; call 2 captures them again
    assert k.graph_counts() == (6, 3)


def test_lasm_key_replays(B):
    H, W, C, n, r, T = 48, 48, 3, 4, 5, 4
    pm = lasm_key(n, 6600)
    frames = uniform_frames(H, W, C, T, 6601)
    s_c = confusion_seeds(T, 6602)
    want = oracle.LasmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    print("[case] graph 2DLASM", flush=True)
    F = H * W * C
    buf_in = torch.empty(F, dtype=torch.uint8, device="cuda:0")
    buf_out = torch.empty_like(buf_in)
    k = B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
    k.set_launch(use_graph=1)
    for t in range(T):
        buf_in.copy_(torch.from_numpy(np.ascontiguousarray(frames[t]).reshape(-1)))
        k.encrypt(buf_in, buf_out, s_c[t:t + 1])
        torch.cuda.synchronize()
        assert np.array_equal(buf_out.cpu().numpy().reshape(H, W, C), want[t]), f"frame {t}"
    assert k.graph_counts() == (1, T - 1)
    k.sync()
