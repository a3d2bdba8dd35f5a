"""GPU parity of the serving loop (cv_server_* / cv_stream_*): frames of
several live streams, submitted interleaved and batched by the worker
thread into rounds ticks with keystream generated ahead, come out byte for
byte as the CPU oracle encrypts or decrypts each stream on its own."""
import time

import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (name, H, W, C, n, r, frames, decrypt)
SERVED = [
    ("srv-rgb48", 48, 48, 3, 8, 5, 7, False),
    ("srv-wide", 48, 64, 3, 5, 5, 5, True),
    ("srv-rgba", 33, 16, 4, 4, 3, 6, False),
    ("srv-n32", 96, 96, 3, 32, 5, 4, False),
    ("srv-gray", 32, 32, 1, 4, 5, 5, False),   # C = 1: the key's own path inside the server
    ("srv-odd", 31, 17, 3, 7, 4, 3, True),     # W % 16 != 0: likewise
]


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _wait(stream, ticket, timeout=20.0):
    t0 = time.time()
    while True:
        done, lat = stream.poll(ticket)
        if done:
            return lat
        assert time.time() - t0 < timeout, "frame not done in time"
        time.sleep(0.0005)


@pytest.mark.parametrize("budget,split", [(256 << 20, 1), (0, 1), (256 << 20, 2), (256 << 20, 0)])
def test_served_streams_match_oracle(B, budget, split):
    """Interleaved submission to streams of mixed sizes and directions equals
    the oracle frame by frame; with a fixed device-memory budget, and with
    budget 0 (rings allocated as streams open, by the free memory); with the
    keystream on a quarter or a half of every XCD's CUs, or on shared CUs."""
    srv = B.Server(hbm_budget=budget, ring_frames=2, queue_frames=3, split_cus=split)
    assert srv.stats()["hbm_budget"] == budget
    assert srv.stats()["split_cus"] == split
    cases = []
    for i, (name, H, W, C, n, r, T, dec) in enumerate(SERVED):
        pm = plcm_key(n, 5100 + i)
        frames = uniform_frames(H, W, C, T, 5200 + i)
        s_c = confusion_seeds(T, 5300 + i)
        ref = oracle.PlcmKey(H, W, C, n, r, pm)
        want = ref.decrypt(frames, s_c) if dec else ref.encrypt(frames, s_c)
        st = srv.open(H, W, C, n, r, pm, decrypt=dec)
        src = [torch.from_numpy(np.ascontiguousarray(frames[t]).reshape(-1)).to("cuda:0")
               for t in range(T)]
        out = [torch.empty_like(x) for x in src]
        cases.append(dict(name=name, st=st, src=src, out=out, s_c=s_c, want=want,
                          next=0, tickets=[]))
    if budget == 0:  # one chunk of at least 4 GiB holds every ring
        assert srv.stats()["hbm_budget"] >= 4 << 30
    print(f"[case] served streams, interleaved submission, budget {budget} split {split}", flush=True)
    torch.cuda.synchronize()
    # round-robin submission, retrying streams whose queue is full
    pending = True
    t0 = time.time()
    while pending:
        pending = False
        for c in cases:
            if c["next"] < len(c["src"]):
                pending = True
                t = c["next"]
                tk = c["st"].try_submit(c["src"][t], c["out"][t], int(c["s_c"][t]))
                if tk is not None:
                    assert tk == t
                    c["tickets"].append(tk)
                    c["next"] += 1
        assert time.time() - t0 < 60, "submission did not finish"
        time.sleep(0.0002)
    srv.drain()
    for c in cases:
        for t, tk in enumerate(c["tickets"]):
            lat = _wait(c["st"], tk)
            assert lat >= 0.0
            got = c["out"][t].cpu().numpy().reshape(c["want"][t].shape)
            assert np.array_equal(got, c["want"][t]), \
                f"{c['name']} frame {t}: {np.count_nonzero(got != c['want'][t])} bytes differ"
    stats = srv.stats()
    assert stats["frames_done"] == sum(len(c["src"]) for c in cases)
    assert stats["rounds_ticks"] >= 1 and stats["keystream_launches"] >= 1
    assert stats["open_streams"] == len(cases)
    for c in cases:
        c["st"].close()
    assert srv.stats()["open_streams"] == 0 and srv.stats()["hbm_used"] == 0
    srv.close()


def test_served_round_trip_and_late_open(B):
    """An encrypting and a decrypting stream of the same key in one server,
    the decrypting one opened after the first frames were served."""
    H, W, C, n, r, T = 64, 64, 3, 8, 5, 6
    pm = plcm_key(n, 77)
    frames = uniform_frames(H, W, C, T, 78)
    s_c = confusion_seeds(T, 79)
    srv = B.Server(hbm_budget=64 << 20)
    enc = srv.open(H, W, C, n, r, pm)
    src = [torch.from_numpy(np.ascontiguousarray(frames[t]).reshape(-1)).to("cuda:0")
           for t in range(T)]
    mid = [torch.empty_like(x) for x in src]
    back = [torch.empty_like(x) for x in src]
    print("[case] served round trip", flush=True)
    for t in range(3):
        _wait(enc, enc.submit(src[t], mid[t], int(s_c[t])))
    dec = srv.open(H, W, C, n, r, pm, decrypt=True)
    for t in range(3, T):
        enc.submit(src[t], mid[t], int(s_c[t]))
        srv.drain()
    for t in range(T):
        dec.submit(mid[t], back[t], int(s_c[t]))
        srv.drain()
    for t in range(T):
        assert torch.equal(back[t], src[t]), f"frame {t} did not decrypt"
    srv.close()


def test_server_admission_and_queue_limits(B):
    """A stream is admitted only while the budget holds its keystream ring;
    a full queue answers CV_E_AGAIN; closing frees the ring."""
    H, W, C, n, r = 48, 48, 3, 8, 5
    ring = 2 * r * H * W * C
    srv = B.Server(hbm_budget=ring + ring // 2, ring_frames=2, queue_frames=2)
    a = srv.open(H, W, C, n, r, plcm_key(n, 1))
    with pytest.raises(B.CvError) as e:
        srv.open(H, W, C, n, r, plcm_key(n, 2))
    assert e.value.status == B.CV_E_AGAIN
    for bad in (-1, 4):  # the split takes 0..3 quarters
        assert B.load().cv_server_tune(srv._h, 2, 2, bad) == B.CV_E_INVAL
    assert B.load().cv_server_tune(srv._h, 2, 2, 2) == B.CV_E_STATE  # a stream is open
    src = torch.from_numpy(uniform_frames(H, W, C, 3, 4).reshape(3, -1)).to("cuda:0")
    out = torch.empty_like(src)
    print("[case] server queue limits", flush=True)
    t0 = a.try_submit(src[0], out[0], 5)
    t1 = a.try_submit(src[1], out[1], 6)
    assert (t0, t1) == (0, 1)
    t2 = a.try_submit(src[2], out[2], 7)   # may be refused while both are in flight
    srv.drain()
    if t2 is None:
        assert a.submit(src[2], out[2], 7) == 2
        srv.drain()
    with pytest.raises(B.CvError):
        a.submit(src[0], src[0], 5)          # frame == out
    with pytest.raises(B.CvError):
        a.submit(src[0], out[0], 0)          # s_c = 0
    with pytest.raises(B.CvError):
        a.poll(99)                           # ticket not issued
    a.close()
    b = srv.open(H, W, C, n, r, plcm_key(n, 2))
    b.close()
    srv.close()
