"""Oracle parity at the largest frame sizes of the batched and served
workloads: 1920x1080x3 streams with 8 subframes (bands of 135 rows, 777,600
bytes, more than one LDS tile per band; one encrypting, one decrypting) and
a 3840x2160x3 stream with 64 subframes, inside cv_batch_run ticks and
through the server, beside 64 small streams of 32 subframes each, so that
one keystream launch holds more than 2048 chains (more than 64 generator
workgroups: 32-step blocks).  Every byte of every stream is checked."""
import time

import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import (CorrelatedVideo, confusion_seeds, plcm_key,
                                         uniform_frames)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

R = 5
# (H, W, C, n, decrypt)
BIG = [(1080, 1920, 3, 8, False), (2160, 3840, 3, 64, False), (1080, 1920, 3, 8, True)]
SMALL = [(64, 64, 3, 32, False)] * 64


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _specs():
    specs = BIG + SMALL
    assert sum(s[3] for s in specs) > 2048
    return specs


def _frames(i, H, W, C, T, t0):
    if i < len(BIG):
        return CorrelatedVideo(H, W, C, 9100 + i).frames(t0, T)
    return uniform_frames(H, W, C, T, 9200 + 10 * i + t0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda:0")


def test_batch_ticks_with_1080p_and_4k_streams(B):
    specs = _specs()
    keys = [B.Key(H, W, C, n, R, plcm_key(n, 9000 + i)) for i, (H, W, C, n, _) in enumerate(specs)]
    refs = [oracle.PlcmKey(H, W, C, n, R, plcm_key(n, 9000 + i))
            for i, (H, W, C, n, _) in enumerate(specs)]
    b = B.Batch()
    for tick in range(2):
        print(f"[case] batch tick {tick}: 1080p n=8 enc+dec, 4K n=64, 64 x 64^2 n=32", flush=True)
        items, wants = [], []
        for i, (H, W, C, n, dec) in enumerate(specs):
            frames = _frames(i, H, W, C, 1, tick)
            s_c = confusion_seeds(1, 9300 + 10 * i + tick)
            src = _dev(frames)
            items.append((keys[i], src, torch.empty_like(src), s_c, dec))
            wants.append((refs[i].decrypt if dec else refs[i].encrypt)(frames, s_c))
        b.run(items)
        b.sync()
        torch.cuda.synchronize()
        for i, (it, want) in enumerate(zip(items, wants)):
            got = it[2].cpu().numpy().reshape(want.shape)
            assert np.array_equal(got, want), \
                f"tick {tick} stream {i} {specs[i]}: {np.count_nonzero(got != want)} bytes differ"
    b.close()


def test_served_1080p_and_4k_streams(B):
    specs = _specs()
    T = 2
    srv = B.Server(hbm_budget=2 << 30, ring_frames=2, queue_frames=2)
    cases = []
    for i, (H, W, C, n, dec) in enumerate(specs):
        pm = plcm_key(n, 9400 + i)
        frames = _frames(i, H, W, C, T, 0)
        s_c = confusion_seeds(T, 9500 + i)
        ref = oracle.PlcmKey(H, W, C, n, R, pm)
        want = ref.decrypt(frames, s_c) if dec else ref.encrypt(frames, s_c)
        st = srv.open(H, W, C, n, R, pm, decrypt=dec)
        src = [_dev(frames[t]) for t in range(T)]
        cases.append(dict(spec=(H, W, C, n, dec), st=st, src=src,
                          out=[torch.empty_like(x) for x in src], s_c=s_c, want=want,
                          next=0, tickets=[]))
    torch.cuda.synchronize()
    print(f"[case] served: {len(cases)} streams incl. 1080p n=8 enc+dec and 4K n=64", flush=True)
    pending, t0 = True, time.time()
    while pending:
        pending = False
        for c in cases:
            if c["next"] < T:
                pending = True
                tk = c["st"].try_submit(c["src"][c["next"]], c["out"][c["next"]],
                                        int(c["s_c"][c["next"]]))
                if tk is not None:
                    c["tickets"].append(tk)
                    c["next"] += 1
        assert time.time() - t0 < 60, "submission did not finish"
        time.sleep(0.0002)
    srv.drain()
    torch.cuda.synchronize()
    for c in cases:
        assert c["tickets"] == list(range(T))
        for t in range(T):
            done, _ = c["st"].poll(t)
            assert done
            got = c["out"][t].cpu().numpy().reshape(c["want"][t].shape)
            assert np.array_equal(got, c["want"][t]), \
                f"{c['spec']} frame {t}: {np.count_nonzero(got != c['want'][t])} bytes differ"
    assert srv.stats()["frames_done"] == T * len(cases)
    srv.close()
