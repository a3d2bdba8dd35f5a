"""The autotuners and their cache (CV_TUNE_CACHE): cv_batch_autotune over
the kernel, G, groups in flight and the LDS tiling, and cv_key_autotune over
the fused kernels and frame groups.  The first call for a shape class times
the candidates and stores the winner in the JSON file; a later call (another
batch object, another key) takes it from the file without timing.  Ticks
and frames with the chosen shapes equal the oracle byte for byte."""
import json

import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (H, W, C, n) of the batched streams: row-run eligible widths and one that is not
BATCH = [(48, 48, 3, 8), (96, 96, 3, 16), (64, 48, 3, 4), (48, 64, 3, 5)]


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CV_TUNE_CACHE", str(path))
    return path


def _items(B, seed, decrypt=False):
    items, wants = [], []
    for i, (H, W, C, n) in enumerate(BATCH):
        pm = plcm_key(n, seed + i)
        frames = uniform_frames(H, W, C, 1, seed + 10 + i)
        s_c = confusion_seeds(1, seed + 20 + i)
        ref = oracle.PlcmKey(H, W, C, n, 5, pm)
        wants.append((ref.decrypt if decrypt else ref.encrypt)(frames, s_c))
        src = torch.from_numpy(frames.reshape(-1)).to("cuda:0")
        items.append((B.Key(H, W, C, n, 5, pm), src, torch.empty_like(src), s_c, decrypt))
    return items, wants


def _check(items, wants):
    torch.cuda.synchronize()
    for it, want in zip(items, wants):
        assert np.array_equal(it[2].cpu().numpy().reshape(want.shape), want)


@pytest.mark.parametrize("decrypt", [False, True])
def test_batch_autotune_cache(B, cache, decrypt):
    print(f"[case] batch autotune cache decrypt={decrypt}", flush=True)
    items, wants = _items(B, 9600 + 100 * decrypt, decrypt)
    b1 = B.Batch()
    best1 = b1.autotune(items)
    info1 = b1.info()
    assert info1["tune_shapes_timed"] >= 8 and info1["tune_cache_hits"] == 0
    table = json.loads(cache.read_text())
    assert len(table) == 1
    (key, entry), = table.items()
    assert key.startswith("batch|") and entry["threads"] == best1["threads"]
    assert entry["group_wgs"] == best1["group_wgs"]
    b1.run(items)
    b1.sync()
    _check(items, wants)
    # a new batch object with the same shape class: taken from the file
    items2, wants2 = _items(B, 9600 + 100 * decrypt, decrypt)
    b2 = B.Batch()
    best2 = b2.autotune(items2)
    info2 = b2.info()
    assert info2["tune_cache_hits"] == 1 and info2["tune_shapes_timed"] == 0
    assert best2 == best1
    b2.run(items2)
    b2.sync()
    _check(items2, wants2)
    b1.close()
    b2.close()


def test_batch_cache_file_that_does_not_parse_is_replaced(B, cache):
    cache.write_text("{ not json")
    items, wants = _items(B, 9900)
    b = B.Batch()
    b.autotune(items)
    assert b.info()["tune_shapes_timed"] > 0
    assert len(json.loads(cache.read_text())) == 1
    b.run(items)
    b.sync()
    _check(items, wants)
    b.close()


@pytest.mark.parametrize("decrypt", [False, True])
@pytest.mark.parametrize("geom", [(768, 768, 3, 16, 6), (48, 64, 3, 5, 20)],
                         ids=["rgb768", "rgb48x64"])
def test_key_autotune_cache(B, cache, geom, decrypt):
    H, W, C, n, T = geom
    r = 5
    print(f"[case] key autotune {geom} decrypt={decrypt}", flush=True)
    pm = plcm_key(n, 9700 + H)
    frames = uniform_frames(H, W, C, T, 9701 + H)
    s_c = confusion_seeds(T, 9702 + H)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.decrypt(frames, s_c) if decrypt else ref.encrypt(frames, s_c)
    k1 = B.Key(H, W, C, n, r, pm)
    state0 = k1.get_state()
    l1, hit1 = k1.autotune(decrypt, T)
    assert not hit1 and l1["round_variant"] in (2, 3) and l1["fused_groups"] >= 8
    x, fi = k1.get_state()
    assert fi == state0[1] and np.array_equal(x, state0[0])    # the generator did not move
    table = json.loads(cache.read_text())
    assert any(k.startswith("key|") for k in table)
    src = torch.from_numpy(frames.reshape(-1)).to("cuda:0")
    out = torch.empty_like(src)
    (k1.decrypt if decrypt else k1.encrypt)(src, out, s_c)
    k1.sync()
    assert np.array_equal(out.cpu().numpy().reshape(want.shape), want)
    k2 = B.Key(H, W, C, n, r, pm)
    l2, hit2 = k2.autotune(decrypt, T)
    assert hit2 and l2 == l1
    out2 = torch.empty_like(src)
    (k2.decrypt if decrypt else k2.encrypt)(src, out2, s_c)
    k2.sync()
    assert torch.equal(out2, out)


def test_key_autotune_rejects(B, cache):
    k = B.Key(31, 17, 3, 7, 4, plcm_key(7, 1))     # W % 16 != 0: no fused path
    with pytest.raises(B.CvError) as e:
        k.autotune(False, 4)
    assert e.value.status == B.CV_E_INVAL
    k2 = B.Key(48, 48, 3, 8, 5, plcm_key(8, 2))
    with pytest.raises(B.CvError):
        k2.autotune(False, 0)
