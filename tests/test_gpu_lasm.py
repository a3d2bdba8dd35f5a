"""GPU parity of the 2DLASM generator (Sec. 3, Eq. (6)) against the CPU
oracle, bit for bit: the correctly rounded sine on millions of arguments
(fast path and exact path), the keystream, the whole cipher in both
directions, and 2DLASM streams inside batches and the server."""
import time

import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import confusion_seeds, lasm_key, plcm_key, uniform_frames

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PI = 3.141592653589793


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda:0")


def _host(t, shape):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


def _args(n, seed):
    r = np.random.default_rng(seed)
    t = np.concatenate([
        r.uniform(0.0, PI, n),
        np.exp(r.uniform(np.log(2.0 ** -60), np.log(PI), n // 4)),
        np.array([0.0, 5e-324, 1e-300, 2.0 ** -30, PI, np.nextafter(PI, 0), PI / 2,
                  np.nextafter(PI / 2, 0), np.nextafter(PI / 2, 4), 1.0, 3.0]),
    ])
    return t


@pytest.mark.parametrize("force_exact,n", [(False, 4_000_000), (True, 400_000)])
def test_cr_sin_matches_oracle(B, force_exact, n):
    t = _args(n, 7 + force_exact)
    print(f"[case] cr_sin force_exact={force_exact} n={t.size}", flush=True)
    want = oracle.cr_sin_array(t)
    td = torch.from_numpy(t).to("cuda:0")
    out = torch.empty_like(td)
    certain = B.cr_sin(td, out, force_exact=force_exact)
    got = out.cpu().numpy()
    bad = np.flatnonzero(got.view(np.uint64) != want.view(np.uint64))
    assert bad.size == 0, f"{bad.size} differ, e.g. t={t[bad[:3]]} got={got[bad[:3]]} want={want[bad[:3]]}"
    assert certain


GEOMS = [
    ("l-rgb48", 48, 48, 3, 8, 5, 2),
    ("l-ragged", 20, 36, 3, 3, 5, 2),
    ("l-rows", 9, 9, 1, 9, 3, 2),
    ("l-oneband", 17, 3, 1, 1, 5, 2),
    ("l-rgba", 40, 24, 4, 6, 5, 2),
    ("l-many", 64, 48, 3, 40, 5, 1),   # more than 32 chains: two workgroups
]


@pytest.mark.parametrize("geom", GEOMS, ids=[g[0] for g in GEOMS])
def test_lasm_keystream_and_cipher(B, geom):
    name, H, W, C, n, r, T = geom
    pm = lasm_key(n, 300 + H + W)
    frames = uniform_frames(H, W, C, T, 400 + H)
    s_c = confusion_seeds(T, 500 + W)
    print(f"[case] 2DLASM {name}", flush=True)
    ref = oracle.LasmKey(H, W, C, n, r, pm)
    ks_want = ref.keystream(T)
    k = B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
    ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
    k.keystream(ks, T)
    got = _host(ks, ks_want.shape)
    assert np.array_equal(got, ks_want), f"{np.count_nonzero(got != ks_want)} keystream bytes differ"
    x, fi = k.get_state()
    assert fi == T and np.array_equal(x, ref.state())
    # whole cipher, plain and fused paths, then decryption
    want = oracle.LasmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    for path in (B.CV_PATH_PLAIN, B.CV_PATH_FUSED):
        enc, dec = torch.empty_like(src), torch.empty_like(src)
        ke = B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
        ke.set_path(path)
        ke.encrypt(src, enc, s_c)
        assert np.array_equal(_host(enc, frames.shape), want), f"path {path}"
        kd = B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
        kd.set_path(path)
        kd.decrypt(enc, dec, s_c)
        assert torch.equal(dec, src)
        ke.get_state(), kd.get_state()  # raise if a sine was undecided


def test_lasm_full_size(B):
    H, W, C, n, r, T = 768, 768, 3, 16, 5, 1
    pm = lasm_key(n, 768)
    frames = uniform_frames(H, W, C, T, 769)
    s_c = confusion_seeds(T, 770)
    print("[case] 2DLASM rgb768", flush=True)
    want = oracle.LasmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc = torch.empty_like(src)
    k = B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
    k.encrypt(src, enc, s_c)
    got = _host(enc, frames.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"


def test_lasm_in_batch_and_server(B):
    """2DLASM streams run beside PLCM streams in a batch tick and in the
    server, with the oracle's bytes."""
    H, W, C, n, r = 48, 64, 3, 4, 5
    pl, pp = lasm_key(n, 61), plcm_key(n, 62)
    frames = uniform_frames(H, W, C, 2, 63)
    s_c = confusion_seeds(2, 64)
    want_l = oracle.LasmKey(H, W, C, n, r, pl).encrypt(frames, s_c)
    want_p = oracle.PlcmKey(H, W, C, n, r, pp).encrypt(frames, s_c)
    src = _dev(frames)
    print("[case] 2DLASM batch", flush=True)
    kl = B.Key(H, W, C, n, r, pl, map=B.CV_MAP_2DLASM)
    kp = B.Key(H, W, C, n, r, pp)
    ol, op = torch.empty_like(src), torch.empty_like(src)
    b = B.Batch()
    b.run([(kl, src, ol, s_c), (kp, src, op, s_c)])
    b.sync()
    assert b.info()["last_fallback_items"] == 1
    assert np.array_equal(_host(ol, frames.shape), want_l)
    assert np.array_equal(_host(op, frames.shape), want_p)
    b.close()
    print("[case] 2DLASM server", flush=True)
    srv = B.Server(hbm_budget=64 << 20)
    st = srv.open(H, W, C, n, r, pl, map=B.CV_MAP_2DLASM)
    fr = [_dev(frames[t]) for t in range(2)]
    out = [torch.empty_like(x) for x in fr]
    for t in range(2):
        st.submit(fr[t], out[t], int(s_c[t]))
    srv.drain()
    for t in range(2):
        assert np.array_equal(_host(out[t], frames[t].shape), want_l[t])
    srv.close()


def test_lasm_key_errors(B):
    H, W, C, n, r = 16, 16, 3, 2, 5
    good = lasm_key(n, 1)
    for bad_mu in (0.39, 0.43, 0.95, 0.36, 1.01):
        pm = good.copy()
        pm[1, 2] = bad_mu
        with pytest.raises(B.CvError) as e:
            B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
        assert e.value.status == B.CV_E_INVAL
    pm = good.copy()
    pm[0, 1] = 1.0  # y0 outside (0,1)
    with pytest.raises(B.CvError):
        B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)
    with pytest.raises(B.CvError):
        B.Key(H, W, C, n, r, good[:, :4], map=B.CV_MAP_2DLASM)  # 4 doubles per record
    pm = good.copy()
    pm[0, 2] = 1.0  # mu = 1 is admissible
    B.Key(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM)


def test_several_lasm_streams_in_the_server(B):
    """2DLASM streams of different sizes beside a PLCM stream in the server:
    one keystream launch holds the chains of every 2DLASM stream (of unequal
    lengths); each stream's frames equal the oracle's."""
    r = 5
    specs = [(48, 64, 3, 4, True), (32, 48, 3, 2, True), (64, 64, 4, 8, True), (48, 48, 3, 4, False)]
    T = 3
    srv = B.Server(hbm_budget=256 << 20, ring_frames=2, queue_frames=T)
    cases = []
    for i, (H, W, C, n, lasm) in enumerate(specs):
        pm = lasm_key(n, 8100 + i) if lasm else plcm_key(n, 8100 + i)
        frames = uniform_frames(H, W, C, T, 8200 + i)
        s_c = confusion_seeds(T, 8300 + i)
        ref = oracle.LasmKey(H, W, C, n, r, pm) if lasm else oracle.PlcmKey(H, W, C, n, r, pm)
        st = srv.open(H, W, C, n, r, pm, map=B.CV_MAP_2DLASM if lasm else B.CV_MAP_PLCM)
        src = [_dev(frames[t]) for t in range(T)]
        out = [torch.empty_like(x) for x in src]
        cases.append((st, src, out, s_c, ref.encrypt(frames, s_c)))
    print("[case] several 2DLASM streams in the server", flush=True)
    for t in range(T):
        for st, src, out, s_c, _ in cases:
            st.submit(src[t], out[t], int(s_c[t]))
    srv.drain()
    for i, (st, src, out, s_c, want) in enumerate(cases):
        for t in range(T):
            got = _host(out[t], want[t].shape)
            assert np.array_equal(got, want[t]), f"stream {i} frame {t}"
    srv.close()
