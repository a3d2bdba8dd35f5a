"""GPU parity: libchaosvid (HIP, gfx950) against the CPU oracle, byte for
byte, through the C ABI.  Bar: bit-exact (the cipher is byte and index work
and its FP64 chaotic maps admit no rounding drift)."""
import numpy as np
import pytest

import oracle
from paper_2302_07411_amd.inputs import (CorrelatedVideo, confusion_seeds, plcm_key,
                                         uniform_frames)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (name, H, W, C, n, r, T)
GEOMS = [
    ("gray256", 256, 256, 1, 4, 5, 1),     # the single-frame gray case
    ("rgb48", 48, 48, 3, 8, 5, 3),
    ("ragged", 20, 36, 3, 3, 5, 2),        # non-square, n does not divide H, unaligned rows
    ("tall", 36, 20, 3, 5, 2, 2),
    ("rowbands", 9, 9, 1, 9, 3, 2),        # one row per band
    ("oneband", 17, 3, 1, 1, 5, 2),        # a single band seeds itself
    ("odd", 31, 17, 3, 7, 4, 2),
    ("rgba", 40, 24, 4, 6, 5, 2),
    ("wide", 24, 4096, 3, 2, 5, 1),        # bands span several LDS tiles
    ("tiny", 2, 1, 1, 1, 1, 3),            # smallest legal frame: 2 bytes
]
IDS = [g[0] for g in GEOMS]


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


def _case(name, H, W, C, n, r, T, seed=0):
    pm = plcm_key(n, 2000 + seed + H * 7 + W)
    frames = uniform_frames(H, W, C, T, 1000 + seed + H)
    s_c = confusion_seeds(T, 3000 + seed + W)
    print(f"[case] {name} H={H} W={W} C={C} n={n} r={r} T={T} seed={seed}", flush=True)
    return pm, frames, s_c


@pytest.mark.parametrize("variant", [0, 5])
@pytest.mark.parametrize("geom", GEOMS, ids=IDS)
def test_keystream_parity(B, geom, variant):
    """Every geometry's keystream and final state against the oracle, with
    the default generator and with planted errors (chains of one step to a
    few blocks: repairs of a first, a last and a single block)."""
    name, H, W, C, n, r, T = geom
    pm, _, _ = _case(*geom)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.keystream(T)
    key = B.Key(H, W, C, n, r, pm)
    key.set_launch(prbg_variant=variant)
    ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
    key.keystream(ks, T)
    got = _host(ks, want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} keystream bytes differ"
    x, fi = key.get_state()
    assert fi == T
    assert np.array_equal(x[:, 0], ref.x1) and np.array_equal(x[:, 1], ref.x2)


@pytest.mark.parametrize("geom", GEOMS, ids=IDS)
def test_rounds_parity(B, geom):
    """The r rounds alone, fed the oracle's keystream."""
    name, H, W, C, n, r, T = geom
    pm, frames, s_c = _case(*geom, seed=1)
    ks = oracle.PlcmKey(H, W, C, n, r, pm).keystream(T)
    want = np.empty_like(frames)
    for t in range(T):
        g = oracle.gtable(H, int(s_c[t]))
        A = frames[t]
        for j in range(r):
            A = oracle.diffuse(oracle.confuse(A, g), n, r, j, ks[t])
        want[t] = A
    key = B.Key(H, W, C, n, r, pm)
    src, ksd = _dev(frames), _dev(ks)
    enc = torch.empty_like(src)
    key.apply_rounds(False, src, enc, ksd, s_c)
    got = _host(enc, frames.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} cipher bytes differ"
    dec = torch.empty_like(src)
    key.apply_rounds(True, _dev(want), dec, ksd, s_c)
    assert np.array_equal(_host(dec, frames.shape), frames)


@pytest.mark.parametrize("geom", GEOMS, ids=IDS)
def test_encrypt_decrypt_parity(B, geom):
    name, H, W, C, n, r, T = geom
    pm, frames, s_c = _case(*geom, seed=2)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc, dec = torch.empty_like(src), torch.empty_like(src)
    B.Key(H, W, C, n, r, pm).encrypt(src, enc, s_c)
    got = _host(enc, frames.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} cipher bytes differ"
    B.Key(H, W, C, n, r, pm).decrypt(enc, dec, s_c)
    assert np.array_equal(_host(dec, frames.shape), frames)


def test_decrypt_matches_oracle_on_foreign_cipher(B):
    """Decrypting bytes that are not a valid cipher of anything in
    particular: GPU and oracle must still agree byte for byte."""
    H, W, C, n, r, T = 30, 26, 3, 4, 5, 2
    pm, frames, s_c = _case("foreign", H, W, C, n, r, T, seed=3)
    want = oracle.PlcmKey(H, W, C, n, r, pm).decrypt(frames, s_c)
    src = _dev(frames)
    out = torch.empty_like(src)
    B.Key(H, W, C, n, r, pm).decrypt(src, out, s_c)
    assert np.array_equal(_host(out, frames.shape), want)


def test_state_continuation_and_checkpoint(B):
    H, W, C, n, r, T = 32, 40, 3, 4, 5, 6
    pm, _, s_c = _case("continuation", H, W, C, n, r, T, seed=4)
    frames = CorrelatedVideo(H, W, C, 5).frames(0, T)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    out = torch.empty_like(src)
    F = H * W * C
    key = B.Key(H, W, C, n, r, pm)
    key.encrypt(src[:2 * F], out[:2 * F], s_c[:2])
    state, fi = key.get_state()
    assert fi == 2
    key.encrypt(src[2 * F:4 * F], out[2 * F:4 * F], s_c[2:4])
    # resume frames 4.. on a fresh key from the checkpoint after frame 4
    state4, fi4 = key.get_state()
    fresh = B.Key(H, W, C, n, r, pm)
    fresh.set_state(state4, fi4)
    fresh.encrypt(src[4 * F:], out[4 * F:], s_c[4:])
    assert np.array_equal(_host(out, frames.shape), want)


@pytest.mark.parametrize("launch", [
    dict(batch_frames=1), dict(batch_frames=2, threads=256, prbg_variant=1), dict(threads=64, tile_rows_enc=1,
                                                                  tile_rows_dec=1),
    dict(threads=512, tile_rows_enc=3, tile_rows_dec=5, prbg_variant=2), dict(threads=128, tile_rows_enc=7,
                                                              tile_rows_dec=64),
    dict(prbg_variant=3), dict(prbg_variant=4), dict(batch_frames=2, prbg_variant=5),
])
def test_launch_shapes_give_identical_bytes(B, launch):
    H, W, C, n, r, T = 50, 44, 3, 6, 5, 5
    pm, frames, s_c = _case(f"launch {launch}", H, W, C, n, r, T, seed=5)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc, dec = torch.empty_like(src), torch.empty_like(src)
    k = B.Key(H, W, C, n, r, pm)
    k.set_launch(**launch)
    k.encrypt(src, enc, s_c)
    assert np.array_equal(_host(enc, frames.shape), want)
    k2 = B.Key(H, W, C, n, r, pm)
    k2.set_launch(**launch)
    k2.decrypt(enc, dec, s_c)
    assert np.array_equal(_host(dec, frames.shape), frames)


def test_special_orbits(B):
    """Keys on the PLCM's special orbits (x0 = p, x0 = 1/2 reach the fixed
    point 0): the degenerate map contributes zero bytes."""
    H, W, C, n, r, T = 16, 16, 1, 4, 5, 2
    pm = plcm_key(n, 77)
    pm[0, 0] = pm[0, 1]          # x0 = p -> 0
    pm[1, 2] = 0.5               # x0 = 1/2 -> 1 -> 0
    pm[2, 0] = 0.125
    pm[2, 1] = 0.25              # exact dyadic orbit to 0
    pm[3, 0], pm[3, 2] = pm[3, 1], pm[3, 3]   # both maps degenerate: zero keystream
    _, frames, s_c = _case("special", H, W, C, n, r, T, seed=6)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want_ks = ref.keystream(T)
    key = B.Key(H, W, C, n, r, pm)
    ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
    key.keystream(ks, T)
    assert np.array_equal(_host(ks, want_ks.shape), want_ks)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc = torch.empty_like(src)
    B.Key(H, W, C, n, r, pm).encrypt(src, enc, s_c)
    assert np.array_equal(_host(enc, frames.shape), want)


def test_exact_division_path_and_tiny_keys(B):
    """Keys outside the reciprocal-division domain (p < 2^-64 or a tiny
    initial value) run the IEEE-division path; the same key with the path
    forced gives the same bytes as the reciprocal path."""
    H, W, C, n, r, T = 24, 20, 3, 4, 5, 3
    pm = plcm_key(n, 31)
    pm[1, 0] = 1e-300                 # tiny initial value
    pm[2, 3] = 2.0 ** -70             # tiny control parameter
    _, frames, s_c = _case("tiny-keys", H, W, C, n, r, T, seed=8)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc = torch.empty_like(src)
    B.Key(H, W, C, n, r, pm).encrypt(src, enc, s_c)
    assert np.array_equal(_host(enc, frames.shape), want)
    pm2 = plcm_key(n, 32)
    ref = oracle.PlcmKey(H, W, C, n, r, pm2).keystream(T)
    for variant in (0, 1, 2, 3, 4, 5):
        k = B.Key(H, W, C, n, r, pm2)
        k.set_launch(prbg_variant=variant)
        ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
        k.keystream(ks, T)
        assert np.array_equal(_host(ks, ref.shape), ref)


@pytest.mark.parametrize("variant", [0, 2, 3, 4, 5])
def test_fast_division_domain_edge(B, variant):
    """Keys at the edge of the reciprocal division's domain (p >= 2^-64,
    states 0 or >= 2^-800), which the key set-up accepts for the fast
    generators: the smallest p (2^-64, so nearly every step takes the second
    piece with numerators x - p down to ulp(p) = 2^-116), the largest p
    (1/2 - ulp, so 1/2 - p = 2^-54), the smallest initial state (2^-800,
    growing by at least 2 per step through the first piece), and the largest
    (1 - 2^-53, which folds to 2^-53).  Keystream and final state against the
    oracle for every fast variant, planted errors included."""
    H, W, C, n, r, T = 64, 32, 3, 4, 5, 3
    pm = plcm_key(n, 91)
    pm[0, 1] = 2.0 ** -64
    pm[1, 3] = np.nextafter(0.5, 0.0)
    pm[2, 0] = 2.0 ** -800
    pm[3, 2] = np.nextafter(1.0, 0.0)
    for x0, p in ((pm[:, 0], pm[:, 1]), (pm[:, 2], pm[:, 3])):
        assert np.all(p >= 2.0 ** -64) and np.all(x0 >= 2.0 ** -800)
    print(f"[case] fast-division domain edge variant={variant}", flush=True)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.keystream(T)
    key = B.Key(H, W, C, n, r, pm)
    key.set_launch(prbg_variant=variant)
    ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
    key.keystream(ks, T)
    got = _host(ks, want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} keystream bytes differ"
    x, _ = key.get_state()
    assert np.array_equal(x[:, 0], ref.x1) and np.array_equal(x[:, 1], ref.x2)


@pytest.mark.parametrize("variant", [2, 3, 4, 5])
def test_long_keystream(B, variant):
    """About 26 million chain steps (52 million divisions) against the
    oracle: the reciprocal division over long chaotic orbits, 32 chains (two
    wavefronts in the per-piece variant), frames straddling ring blocks.
    Variant 4 is the verified two-operation quotient; variant 5 plants a
    one-bit error in every 29th producer step of every lane (found by the
    checkpoint comparison) and in every 58th step of the verifiers'
    recomputation (found by the per-step check), so the bytes are right
    only if the verifiers catch every planted error and the repair
    recomputes the orbit."""
    H, W, C, n, r, T = 1024, 1024, 3, 32, 5, 10
    pm = plcm_key(n, 4242)
    print(f"[case] long keystream H={H} W={W} C={C} n={n} T={T} variant={variant}", flush=True)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.keystream(T)
    key = B.Key(H, W, C, n, r, pm)
    key.set_launch(prbg_variant=variant)
    ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
    key.keystream(ks, T)
    got = _host(ks, want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    x, _ = key.get_state()
    assert np.array_equal(x[:, 0], ref.x1) and np.array_equal(x[:, 1], ref.x2)


@pytest.mark.parametrize("n", [2048, 2049, 2112])
@pytest.mark.parametrize("variant", [4, 5])
def test_many_workgroups_keystream(B, variant, n):
    """2048 chains fill 64 workgroups, the most that still run 64-step
    blocks; 2049 and 2112 chains take 65 and 66 workgroups and 32-step
    blocks (the configuration the serving loop uses). All against the
    oracle, with and without planted errors."""
    H, W, C, r, T = n, 64, 1, 5, 4
    pm = plcm_key(n, 4343)
    print(f"[case] many workgroups H={H} W={W} n={n} T={T} variant={variant}", flush=True)
    ref = oracle.PlcmKey(H, W, C, n, r, pm)
    want = ref.keystream(T)
    key = B.Key(H, W, C, n, r, pm)
    key.set_launch(prbg_variant=variant)
    ks = torch.empty(T * r * H * W * C, dtype=torch.uint8, device="cuda:0")
    key.keystream(ks, T)
    got = _host(ks, want.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    x, _ = key.get_state()
    assert np.array_equal(x[:, 0], ref.x1) and np.array_equal(x[:, 1], ref.x2)


@pytest.mark.parametrize("name,H,W,C,n,r,T", [
    ("rgb480", 480, 480, 3, 8, 5, 3),
    ("rgb768", 768, 768, 3, 16, 5, 3),
])
def test_full_size_video(B, name, H, W, C, n, r, T):
    """The video workloads at their real frame sizes and subframe counts,
    correlated frames, default launch shape; every byte checked."""
    pm = plcm_key(n, 2000 + H)
    frames = CorrelatedVideo(H, W, C, 1000 + H).frames(0, T)
    s_c = confusion_seeds(T, 2000 + H)
    print(f"[case] {name} T={T}", flush=True)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc, dec = torch.empty_like(src), torch.empty_like(src)
    B.Key(H, W, C, n, r, pm).encrypt(src, enc, s_c)
    got = _host(enc, frames.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    B.Key(H, W, C, n, r, pm).decrypt(enc, dec, s_c)
    assert torch.equal(dec, src)


def test_errors_leave_the_key_unchanged(B):
    H, W, C, n, r = 16, 16, 3, 2, 5
    pm, frames, s_c = _case("errors", H, W, C, n, r, 2, seed=7)
    key = B.Key(H, W, C, n, r, pm)
    src = _dev(frames)
    out = torch.empty_like(src)
    before = key.get_state()
    with pytest.raises(B.CvError) as e:
        key.encrypt(src, out, [5, 0])
    assert e.value.status == B.CV_E_INVAL
    with pytest.raises(B.CvError):
        key.encrypt(src, src, s_c)                   # in/out overlap
    with pytest.raises(B.CvError):
        key.set_launch(threads=100)
    with pytest.raises(B.CvError):
        key.set_state(np.full((n, 2), 1.5), 0)
    after = key.get_state()
    assert np.array_equal(before[0], after[0]) and before[1] == after[1]
    # the key still works and matches the oracle from frame 0
    key.encrypt(src, out, s_c)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    assert np.array_equal(_host(out, frames.shape), want)


def test_zero_frames_is_a_noop(B):
    H, W, C, n, r = 8, 8, 1, 2, 5
    key = B.Key(H, W, C, n, r, plcm_key(n, 1))
    empty = torch.empty(0, dtype=torch.uint8, device="cuda:0")
    key.encrypt(empty, empty, [])
    assert key.get_state()[1] == 0


# Geometries the pixel-word kernels take (C in {3,4}, W % 16 == 0): wide,
# tall, one band, bands split over several LDS tiles, 4 channels.
PW_GEOMS = [
    ("pw-rgb48", 48, 48, 3, 8, 5, 2),
    ("pw-wide", 48, 64, 3, 5, 5, 2),
    ("pw-tall", 80, 32, 3, 7, 5, 2),
    ("pw-rgba", 33, 16, 4, 4, 3, 2),
    ("pw-rgba-wide", 20, 48, 4, 3, 5, 2),
    ("pw-oneband", 64, 48, 3, 1, 5, 2),
    ("pw-rowbands", 12, 16, 3, 12, 2, 2),
]


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("tile", [0, 1, 3])
@pytest.mark.parametrize("geom", PW_GEOMS, ids=[g[0] for g in PW_GEOMS])
def test_round_variants(B, geom, variant, tile):
    """Byte kernels (1) and pixel-word kernels (2) against the oracle, with
    the default and with tiny LDS tiles (a band over many tiles)."""
    name, H, W, C, n, r, T = geom
    pm, frames, s_c = _case(f"{name} round_variant={variant} tile={tile}", H, W, C, n, r, T,
                            seed=9)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    launch = dict(round_variant=variant)
    if tile:
        launch.update(tile_rows_enc=tile, tile_rows_dec=tile, tile_rows_pw=tile)
    src = _dev(frames)
    enc, dec = torch.empty_like(src), torch.empty_like(src)
    k = B.Key(H, W, C, n, r, pm)
    k.set_launch(**launch)
    k.encrypt(src, enc, s_c)
    got = _host(enc, frames.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    k2 = B.Key(H, W, C, n, r, pm)
    k2.set_launch(**launch)
    k2.decrypt(enc, dec, s_c)
    assert np.array_equal(_host(dec, frames.shape), frames)


# wide frames: the row-run encryption kernel splits a band into several LDS
# tiles (19 rows of 1920 pixels), with W a multiple of H and not
FUSED_GEOMS = PW_GEOMS + [
    ("wide1920-full", 64, 1920, 3, 2, 5, 2),
    ("wide1920", 100, 1920, 3, 3, 5, 2),
    # tall narrow bands: LDS tiles of more rows than a third of the
    # workgroup's threads (each row has three wrap words), one tile per band
    # (512 rows) and two tiles per band (1017 + 383 rows)
    ("tall-narrow", 4096, 16, 3, 8, 5, 2),
    ("tall-narrow-rgba", 2800, 32, 4, 2, 3, 2),
]


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("groups", [0, 8])
@pytest.mark.parametrize("geom", FUSED_GEOMS, ids=[g[0] for g in FUSED_GEOMS])
def test_fused_path(B, geom, groups, variant):
    """All r rounds in one persistent launch (groups of n workgroups with a
    barrier per round): same bytes as the oracle.  With 8 groups and 20
    frames every group walks several frames.  Variant 2 encrypts with the
    pixel-word tiles, variant 3 by whole source-row runs."""
    name, H, W, C, n, r, _ = geom
    T = 20 if W < 1000 else 4
    pm, frames, s_c = _case(f"{name} fused groups={groups} variant={variant}", H, W, C, n, r, T,
                            seed=10)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc, dec = torch.empty_like(src), torch.empty_like(src)
    k = B.Key(H, W, C, n, r, pm)
    k.set_path(B.CV_PATH_FUSED)
    k.set_launch(fused_groups=groups, round_variant=variant)
    assert k.get_launch()["fused_groups"] > 0
    k.encrypt(src, enc, s_c)
    k.get_state()   # raises if a group barrier timed out or a group spanned XCDs
    got = _host(enc, frames.shape)
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} bytes differ"
    k2 = B.Key(H, W, C, n, r, pm)
    k2.set_path(B.CV_PATH_FUSED)
    k2.set_launch(fused_groups=groups, round_variant=variant)
    k2.decrypt(enc, dec, s_c)
    k2.get_state()
    assert np.array_equal(_host(dec, frames.shape), frames)


def test_fused_path_full_size(B):
    H, W, C, n, r, T = 768, 768, 3, 16, 5, 6
    pm = plcm_key(n, 2000 + H)
    frames = CorrelatedVideo(H, W, C, 1000 + H).frames(0, T)
    s_c = confusion_seeds(T, 2000 + H)
    print("[case] fused rgb768", flush=True)
    want = oracle.PlcmKey(H, W, C, n, r, pm).encrypt(frames, s_c)
    src = _dev(frames)
    enc, dec = torch.empty_like(src), torch.empty_like(src)
    k = B.Key(H, W, C, n, r, pm)
    k.set_path(B.CV_PATH_FUSED)
    k.encrypt(src, enc, s_c)
    assert np.array_equal(_host(enc, frames.shape), want)
    k2 = B.Key(H, W, C, n, r, pm)
    k2.set_path(B.CV_PATH_FUSED)
    k2.decrypt(enc, dec, s_c)
    assert torch.equal(dec, src)
