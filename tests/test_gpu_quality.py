"""Sec. 4 and 5 measures of GPU ciphertexts through the statistical harness
(seeded inputs, so every outcome is fixed): uniformity below the paper's
chi-square critical value, entropy near 8, local entropy near its expected
value, adjacent-pixel correlation near 0, NPCR/UACI within the paper's 512^2
thresholds with the same keystream, key sensitivity at delta = 1e-9, and
decryption under channel noise."""
import numpy as np
import pytest

from paper_2302_07411_amd import analysis as A
from paper_2302_07411_amd.inputs import CorrelatedVideo, confusion_seeds, plcm_key

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2302_07411_amd import binding
    binding.load()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return binding


def _enc(B, H, W, C, n, r, pm, frames, s_c):
    src = torch.from_numpy(np.ascontiguousarray(frames).reshape(-1)).cuda()
    out = torch.empty_like(src)
    B.Key(H, W, C, n, r, pm).encrypt(src, out, s_c)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(frames.shape)


def test_cipher_statistics(B):
    H, W, C, n, r = 768, 768, 3, 16, 5
    print("[case] statistics 768", flush=True)
    frames = CorrelatedVideo(H, W, C, 901).frames(0, 1)
    cipher = _enc(B, H, W, C, n, r, plcm_key(n, 902), frames, confusion_seeds(1, 903))[0]
    s = A.frame_summary(frames[0], cipher, np.random.default_rng(904))
    assert max(s["chi2"]) < A.CHI2_CRITICAL_005
    assert min(s["entropy"]) > 7.999
    assert all(7.89 < h < 7.915 for h in s["local_entropy"])
    for c in s["corr_cipher"]:
        assert all(abs(v) < 0.02 for v in c.values())
    for c in s["corr_plain"]:
        assert all(v > 0.8 for v in c.values())  # the synthetic video is correlated
    assert min(s["variance_plain"]) > 10 * max(s["variance_cipher"])


def test_differential_512(B):
    H, W, C, n, r = 512, 512, 3, 16, 5
    print("[case] NPCR/UACI 512", flush=True)
    k = B.Key(H, W, C, n, r, plcm_key(n, 911))
    ks = torch.empty(r * H * W * C, dtype=torch.uint8, device="cuda")
    k.keystream(ks, 1)
    sc = confusion_seeds(1, 912)
    p0 = CorrelatedVideo(H, W, C, 913).frame(0)
    pd = torch.from_numpy(p0.reshape(-1)).cuda()
    c1, c2 = torch.empty_like(pd), torch.empty_like(pd)
    k.apply_rounds(False, pd, c1, ks, sc)
    a1 = c1.cpu().numpy().reshape(H, W, C)
    rng = np.random.default_rng(914)
    npcr, uaci = [], []
    for _ in range(20):
        p2 = p0.copy()
        i, j, c = int(rng.integers(H)), int(rng.integers(W)), int(rng.integers(C))
        p2[i, j, c] = (int(p2[i, j, c]) + 1) % 256  # one step: the low bit always flips
        k.apply_rounds(False, torch.from_numpy(p2.reshape(-1)).cuda(), c2, ks, sc)
        a2 = c2.cpu().numpy().reshape(H, W, C)
        npcr.append(np.mean([A.npcr(a1[..., q], a2[..., q]) for q in range(C)]))
        uaci.append(np.mean([A.uaci(a1[..., q], a2[..., q]) for q in range(C)]))
    assert np.mean(npcr) > A.NPCR_MIN_512
    assert A.UACI_RANGE_512[0] <= np.mean(uaci) <= A.UACI_RANGE_512[1]
    assert min(npcr) > 99.4   # a change anywhere reaches the whole frame
    # a change confined to bits >= 1 never reaches bit 0 (Eq. 3 is linear in
    # the high bits): NPCR settles near 100 * (1 - 1/128)
    p2 = p0.copy()
    p2[7, 9, 1] ^= 2
    k.apply_rounds(False, torch.from_numpy(p2.reshape(-1)).cuda(), c2, ks, sc)
    a2 = c2.cpu().numpy().reshape(H, W, C)
    assert 98.9 < A.npcr(a1, a2) < 99.5
    assert np.all(((a1 ^ a2) & 1) == 0)


def test_key_sensitivity_and_noise(B):
    """The paper moves the key K (the master generator's initial value or
    control parameter) by 1e-9; through the key schedule that changes every
    band's parameters and every frame's confusion seed."""
    H, W, C, n, r = 256, 256, 3, 8, 5
    print("[case] key sensitivity 256", flush=True)
    K = [0.6180339887, 0.2718281828, 0.3141592653, 0.1414213562]
    pm, sc = B.key_schedule(K, n, 0, 1)
    frames = CorrelatedVideo(H, W, C, 922).frames(0, 1)
    cipher = _enc(B, H, W, C, n, r, pm, frames, sc)

    def dec(pm_, sc_, c):
        src = torch.from_numpy(np.ascontiguousarray(c).reshape(-1)).cuda()
        out = torch.empty_like(src)
        B.Key(H, W, C, n, r, pm_).decrypt(src, out, sc_)
        torch.cuda.synchronize()
        return out.cpu().numpy().reshape(c.shape)

    good = dec(pm, sc, cipher)
    assert np.array_equal(good, frames)
    for q in (0, 1):  # x0 or p of the master generator moved by 1e-9
        K2 = list(K)
        K2[q] += 1e-9
        pm2, sc2 = B.key_schedule(K2, n, 0, 1)
        bad = dec(pm2, sc2, cipher)
        assert abs(A.correlation(good, bad)) < 0.02
        assert A.npcr(bad, frames) > 99.0
    rng = np.random.default_rng(924)
    ps = [A.psnr(frames, dec(pm, sc, A.salt_and_pepper(cipher[0], f, rng)[None]))
          for f in (0.01, 0.03, 0.05)]
    assert ps[0] > ps[1] > ps[2]
