"""GPU parity of the ciphertext product with relinearization (Sec. 2.2.3) and of the
operations built on it: key-switching keys and products are compared with the CPU
oracle residue by residue (bit-exact); the squared-difference image match (Sec. 4.4.3)
and the watermark (Sec. 4.4.4) are checked on their decrypted values as well."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PROD_TOL = 0.05  # pixel^2 units after the product and one rescale (oracle pin tolerance)
CUBE_TOL = 2.0   # a second product at level 2 decodes at scale ~2^18 (N=4096, 36-bit primes): noise ~0.5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_03568_amd as P

    P.lib()
    return P


@pytest.fixture(scope="module")
def W():
    from paper_2409_03568_amd import workloads

    return workloads


def _make(P, oracle_mod, W, cfg):
    c = W.CONFIGS[cfg]
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale)
    o = oracle_mod.Oracle(c.log_n, c.num_primes, c.prime_bits, c.log_scale)
    ctx.keygen(W.keygen_seed(cfg))
    o.keygen(W.keygen_seed(cfg))
    rseed = (W.keygen_seed(cfg)[0] ^ 0x5E1, cfg)
    ctx.relin_keygen(rseed)
    o.relin_keygen(rseed)
    return ctx, o


@pytest.fixture(scope="module")
def c1(P, oracle_mod, W):
    _say("[gpu] mul context C1 (N=4096, 3x36-bit)")
    return _make(P, oracle_mod, W, 1)


@pytest.fixture(scope="module")
def c2(P, oracle_mod, W):
    _say("[gpu] mul context C2 (N=8192, 4x50-bit)")
    return _make(P, oracle_mod, W, 2)


def _dev(px):
    import torch

    return torch.from_numpy(np.ascontiguousarray(px, dtype=np.uint8).reshape(-1)).cuda()


def _np(cts):
    import torch

    torch.cuda.synchronize()
    return cts.to_numpy().reshape(cts.count, -1)


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_relin_keys_bitexact(request, which):
    ctx, o = request.getfixturevalue(which)
    _say("[gpu] relin keys %s" % which)
    evk, qP = ctx.relin_keys_export()
    assert qP == o.qP
    ref = o.evk.reshape(evk.shape)
    bad = np.argwhere(np.any(evk != ref, axis=-1))
    assert bad.size == 0, "mismatching (digit, prime, poly): %s" % bad[:8].tolist()


def test_mul_c1_bitexact_and_decrypts(c1, W):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:64]
    _say("[gpu] mul C1 32 pairs")
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    a, b = cts[0:32], cts[32:64]
    A, B = _np(a), _np(b)
    m = ctx.mul(a, b)
    assert m.level == 3 and m.scale == a.scale * b.scale
    g = _np(m)
    for i in range(32):
        assert np.array_equal(g[i], o.mul(A[i], B[i])), i
    r = ctx.rescale(m)
    dec = ctx.decrypt_pixels(r).cpu().numpy()
    want = px[:32].astype(np.float64) * px[32:64]
    assert np.max(np.abs(dec - want)) < PROD_TOL


def test_mul_lower_level_and_unequal_scales(c1, W):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:16]
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    # level 2 at scale Delta: a fractional constant and a rescale
    h = ctx.rescale(ctx.mul_const(cts, 0.5))
    H = _np(h)
    assert h.level == 2
    m = ctx.mul(h[0:8], h[8:16])
    g = _np(m)
    for i in range(8):
        assert np.array_equal(g[i], o.mul(H[i], H[8 + i], level=2)), i
    dec = ctx.decrypt_pixels(ctx.rescale(m)).cpu().numpy()
    want = 0.25 * px[:8].astype(np.float64) * px[8:16]
    assert np.max(np.abs(dec - want)) < CUBE_TOL
    # one level, two scales: a rescaled product (Delta^2 / q_2) times a rescaled
    # fractional constant (Delta)
    p2 = ctx.rescale(ctx.mul(cts[0:8], cts[0:8]))
    t3 = ctx.rescale(ctx.mul_const(cts[0:8], 1.0 / 3.0))
    assert p2.level == t3.level == 2 and p2.scale != t3.scale
    sq = ctx.mul(p2, t3)
    assert sq.scale == p2.scale * t3.scale
    g, P2, T3 = _np(sq), _np(p2), _np(t3)
    for i in range(8):
        assert np.array_equal(g[i], o.mul(P2[i], T3[i], level=2)), i
    dec = ctx.decrypt_pixels(ctx.rescale(sq)).cpu().numpy()
    want = px[:8].astype(np.float64) ** 3 / 3.0
    assert np.max(np.abs(dec - want)) < CUBE_TOL


def test_mul_in_place_and_errors(P, c1, W):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:8]
    a = ctx.encrypt_pixels(_dev(px), (7, 7))
    b = ctx.encrypt_pixels(_dev(px[::-1].copy()), (8, 8))
    ref = _np(ctx.mul(a, b))
    ctx.mul(a, b, out=a)
    assert np.array_equal(_np(a), ref)
    a = ctx.encrypt_pixels(_dev(px), (7, 7))
    ctx.mul(a, b, out=b)
    assert np.array_equal(_np(b), ref)
    empty = ctx.mul(a[0:0], a[0:0])
    assert empty.count == 0
    with pytest.raises(P.CkksError) as ei:
        ctx.mul(a, ctx.rescale(a))
    assert ei.value.name == "CKKS_ELEVEL"
    with pytest.raises(P.CkksError) as ei:
        ctx.mul(a[0:4], a[0:3])
    assert ei.value.name == "CKKS_EINVAL"
    fresh = P.Context(12, 3, 36, 30)
    fresh.keygen((1, 1))
    f = fresh.encrypt_pixels(_dev(px), (1, 1))
    with pytest.raises(P.CkksError) as ei:
        fresh.mul(f, f)
    assert ei.value.name == "CKKS_ESTATE"
    ctx.stream_sync()


def test_mul_c2_full_size_sampled(c2, W):
    """256x256 pairs at N=8192 in one call (the launch the benchmark times); 48 sampled
    products against the oracle."""
    ctx, o = c2
    a_img, b_img = W.matching_pair(2, 256, 256)
    _say("[gpu] mul C2 65536 pairs")
    a = ctx.encrypt_pixels(_dev(a_img), W.job_seed(2, 0))
    b = ctx.encrypt_pixels(_dev(b_img), W.job_seed(2, 1))
    m = ctx.mul(a, b)
    rng = np.random.default_rng(22)
    idx = np.concatenate([[0, 1, 2047, 2048, 65535], rng.choice(65536, 43, replace=False)])
    import torch

    torch.cuda.synchronize()
    for i in idx:
        i = int(i)
        A = a[i:i + 1].to_numpy().reshape(-1)
        B = b[i:i + 1].to_numpy().reshape(-1)
        G = m[i:i + 1].to_numpy().reshape(-1)
        assert np.array_equal(G, o.mul(A, B)), i
    dec = ctx.decrypt_pixels(ctx.rescale(m)).cpu().numpy()
    want = a_img.reshape(-1).astype(np.float64) * b_img.reshape(-1)
    assert np.max(np.abs(dec - want)) < PROD_TOL


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_image_matching_l1(request, W, which):
    """Squared differences under encryption, decrypted, square-rooted and summed by
    the client: the L1 distance of the two images exactly (Sec. 4.4.3)."""
    ctx, o = request.getfixturevalue(which)
    H, Wd = (32, 32) if which == "c1" else (96, 80)
    a_img, b_img = W.matching_pair(31, H, Wd)
    _say("[gpu] image match %s %dx%d" % (which, H, Wd))
    a = ctx.encrypt_pixels(_dev(a_img), (31, 1))
    b = ctx.encrypt_pixels(_dev(b_img), (31, 2))
    d = ctx.sub(a, b)
    sq = ctx.rescale(ctx.mul(d, d))
    dec = ctx.decrypt_pixels(sq).cpu().numpy()
    diff = a_img.astype(np.int64).reshape(-1) - b_img.astype(np.int64).reshape(-1)
    assert np.max(np.abs(dec - diff.astype(np.float64) ** 2)) < PROD_TOL
    l1 = np.sqrt(np.rint(dec).clip(0)).sum()
    assert l1 == np.abs(diff).sum()
    # a sampled pixel against the oracle, ciphertext for ciphertext
    k = (H * Wd) // 2 + 3
    A, B = a[k:k + 1].to_numpy().reshape(-1), b[k:k + 1].to_numpy().reshape(-1)
    D = o.sub(A, B)
    ref, _ = o.rescale(o.mul(D, D), level=o.L, scale=a.scale * a.scale)
    assert np.array_equal(sq[k:k + 1].to_numpy().reshape(-1), ref)


def test_watermark_single_ciphertext(c1, W):
    """The watermark adds a plaintext to one pixel's ciphertext only (Sec. 4.4.4)."""
    ctx, o = c1
    img = W.config_image(1)
    px = img.reshape(-1)
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    before = _np(cts)
    y, x = 13, 21
    k = y * img.shape[1] + x
    ctx.add_const(cts[k:k + 1], 100.0)
    after = _np(cts)
    changed = np.nonzero(np.any(after != before, axis=1))[0]
    assert changed.tolist() == [k]
    assert np.array_equal(after[k], o.add_const(before[k], 100.0))
    dec = ctx.decrypt_pixels(cts).cpu().numpy()
    want = px.astype(np.float64)
    want[k] += 100.0
    assert np.max(np.abs(dec - want)) < 1e-4


def test_autotune_times_the_product(c1, W):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:16]
    cts = ctx.encrypt_pixels(_dev(px), (9, 9))
    before = _np(ctx.mul(cts[0:8], cts[8:16]))
    _say("[gpu] autotune with key-switching keys")
    rep = ctx.autotune(256)
    assert rep["mul_width"] in (8, 16, 32)
    assert all(np.isfinite(v) and v > 0 for v in rep["mul_ms"].values())
    after = _np(ctx.mul(cts[0:8], cts[8:16]))
    assert np.array_equal(before, after)
    for w in (8, 16, 32):
        ctx.set_ntt_width(w)
        assert np.array_equal(_np(ctx.mul(cts[0:8], cts[8:16])), before), w
