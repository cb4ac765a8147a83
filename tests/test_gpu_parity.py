"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Ciphertexts are compared residue by residue (bit-exact); decrypted pixels to 1e-4
pixel units (the tolerance of the plain-encryption target; the GPU and oracle decode
the same integers, so the observed difference is ~1e-12).  Small configurations are
compared in full; the 256x256 N=8192 workload is run at full size, in the launch
configuration the benchmark times, and compared on sampled ciphertexts that the
oracle computes one by one.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEC_TOL = 1e-4


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


def _make(P, oracle_mod, W, cfg, sigma=3.2, seed=None):
    c = W.CONFIGS[cfg]
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, sigma=sigma)
    o = oracle_mod.Oracle(c.log_n, c.num_primes, c.prime_bits, c.log_scale, sigma=sigma)
    seed = W.keygen_seed(cfg) if seed is None else seed
    ctx.keygen(seed)
    o.keygen(seed)
    return ctx, o


@pytest.fixture(scope="module")
def c1(P, oracle_mod, W):
    _say("[gpu] context C1 (N=4096, 3x36-bit)")
    return _make(P, oracle_mod, W, 1)


@pytest.fixture(scope="module")
def c2(P, oracle_mod, W):
    _say("[gpu] context C2 (N=8192, 4x50-bit)")
    return _make(P, oracle_mod, W, 2)


def _dev(px):
    import torch

    return torch.from_numpy(np.ascontiguousarray(px, dtype=np.uint8).reshape(-1)).cuda()


def _np(cts):
    import torch

    torch.cuda.synchronize()
    return cts.to_numpy().reshape(cts.count, -1)


# ---------------------------------------------------------------------------
# keys
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["c1", "c2"])
def test_keygen_bitexact(request, which):
    ctx, o = request.getfixturevalue(which)
    s, pk = ctx.keys_export()
    assert np.array_equal(s, o.s)
    assert np.array_equal(pk, o.pk)


def test_keys_import(P, oracle_mod, W, c1):
    _, o0 = c1
    ctx = P.Context(12, 3, 36, 30)
    o = oracle_mod.Oracle(12, 3, 36, 30)
    s, pk = o.keygen((777, 888))
    ctx.keys_import(s, pk)
    px = W.uniform_image(11, 4, 16).reshape(-1)
    got = _np(ctx.encrypt_pixels(_dev(px), (5, 6), first_index=40))
    assert np.array_equal(got, o.encrypt_batch(px, (5, 6), first_index=40))


# ---------------------------------------------------------------------------
# plain encryption and decryption
# ---------------------------------------------------------------------------
def test_encrypt_c1_full_bitexact(c1, W):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)
    _say("[gpu] encrypt C1 1024 pixels")
    got = _np(ctx.encrypt_pixels(_dev(px), W.job_seed(1)))
    ref = o.encrypt_batch(px, W.job_seed(1))
    assert got.shape == ref.shape
    bad = np.nonzero(np.any(got != ref, axis=1))[0]
    assert bad.size == 0, "mismatching ciphertexts: %s" % bad[:10]


def test_decrypt_c1(c1, W):
    import torch

    ctx, o = c1
    px = W.config_image(1).reshape(-1)
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    got = ctx.decrypt_pixels(cts).cpu().numpy()
    ref = o.decrypt_batch(_np(cts))
    assert np.max(np.abs(got - ref)) < 1e-9
    assert np.max(np.abs(got - px)) < DEC_TOL


def test_batch_index_and_stream_invariance(c1, W):
    import torch

    ctx, o = c1
    px = W.config_image(1).reshape(-1)
    full = _np(ctx.encrypt_pixels(_dev(px), W.job_seed(1)))
    part = _np(ctx.encrypt_pixels(_dev(px[100:357]), W.job_seed(1), first_index=100))
    assert np.array_equal(part, full[100:357])
    one = _np(ctx.encrypt_pixels(_dev(px[5:6]), W.job_seed(1), first_index=5))
    assert np.array_equal(one[0], full[5])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = ctx.encrypt_pixels(_dev(px[:64]), W.job_seed(1), stream=s)
    s.synchronize()
    assert np.array_equal(_np(out), full[:64])
    # empty input is a no-op
    empty = ctx.empty(0)
    ctx.encrypt_pixels(_dev(px[:0]), W.job_seed(1), out=empty)
    assert empty.count == 0


@pytest.mark.parametrize("cfg", [1, 2])
def test_ntt_width_invariance(P, oracle_mod, W, cfg):
    # every thread shape of the NTT kernels gives the same ciphertexts, keys and decryptions
    c = W.CONFIGS[cfg]
    px = W.config_image(cfg).reshape(-1)[:96]
    outs, decs, keys = [], [], []
    for width in (8, 16, 32):
        ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale)
        ctx.set_ntt_width(width)
        assert ctx.ntt_width() == width
        ctx.keygen(W.keygen_seed(cfg))
        keys.append(ctx.keys_export())
        cts = ctx.encrypt_pixels(_dev(px), W.job_seed(cfg), first_index=7)
        outs.append(_np(cts))
        decs.append(ctx.decrypt_pixels(cts).cpu().numpy())
    for i in (1, 2):
        assert np.array_equal(keys[0][0], keys[i][0]) and np.array_equal(keys[0][1], keys[i][1])
        assert np.array_equal(outs[0], outs[i])
        # the decoded value is a floating-point sum whose order follows the workgroup shape
        assert np.max(np.abs(decs[0] - decs[i])) < 1e-9
    o = oracle_mod.Oracle(c.log_n, c.num_primes, c.prime_bits, c.log_scale)
    o.keygen(W.keygen_seed(cfg))
    for t in (0, 50, 95):
        assert np.array_equal(outs[0][t], o.encrypt(int(px[t]), W.job_seed(cfg), 7 + t))
    with pytest.raises(P.CkksError):
        ctx.set_ntt_width(64)


def test_noiseless_roundtrip(P, oracle_mod, W):
    ctx, o = _make(P, oracle_mod, W, 1, sigma=0.0, seed=(1, 2))
    px = np.array([0, 1, 17, 128, 254, 255], dtype=np.uint8)
    cts = ctx.encrypt_pixels(_dev(px), (3, 4))
    got = _np(cts)
    assert np.array_equal(got, o.encrypt_batch(px, (3, 4)))
    dec = ctx.decrypt_pixels(cts).cpu().numpy()
    assert np.max(np.abs(dec - px)) < 1e-6


@pytest.mark.slow
def test_encrypt_c2_full_size_sampled(c2, W):
    import torch

    ctx, o = c2
    px = W.config_image(2).reshape(-1)
    n = px.size
    _say("[gpu] encrypt C2 65536 pixels")
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(2))
    dec = ctx.decrypt_pixels(cts).cpu().numpy()
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    idx = sorted(set([0, 1, 255, 256, n // 2, n - 1] + [int(i) for i in rng.integers(0, n, 14)]))
    for t in idx:
        got = cts.data[t].cpu().numpy().view(np.uint64).reshape(-1)
        ref = o.encrypt(int(px[t]), W.job_seed(2), t)
        assert np.array_equal(got, ref), t
        assert abs(dec[t] - o.decrypt(ref)) < 1e-9
    assert np.max(np.abs(dec - px)) < DEC_TOL


# ---------------------------------------------------------------------------
# homomorphic operations
# ---------------------------------------------------------------------------
def test_add_sub_mul_const_rescale_c1(c1, W):
    import torch

    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:16]
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    a, b = cts[0:8], cts[8:16]
    A, B = _np(a), _np(b)
    got = _np(ctx.add(a, b))
    assert all(np.array_equal(got[i], o.add(A[i], B[i])) for i in range(8))
    got = _np(ctx.sub(a, b))
    assert all(np.array_equal(got[i], o.sub(A[i], B[i])) for i in range(8))
    for c in (3.0, -2.0, 1.0 / 9.0, 0.3):
        r = ctx.mul_const(a, c)
        g = _np(r)
        for i in range(8):
            ref, sc = o.mul_const(A[i], c)
            assert np.array_equal(g[i], ref), c
            assert r.scale == sc
    m = ctx.mul_const(a, 1.0 / 9.0)
    r = ctx.rescale(m)
    g = _np(r)
    for i in range(8):
        mref, sc = o.mul_const(A[i], 1.0 / 9.0)
        ref, sc2 = o.rescale(mref, level=3, scale=sc)
        assert np.array_equal(g[i], ref)
        assert r.scale == sc2 == o.scale
    dec = ctx.decrypt_pixels(r).cpu().numpy()
    assert np.max(np.abs(dec - px[:8] / 9.0)) < 1e-3
    # in-place add aliasing the first operand
    a2 = ctx.encrypt_pixels(_dev(px[:8]), W.job_seed(1))
    ctx.add(a2, b, out=a2)
    assert np.array_equal(_np(a2), _np(ctx.add(a, b)))


def test_add_const_c1(c1, W):
    import torch

    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:8]
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    A = _np(cts)
    ctx.add_const(cts, 50.0)
    g = _np(cts)
    for i in range(8):
        assert np.array_equal(g[i], o.add_const(A[i], 50.0))
    bvals = np.array([-40, -3.5, 0, 1, 7, 12.25, 39, 40], dtype=np.float64)
    cts2 = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    ctx.add_const(cts2, per_ct=torch.from_numpy(bvals).cuda())
    g2 = _np(cts2)
    for i in range(8):
        assert np.array_equal(g2[i], o.add_const(A[i], float(bvals[i])))
    dec = ctx.decrypt_pixels(cts2).cpu().numpy()
    assert np.max(np.abs(dec - (px + bvals))) < DEC_TOL


def test_add_const_large_scale(c1, W):
    # after a fractional mul_const the scale is Delta * q: the encoded constant exceeds 2^52
    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:4]
    cts = ctx.encrypt_pixels(_dev(px), W.job_seed(1))
    m = ctx.mul_const(cts, 0.5)
    M = _np(m)
    ctx.add_const(m, 10.0)
    g = _np(m)
    for i in range(4):
        assert np.array_equal(g[i], o.add_const(M[i], 10.0, level=3, scale=m.scale))


# ---------------------------------------------------------------------------
# mean filter
# ---------------------------------------------------------------------------
def _box(img, k):
    R = k // 2
    H, Wd = img.shape
    pad = np.pad(img.astype(np.float64), R, mode="edge")
    out = np.zeros((H, Wd))
    for dy in range(k):
        for dx in range(k):
            out += pad[dy:dy + H, dx:dx + Wd]
    return out / (k * k)


@pytest.mark.parametrize("k", [3, 5, 1])
def test_mean_filter_c1(c1, W, k):
    ctx, o = c1
    img = W.config_image(1)
    H, Wd = img.shape
    cts = ctx.encrypt_pixels(_dev(img), W.job_seed(1))
    _say("[gpu] mean filter C1 k=%d" % k)
    out = ctx.mean_filter(cts, H, Wd, k)
    assert out.level == 2
    g = _np(out)
    allc = _np(cts)
    rng = np.random.default_rng(k)
    pts = {(0, 0), (0, Wd - 1), (H - 1, 0), (H - 1, Wd - 1), (1, 1), (H // 2, Wd // 2)}
    pts |= {(int(y), int(x)) for y, x in zip(rng.integers(0, H, 40), rng.integers(0, Wd, 40))}
    for (y, x) in sorted(pts):
        ref, sc = o.mean_filter_pixel(allc, H, Wd, k, y, x)
        assert np.array_equal(g[y * Wd + x], ref), (y, x)
        assert out.scale == sc
    dec = ctx.decrypt_pixels(out).cpu().numpy().reshape(H, Wd)
    assert np.max(np.abs(dec - _box(img, k))) < 1e-3


def test_mean_filter_ragged_shape(c1, W):
    ctx, o = c1
    img = W.uniform_image(21, 7, 13)
    H, Wd = img.shape
    cts = ctx.encrypt_pixels(_dev(img), W.job_seed(1))
    out = ctx.mean_filter(cts, H, Wd, 3)
    g, allc = _np(out), _np(cts)
    for y in range(H):
        for x in (0, 5, Wd - 1):
            ref, _ = o.mean_filter_pixel(allc, H, Wd, 3, y, x)
            assert np.array_equal(g[y * Wd + x], ref), (y, x)
    dec = ctx.decrypt_pixels(out).cpu().numpy().reshape(H, Wd)
    assert np.max(np.abs(dec - _box(img, 3))) < 1e-3


@pytest.mark.parametrize("H,Wd,k", [(1, 1, 3), (1, 37, 3), (37, 1, 5), (3, 37, 5), (2, 17, 3), (5, 33, 7)])
def test_mean_filter_degenerate_and_multi_group_shapes(c1, W, H, Wd, k):
    """Single rows and columns (every window clamped), and widths past one workgroup's 16
    output columns with a ragged last group: every output equals the oracle's."""
    ctx, o = c1
    _say("[gpu] mean filter %dx%d k=%d" % (H, Wd, k))
    img = W.uniform_image(40 + H + Wd, H, Wd)
    cts = ctx.encrypt_pixels(_dev(img), W.job_seed(1))
    out = ctx.mean_filter(cts, H, Wd, k)
    g, allc = _np(out), _np(cts)
    for y in range(H):
        for x in range(Wd):
            ref, _ = o.mean_filter_pixel(allc, H, Wd, k, y, x)
            assert np.array_equal(g[y * Wd + x], ref), (y, x)
    dec = ctx.decrypt_pixels(out).cpu().numpy().reshape(H, Wd)
    assert np.max(np.abs(dec - _box(img, k))) < 1e-3


@pytest.mark.slow
def test_mean_filter_c2_full_size_sampled(c2, W):
    ctx, o = c2
    img = W.config_image(2)
    H, Wd = img.shape
    k = 3
    cts = ctx.encrypt_pixels(_dev(img), W.job_seed(2))
    _say("[gpu] mean filter C2 256x256")
    out = ctx.mean_filter(cts, H, Wd, k)
    dec = ctx.decrypt_pixels(out).cpu().numpy().reshape(H, Wd)
    assert np.max(np.abs(dec - _box(img, k))) < 1e-3
    rng = np.random.default_rng(22)
    pts = [(0, 0), (H - 1, Wd - 1), (0, 100), (128, 0)] + [(int(a), int(b)) for a, b in
                                                            zip(rng.integers(0, H, 4), rng.integers(0, Wd, 4))]
    R = k // 2
    for (y, x) in pts:
        # the k x k window around (y, x) with clamped borders, encrypted by the oracle
        patch = []
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                yy, xx = min(max(y + dy, 0), H - 1), min(max(x + dx, 0), Wd - 1)
                t = yy * Wd + xx
                patch.append(o.encrypt(int(img[yy, xx]), W.job_seed(2), t))
        ref, _ = o.mean_filter_pixel(np.stack(patch), k, k, k, R, R)
        got = out.data[y * Wd + x].cpu().numpy().view(np.uint64).reshape(-1)
        assert np.array_equal(got, ref), (y, x)


# ---------------------------------------------------------------------------
# caches (Sec. 3.2) and their randomness (Sec. 3.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("base,digits", [(16, 2), (2, 8), (4, 4)])
def test_radix_cache_c1(P, c1, W, base, digits):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)
    cache = ctx.cache_build(P.CKKS_CACHE_RADIX, base=base, digits=digits, seed=W.cache_seed(1))
    vals, ent, _ = cache.export()
    assert list(vals) == [0] + [base**i for i in range(digits)]
    ref_ent = o.radix_entries(base, digits, W.cache_seed(1))
    assert np.array_equal(ent, ref_ent)
    cts = ctx.encrypt_cached(cache, _dev(px), W.job_seed(1), first_index=0)
    g = _np(cts)
    sample = range(0, px.size, 1 if base == 16 else 7)
    for t in sample:
        ref = o.radix_encrypt(ref_ent, base, digits, int(px[t]), W.job_seed(1), t)
        assert np.array_equal(g[t], ref), t
    dec = ctx.decrypt_pixels(cts).cpu().numpy()
    assert np.max(np.abs(dec - px)) < 3e-3


@pytest.mark.parametrize("kind,topk,pool", [("topk", 16, 8), ("topk", 300, 4), ("full", 0, 4)])
def test_value_cache_c1(P, oracle_mod, c1, W, kind, topk, pool):
    ctx, o = c1
    img = W.zipf_image(31, 32, 32)
    px = img.reshape(-1)
    seed = W.cache_seed(1)
    if kind == "topk" and topk > 256:
        with pytest.raises(P.CkksError):
            ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=topk, zero_pool=pool, scan_px=_dev(px), seed=seed)
        return
    if kind == "topk":
        cache = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=topk, zero_pool=pool, scan_px=_dev(px), seed=seed)
        expect_vals = oracle_mod.Oracle.topk(oracle_mod.Oracle.histogram(px), topk)
    else:
        cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=pool, seed=seed)
        expect_vals = list(range(256))
    vals, ent, pl = cache.export(pool)
    assert list(vals) == expect_vals
    for i in sorted(set([0, len(vals) - 1, len(vals) // 2])):
        assert np.array_equal(ent[i], o.value_entry(int(vals[i]), seed))
    for u in range(pool):
        assert np.array_equal(pl[u], o.pool_entry(u, seed))
    job = W.job_seed(1)
    cts = ctx.encrypt_cached(cache, _dev(px), job, first_index=1000)
    g = _np(cts)
    plain = o.encrypt_batch(px, job, first_index=1000)  # what every miss must equal
    slot = {int(v): i for i, v in enumerate(vals)}
    for t in range(px.size):
        p = int(px[t])
        if p in slot:
            ref = o.value_encrypt(ent[slot[p]], pl, pool, p, job, 1000 + t)
        else:
            ref = plain[t]
        assert np.array_equal(g[t], ref), t
    dec = ctx.decrypt_pixels(cts).cpu().numpy()
    assert np.max(np.abs(dec - px)) < 2e-4


@pytest.mark.slow
def test_caches_c2_full_size_sampled(P, c2, W):
    ctx, o = c2
    e = W.CONFIGS[2].extras
    img = W.config_image(2)
    px = img.reshape(-1)
    n = px.size
    seed, job = W.cache_seed(2), W.job_seed(2)
    _say("[gpu] caches C2")
    radix = ctx.cache_build(P.CKKS_CACHE_RADIX, base=e["base"], digits=e["digits"], seed=seed)
    value = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=e["topk"], zero_pool=e["pool"], scan_px=_dev(px), seed=seed)
    vals, _, _ = value.export()
    rng = np.random.default_rng(5)
    idx = sorted(set([0, n - 1] + [int(i) for i in rng.integers(0, n, 10)]))
    rent = o.radix_entries(e["base"], e["digits"], seed)
    cts = ctx.encrypt_cached(radix, _dev(px), job)
    for t in idx:
        got = cts.data[t].cpu().numpy().view(np.uint64).reshape(-1)
        assert np.array_equal(got, o.radix_encrypt(rent, e["base"], e["digits"], int(px[t]), job, t)), t
    cts = ctx.encrypt_cached(value, _dev(px), job)
    dec = ctx.decrypt_pixels(cts).cpu().numpy()
    assert np.max(np.abs(dec - px)) < DEC_TOL
    vset = set(int(v) for v in vals)
    miss_idx = [int(i) for i in np.nonzero(~np.isin(px, list(vset)))[0][:3]]
    for t in idx + miss_idx:
        p = int(px[t])
        got = cts.data[t].cpu().numpy().view(np.uint64).reshape(-1)
        if p in vset:
            u = o.pool_pick(job, t, e["pool"])
            ref = o.add(o.value_entry(p, seed), o.pool_entry(u, seed))
        else:
            ref = o.encrypt(p, job, t)
        assert np.array_equal(got, ref), t


# ---------------------------------------------------------------------------
# argument validation through the C ABI
# ---------------------------------------------------------------------------
def test_error_paths(P, c1, W):
    ctx, o = c1
    fresh = P.Context(12, 3, 36, 30)
    px = _dev(W.config_image(1).reshape(-1)[:4])
    with pytest.raises(P.CkksError) as ei:
        fresh.encrypt_pixels(px, (1, 1))
    assert ei.value.name == "CKKS_ESTATE"
    a = ctx.encrypt_pixels(px, (1, 1))
    r = ctx.rescale(a)
    with pytest.raises(P.CkksError) as ei:
        ctx.add(a, r)
    assert ei.value.name in ("CKKS_ELEVEL", "CKKS_EINVAL")
    m = ctx.mul_const(a, 0.5)
    with pytest.raises(P.CkksError) as ei:
        ctx.add(a, m)
    assert ei.value.name == "CKKS_ESCALE"
    r1 = ctx.rescale(r)
    with pytest.raises(P.CkksError) as ei:
        ctx.rescale(r1)
    assert ei.value.name == "CKKS_ELEVEL"
    with pytest.raises(P.CkksError) as ei:
        ctx.mean_filter(a, 3, 3, 3)
    assert ei.value.name == "CKKS_EINVAL"
    with pytest.raises(P.CkksError) as ei:
        ctx.mean_filter(a, 2, 2, 4)
    assert ei.value.name == "CKKS_EUNSUPPORTED"
    with pytest.raises(P.CkksError) as ei:
        ctx.cache_build(P.CKKS_CACHE_RADIX, base=16, digits=1, seed=(1, 1))
    assert ei.value.name == "CKKS_ECACHE"
    ctx.stream_sync()
