"""GPU tests of the C ABI's safety rules, with oracle parity at the corners of the
operations:

* decryption of values whose coefficients pass q_0/2 (the two-limb CRT lift), compared
  with the oracle's all-limb CRT decryption, and the level-1 (limb 0 only) case;
* replacing the keys invalidates key-switching keys, caches, batch plans and servers;
* output buffers that are too small are refused before any work is enqueued;
* caches built by the oracle and imported through the ABI encrypt bit-exactly;
* the non-blocking stream status;
* the mean filter at every supported window (1, 3, 5, 7) and at input levels 2..8,
  residue by residue against the oracle;
* the relinearized product at level 1.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def c1(P, oracle_mod, W):
    _say("[gpu] api context C1 (N=4096, 3x36-bit)")
    ctx = P.Context(12, 3, 36, 30)
    o = oracle_mod.Oracle(12, 3, 36, 30)
    ctx.keygen(W.keygen_seed(1))
    o.keygen(W.keygen_seed(1))
    return ctx, o


def _dev(px):
    import torch

    return torch.from_numpy(np.ascontiguousarray(px, dtype=np.uint8).reshape(-1)).cuda()


def _np(cts):
    import torch

    torch.cuda.synchronize()
    return cts.to_numpy().reshape(cts.count, -1)


# ---------------------------------------------------------------------------
# decryption past the limb-0 bound (Sec. 2.2.2)
# ---------------------------------------------------------------------------
def test_decrypt_sum_past_limb0_bound(c1):
    ctx, o = c1
    n = 300
    px = np.full(n, 255, dtype=np.uint8)
    _say("[gpu] decrypt: sum of %d pixels of 255 at N=4096, scale 2^30" % n)
    cts = ctx.encrypt_pixels(_dev(px), (9, 9))
    acc = ctx.empty(1)
    acc.data.copy_(cts.data[0:1])
    for i in range(1, n):
        ctx.add(acc, cts[i:i + 1], out=acc)
    got = _np(acc)[0]
    ref = o.encrypt_batch(px, (9, 9))
    ref_acc = ref[0]
    for i in range(1, n):
        ref_acc = o.add(ref_acc, ref[i])
    assert np.array_equal(got, ref_acc)
    with pytest.raises(ArithmeticError):
        o.decrypt(ref_acc)  # limb 0 alone no longer decodes this ciphertext
    dec = float(ctx.decrypt_pixels(acc).cpu().numpy()[0])
    exact = o.decrypt_exact(ref_acc)
    assert abs(dec - exact) < 1e-6, (dec, exact)
    assert abs(dec - n * 255) < 3e-3
    # one pixel times 300: the same value, one ciphertext
    m = ctx.mul_const(cts[0:1], 300)
    mref, _ = o.mul_const(ref[0], 300)
    assert np.array_equal(_np(m)[0], mref)
    dm = float(ctx.decrypt_pixels(m).cpu().numpy()[0])
    assert abs(dm - o.decrypt_exact(mref)) < 1e-6
    assert abs(dm - 76500) < 3e-2
    # at level 2 (after a fractional constant and a rescale) the lift uses limbs 0 and 1
    f = ctx.mul_const(acc, 0.999)
    r = ctx.rescale(f)
    fref, sc = o.mul_const(ref_acc, 0.999)
    rref, sc2 = o.rescale(fref, level=3, scale=sc)
    assert np.array_equal(_np(r)[0], rref) and r.scale == sc2
    dr = float(ctx.decrypt_pixels(r).cpu().numpy()[0])
    assert abs(dr - o.decrypt_exact(rref, level=2, scale=sc2)) < 1e-6
    assert abs(dr - 0.999 * n * 255) < 0.1


def test_decrypt_level1_limb0(c1, W):
    ctx, o = c1
    px = W.config_image(1).reshape(-1)[:32]
    a = ctx.encrypt_pixels(_dev(px), (3, 1))
    r1 = ctx.rescale(ctx.mul_const(a, 0.5))
    r2 = ctx.rescale(ctx.mul_const(r1, 0.5))
    assert r2.level == 1
    dec = ctx.decrypt_pixels(r2).cpu().numpy()
    g = _np(r2)
    for i in range(0, 32, 5):
        assert abs(dec[i] - o.decrypt(g[i], level=1, scale=r2.scale)) < 1e-9
    assert np.max(np.abs(dec - px / 4.0)) < 1e-2


# ---------------------------------------------------------------------------
# key replacement
# ---------------------------------------------------------------------------
def test_key_replacement_invalidates(P, W):
    import torch

    _say("[gpu] key replacement")
    ctx = P.Context(12, 3, 36, 30)
    ctx.keygen((1, 1))
    ctx.relin_keygen((2, 2))
    cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=2, seed=(3, 3))
    plan = P.BatchPlan(ctx, cache, 64)
    px = _dev(np.arange(16))
    a = ctx.encrypt_pixels(px, (4, 4))
    ctx.mul(a, a)  # works under the first keys
    torch.cuda.synchronize()
    ctx.keygen((5, 5))  # new keys
    for call in (lambda: ctx.mul(a, a), lambda: ctx.encrypt_cached(cache, px, (4, 4)),
                 lambda: plan.run(px, [16], [0.0], (1, 1)), lambda: P.BatchPlan(ctx, cache, 64),
                 lambda: P.Server(ctx, 1 << 30, filter_k=3, cache=cache),
                 lambda: ctx.image_pipeline(px, 4, 4, (1, 1), 3, 2, 1, cache=cache)):
        with pytest.raises(P.CkksError) as e:
            call()
        assert e.value.name == "CKKS_ESTATE"
    # fresh key-switching keys and a fresh cache work again and decrypt under the new keys
    ctx.relin_keygen((2, 2))
    b = ctx.encrypt_pixels(px, (4, 4))
    sq = ctx.rescale(ctx.mul(b, b))
    dec = ctx.decrypt_pixels(sq).cpu().numpy()
    assert np.max(np.abs(dec - np.arange(16) ** 2)) < 0.05
    cache2 = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=2, seed=(3, 3))
    c = ctx.encrypt_cached(cache2, px, (4, 4))
    assert np.max(np.abs(ctx.decrypt_pixels(c).cpu().numpy() - np.arange(16))) < 2e-4
    plan.close()
    cache.close()
    cache2.close()
    ctx.close()


# ---------------------------------------------------------------------------
# output capacity
# ---------------------------------------------------------------------------
def test_output_capacity_checked(P, c1, W):
    ctx, o = c1
    px = _dev(np.arange(8))
    a = ctx.encrypt_pixels(px, (1, 1))
    small = ctx.empty(7)
    for call in (lambda: ctx.encrypt_pixels(px, (1, 1), out=small), lambda: ctx.add(a, a, out=small),
                 lambda: ctx.sub(a, a, out=small), lambda: ctx.mul_const(a, 3.0, out=small),
                 lambda: ctx.rescale(a, out=ctx.empty(7, 2)), lambda: ctx.mean_filter(a, 2, 4, 3, out=ctx.empty(7, 2))):
        with pytest.raises(P.CkksError) as e:
            call()
        assert e.value.name == "CKKS_EINVAL"
    # a lower-level output of the right count is too small for a full-level result
    with pytest.raises(P.CkksError) as e:
        ctx.add(a, a, out=ctx.empty(8, 2))
    assert e.value.name == "CKKS_EINVAL"
    # a higher-level buffer holds a lower-level result
    big = ctx.empty(8, 3)
    r = ctx.rescale(a, out=big)
    assert r.level == 2


# ---------------------------------------------------------------------------
# cache import (Sec. 3.2: full caching prepared offline)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["radix16", "radix4", "topk", "full"])
def test_cache_import_encrypts_bitexact(P, c1, W, kind):
    ctx, o = c1
    img = W.zipf_image(61, 16, 16)
    px = img.reshape(-1)
    cseed, job = (0xCAC4E, 9), (7, 3)
    _say("[gpu] cache import %s" % kind)
    if kind.startswith("radix"):
        base, digits = (16, 2) if kind == "radix16" else (4, 4)
        ent = o.radix_entries(base, digits, cseed)
        vals = [0] + [base**i for i in range(digits)]
        cache = ctx.cache_import(P.CKKS_CACHE_RADIX, vals, ent, base=base, digits=digits)
        ref = [o.radix_encrypt(ent, base, digits, int(p), job, 50 + t) for t, p in enumerate(px)]
    else:
        npool = 5
        pool = np.stack([o.pool_entry(u, cseed) for u in range(npool)])
        if kind == "topk":
            vals = o.topk(o.histogram(px), 12)
            cache = None
        else:
            vals = list(range(256))
        ent = np.stack([o.value_entry(v, cseed) for v in vals])
        kd = P.CKKS_CACHE_VALUE_TOPK if kind == "topk" else P.CKKS_CACHE_VALUE_FULL
        cache = ctx.cache_import(kd, vals, ent, pool, topk=12 if kind == "topk" else 0, zero_pool=npool)
        slot = {int(v): i for i, v in enumerate(vals)}
        ref = [o.value_encrypt(ent[slot[int(p)]] if int(p) in slot else None, pool, npool, int(p), job, 50 + t)
               for t, p in enumerate(px)]
    ev, ee, ep = cache.export(0 if kind.startswith("radix") else 5)
    assert list(ev) == list(vals) and np.array_equal(ee, np.asarray(ent).reshape(len(vals), -1))
    got = _np(ctx.encrypt_cached(cache, _dev(px), job, first_index=50))
    bad = [t for t in range(px.size) if not np.array_equal(got[t], ref[t])]
    assert not bad, bad[:10]
    cache.close()


def test_cache_import_rejects_bad_input(P, c1):
    ctx, o = c1
    S = 2 * 3 * 4096
    ent = np.zeros((3, S), dtype=np.uint64)
    with pytest.raises(P.CkksError) as e:  # radix values must be 0, 1, base
        ctx.cache_import(P.CKKS_CACHE_RADIX, [0, 1, 15], ent, base=16, digits=2)
    assert e.value.name == "CKKS_ECACHE"
    with pytest.raises(P.CkksError) as e:  # one digit gives no randomness
        ctx.cache_import(P.CKKS_CACHE_RADIX, [0, 1], ent[:2], base=256, digits=1)
    assert e.value.name == "CKKS_ECACHE"
    bad = ent.copy()
    bad[1, 5] = o.q[0]  # not canonical in limb 0
    with pytest.raises(P.CkksError) as e:
        ctx.cache_import(P.CKKS_CACHE_RADIX, [0, 1, 16], bad, base=16, digits=2)
    assert e.value.name == "CKKS_EINVAL"
    with pytest.raises(P.CkksError) as e:  # repeated value
        ctx.cache_import(P.CKKS_CACHE_VALUE_TOPK, [3, 3], ent[:2], np.zeros((1, S), np.uint64), topk=4, zero_pool=1)
    assert e.value.name == "CKKS_ECACHE"
    with pytest.raises(P.CkksError) as e:  # radix base 256, one digit, through the build too
        ctx.cache_build(P.CKKS_CACHE_RADIX, base=256, digits=1, seed=(1, 1))
    assert e.value.name == "CKKS_ECACHE"


# ---------------------------------------------------------------------------
# stream status
# ---------------------------------------------------------------------------
def test_stream_status(P, c1, W):
    import torch

    ctx, o = c1
    s = torch.cuda.Stream()
    px = _dev(np.zeros(4096, dtype=np.uint8))
    out = ctx.empty(4096)
    ctx.encrypt_pixels(px, (1, 1), out=out, stream=s)
    first = ctx.stream_done(s)  # either answer is valid while the launch may still run
    assert first in (True, False)
    s.synchronize()
    assert ctx.stream_done(s) is True
    ctx.stream_sync(s)


# ---------------------------------------------------------------------------
# mean filter at every window and level (Sec. 4.4.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,k", [(2, 3), (2, 7), (3, 7), (5, 5), (6, 3), (7, 7), (8, 1), (8, 7)])
def test_mean_filter_windows_and_levels(P, oracle_mod, W, L, k):
    _say("[gpu] mean filter L=%d k=%d" % (L, k))
    ctx = P.Context(12, L, 36, 30)
    o = oracle_mod.Oracle(12, L, 36, 30)
    ctx.keygen((L, k))
    o.keygen((L, k))
    img = W.uniform_image(100 + L, 9, 11)
    H, Wd = img.shape
    cts = ctx.encrypt_pixels(_dev(img), (k, L))
    out = ctx.mean_filter(cts, H, Wd, k)
    assert out.level == L - 1
    g, allc = _np(out), _np(cts)
    assert np.array_equal(allc, o.encrypt_batch(img.reshape(-1), (k, L)))
    for y in range(H):
        for x in range(Wd):
            ref, sc = o.mean_filter_pixel(allc, H, Wd, k, y, x)
            assert np.array_equal(g[y * Wd + x], ref), (y, x)
            assert out.scale == sc
    dec = ctx.decrypt_pixels(out).cpu().numpy()
    for t in range(0, H * Wd, 7):
        assert abs(dec[t] - o.decrypt(g[t], level=L - 1, scale=out.scale)) < 1e-9
    R = k // 2
    pad = np.pad(img.astype(np.float64), R, mode="edge")
    box = sum(pad[dy:dy + H, dx:dx + Wd] for dy in range(k) for dx in range(k)) / (k * k)
    assert np.max(np.abs(dec.reshape(H, Wd) - box)) < 1e-3
    ctx.close()


# ---------------------------------------------------------------------------
# relinearized product at level 1 (Sec. 2.2.3)
# ---------------------------------------------------------------------------
def test_mul_level1_bitexact(P, oracle_mod, W):
    _say("[gpu] product at level 1")
    ctx = P.Context(12, 3, 36, 30)
    o = oracle_mod.Oracle(12, 3, 36, 30)
    ctx.keygen((11, 1))
    o.keygen((11, 1))
    ctx.relin_keygen((12, 1))
    o.relin_keygen((12, 1))
    px = W.uniform_image(7, 4, 8).reshape(-1)
    a = ctx.encrypt_pixels(_dev(px), (1, 2))
    b = ctx.encrypt_pixels(_dev(px[::-1].copy()), (1, 3))
    a1 = ctx.rescale(ctx.rescale(a))
    b1 = ctx.rescale(ctx.rescale(b))
    assert a1.level == 1
    prod = ctx.mul(a1, b1)
    g, A, B = _np(prod), _np(a1), _np(b1)
    for i in range(px.size):
        assert np.array_equal(g[i], o.mul(A[i], B[i], level=1)), i
    ctx.close()


# ---------------------------------------------------------------------------
# per-call scratch: calls queued back to back on one stream do not wait on the host, and
# their results equal the same calls run one at a time (also across two streams)
# ---------------------------------------------------------------------------
def test_queued_cached_calls_do_not_block(P, c1, W):
    import time

    import torch

    ctx, o = c1
    _say("[gpu] queued cached encryptions")
    big = _dev(W.uniform_image(71, 256, 256))  # 65,536 pixels: several ms of plain encryption
    px = _dev(W.zipf_image(72, 64, 64))
    radix = ctx.cache_build(P.CKKS_CACHE_RADIX, base=16, digits=2, seed=(7, 7))
    value = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=32, zero_pool=8, scan_px=px, seed=(7, 7))
    refs = []
    for cache, seed in ((radix, (1, 1)), (value, (1, 2)), (radix, (1, 3))):
        refs.append(_np(ctx.encrypt_cached(cache, px, seed)).copy())
    st, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    hold = ctx.empty(big.numel())
    outs = [ctx.empty(px.numel()) for _ in range(3)]
    for cache in (radix, value):  # the stream's scratch reaches its size before the timed calls
        ctx.encrypt_cached(cache, px, (5, 5), out=outs[0], stream=st)
    torch.cuda.synchronize()
    ctx.encrypt_pixels(big, (9, 9), out=hold, stream=st)  # keeps the stream busy
    host_ms = []
    for out, (cache, seed) in zip(outs[:2], ((radix, (1, 1)), (value, (1, 2)))):
        t0 = time.perf_counter()
        ctx.encrypt_cached(cache, px, seed, out=out, stream=st)
        host_ms.append((time.perf_counter() - t0) * 1e3)
    ctx.encrypt_cached(radix, px, (1, 3), out=outs[2], stream=st2)
    torch.cuda.synchronize()
    for got, ref in zip(outs, refs):
        assert np.array_equal(_np(got), ref)
    # the second call reuses the stream's scratch while the first is still queued: it must
    # return without waiting for the device (the plain encryption alone takes ~10 ms)
    assert host_ms[1] < 5.0, host_ms
    radix.close()
    value.close()


def test_scratch_of_many_streams(P, c1, W):
    """Cached encryptions and products on more streams than the context keeps scratch
    buffers for (16): each further stream takes over the least recently used buffer, and
    every result stays bit-exact, also with the calls of all streams queued at once."""
    import torch

    ctx, o = c1
    _say("[gpu] cached encryption and products on 24 streams")
    px = _dev(W.zipf_image(73, 32, 32))
    value = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=16, zero_pool=8, scan_px=px, seed=(3, 3))
    refs = [_np(ctx.encrypt_cached(value, px, (2, k))).copy() for k in range(24)]
    streams = [torch.cuda.Stream() for _ in range(24)]
    outs = [ctx.empty(px.numel()) for _ in range(24)]
    for rnd in range(2):  # the second round finds every buffer taken over by another stream
        for k, st in enumerate(streams):
            ctx.encrypt_cached(value, px, (2, k), out=outs[k], stream=st)
        torch.cuda.synchronize()
        for k in range(24):
            assert np.array_equal(_np(outs[k]), refs[k]), (rnd, k)
    ctx.relin_keygen((5, 6))
    a = ctx.encrypt_pixels(px, (4, 1))
    b = ctx.encrypt_pixels(px, (4, 2))
    ref = _np(ctx.mul(a, b)).copy()
    prods = [ctx.empty(px.numel()) for _ in range(20)]
    for k in range(20):
        with torch.cuda.stream(streams[k]):
            ctx.mul(a, b, out=prods[k], stream=streams[k])
    torch.cuda.synchronize()
    for k in range(20):
        assert np.array_equal(_np(prods[k]), ref), k
    value.close()
