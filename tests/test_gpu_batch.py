"""GPU tests of batched images (flat index space, ring buffer, fused brightness, HIP
graph replay) and of the autotuner.

The batched ciphertexts -- encryption (value cache or plain) with each image's brightness
fused into the gather or the encryption kernel -- are compared residue by residue, on
every limb, with the oracle's encryption (or cached encryption) followed by its add_const,
and the batch's decrypted values with the oracle's decryption of those ciphertexts.  The
decrypted values also equal the unbatched calls (encrypt -> add_const -> decrypt) bit for
bit.  Graph replays are checked one by one against the eager result, with unrelated eager
work and synchronizations between them.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_03568_amd as P
    from paper_2409_03568_amd import workloads as W

    _say("[gpu] batch context N=4096, 3x36-bit")
    ctx = P.Context(12, 3, 36, 30)
    ctx.keygen(W.keygen_seed(3))
    return P, W, ctx


def _images(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, 2)))).astype(int)
    imgs = [rng.integers(0, 256, (h, w, 3), dtype=np.uint8) for h, w in sides]
    b = rng.integers(-40, 41, count).astype(np.float64)
    return imgs, b


def _flat(imgs, b):
    px = np.concatenate([im.reshape(-1) for im in imgs])
    ends = np.cumsum([im.size for im in imgs]).astype(np.uint64)
    per_ct = np.repeat(b, [im.size for im in imgs])
    return px, ends, per_ct


def _direct(P, ctx, cache, px_dev, per_ct, seed, first):
    import torch

    ct = ctx.encrypt_cached(cache, px_dev, seed, first) if cache is not None else ctx.encrypt_pixels(px_dev, seed, first)
    pc = torch.from_numpy(per_ct).cuda()
    ctx.add_const(ct, per_ct=pc)
    out = ctx.decrypt_pixels(ct)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kind,chunk", [("topk", 1000), ("full", 4096), ("plain", 777)])
def test_batch_matches_unbatched(env, kind, chunk):
    import torch

    P, W, ctx = env
    imgs, b = _images(31, 7, 5, 24)
    px, ends, per_ct = _flat(imgs, b)
    _say("[gpu] batch %s chunk %d: %d images, %d ciphertexts" % (kind, chunk, len(imgs), px.size))
    px_dev = torch.from_numpy(px).cuda()
    cache = None
    if kind == "topk":
        cache = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=40, zero_pool=8, scan_px=px_dev, seed=(9, 9))
    elif kind == "full":
        cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=8, seed=(9, 9))
    plan = P.BatchPlan(ctx, cache, chunk)
    seed, first = (3, 17), 1000
    got = plan.run(px_dev, ends, b, seed, first)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref = _direct(P, ctx, cache, px_dev, per_ct, seed, first)
    assert np.array_equal(got, ref)
    assert np.max(np.abs(got - (px.astype(np.float64) + per_ct))) < 1e-3
    plan.close()


@pytest.fixture(scope="module")
def env_o(env, oracle_mod):
    P, W, ctx = env
    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen(W.keygen_seed(3))
    return P, W, ctx, o


@pytest.mark.parametrize("kind,chunk", [("topk", 97), ("full", 128), ("plain", 61)])
def test_batch_ciphertexts_match_oracle(env_o, kind, chunk):
    import torch

    P, W, ctx, o = env_o
    imgs, b = _images(33, 4, 3, 9)
    px, ends, per_ct = _flat(imgs, b)
    n = px.size
    _say("[gpu] batch vs oracle %s chunk %d: %d ciphertexts" % (kind, chunk, n))
    px_dev = torch.from_numpy(px).cuda()
    cseed, npool = (0xCAC4E, 33), 4
    cache, entries, pool = None, {}, None
    if kind != "plain":
        pool = np.stack([o.pool_entry(u, cseed) for u in range(npool)])
        if kind == "topk":
            vals = o.topk(o.histogram(px), 20)
            cache = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=20, zero_pool=npool, scan_px=px_dev, seed=cseed)
        else:
            vals = sorted(set(int(v) for v in px))
            cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=npool, seed=cseed)
        entries = {int(v): o.value_entry(int(v), cseed) for v in vals}
    plan = P.BatchPlan(ctx, cache, chunk)
    seed, first = (3, 19), 500
    cts = ctx.empty(n)
    dec = plan.run(px_dev, ends, b, seed, first, cts_out=cts).cpu().numpy()
    assert cts.level == 3 and cts.scale == ctx.scale
    got = cts.to_numpy().reshape(n, -1)
    plain = o.encrypt_batch(px, seed, first_index=first)
    bad = []
    for t in range(n):
        p = int(px[t])
        base = plain[t] if p not in entries else o.value_encrypt(entries[p], pool, npool, p, seed, first + t)
        ref = o.add_const(base, float(per_ct[t]))
        if not np.array_equal(got[t], ref):
            bad.append(t)
        elif t % 7 == 0:
            assert abs(dec[t] - o.decrypt(ref)) < 1e-9, t
    assert not bad, "ciphertexts differing from the oracle: %s" % bad[:10]
    assert np.max(np.abs(dec - (px.astype(np.float64) + per_ct))) < 1e-3
    plan.close()
    if cache is not None:
        cache.close()


def test_batch_graph_replays(env):
    import torch

    P, W, ctx = env
    imgs, b = _images(32, 5, 6, 20)
    px, ends, per_ct = _flat(imgs, b)
    px_dev = torch.from_numpy(px).cuda()
    cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=4, seed=(5, 5))
    _say("[gpu] batch graph replays: %d ciphertexts" % px.size)
    eager_plan = P.BatchPlan(ctx, cache, 600, use_graph=False)
    eager = eager_plan.run(px_dev, ends, b, (1, 2), 0).cpu().numpy()
    plan = P.BatchPlan(ctx, cache, 600, use_graph=True)
    out = torch.empty(px.size, dtype=torch.float64, device="cuda")
    other = torch.from_numpy(np.arange(300, dtype=np.uint8)).cuda()
    for rep in range(5):
        out.fill_(-1.0)
        plan.run(px_dev, ends, b, (1, 2), 0, out=out)  # rep 0 eager + capture, then replays
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), "replay %d differs" % rep
        ct = ctx.encrypt_pixels(other, (8, 8))  # unrelated eager work between replays
        ctx.decrypt_pixels(ct)
        torch.cuda.synchronize()
    # new arguments: recaptured, still equal to eager
    b2 = b + 1.0
    got = plan.run(px_dev, ends, b2, (1, 2), 0, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), eager_plan.run(px_dev, ends, b2, (1, 2), 0).cpu().numpy())
    plan.close()
    eager_plan.close()


def test_batch_errors(env):
    import torch

    P, W, ctx = env
    plan = P.BatchPlan(ctx, None, 16)
    px = torch.zeros(10, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.CkksError):
        plan.run(px, [4, 9], [0.0, 0.0], (1, 1))  # last end != n
    with pytest.raises(P.CkksError):
        plan.run(px, [6, 4, 10], [0.0, 0.0, 0.0], (1, 1))  # not ascending
    with pytest.raises(P.CkksError):
        plan.run(px, [10], [1e30], (1, 1))  # brightness too large
    plan.close()


def test_autotune_keeps_results(env, oracle_mod):
    import torch

    P, W, ctx = env
    _say("[gpu] autotune")
    px = torch.from_numpy(np.arange(64, dtype=np.uint8)).cuda()
    before = ctx.encrypt_pixels(px, (4, 4)).to_numpy().copy()
    rep = ctx.autotune(512)
    assert rep["encrypt_width"] in (8, 16, 32) and rep["decrypt_width"] in (8, 16, 32)
    assert all(v > 0 for v in rep["encrypt_ms"].values()) and all(v > 0 for v in rep["decrypt_ms"].values())
    after = ctx.encrypt_pixels(px, (4, 4))
    torch.cuda.synchronize()
    assert np.array_equal(after.to_numpy(), before)
    dec = ctx.decrypt_pixels(after).cpu().numpy()
    assert np.max(np.abs(dec - np.arange(64))) < 1e-4
