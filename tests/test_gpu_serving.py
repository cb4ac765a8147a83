"""GPU tests of the serving runtime (continuous batching of encrypt -> filter -> decrypt).

Determinism: every job's decrypted pixels are bit-identical whether it runs alone or
among other jobs admitted around it, and equal to the same pipeline called directly
through the C ABI on one stream.  Parity: sampled outputs of jobs run in the mix equal the
oracle's own encryption (full value cache with its pool) -> filter -> decryption of the
same pixels within 1e-9.  Accuracy: the decrypted filter output matches the plaintext
clamp-edge box filter of the job's pixels.  Admission: the device bytes in use never
exceed the budget and oversized jobs are refused.
"""
import sys
import time

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

    _say("[gpu] serving context N=4096, 3x36-bit, full value cache (pool 16)")
    ctx = P.Context(12, 3, 36, 30)
    ctx.keygen(W.keygen_seed(4))
    cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=16, seed=W.cache_seed(4))
    torch.cuda.synchronize()
    return P, W, ctx, cache


def _box(img, k):
    H, W = img.shape
    R = k // 2
    pad = np.pad(img.astype(np.float64), R, mode="edge")
    return sum(pad[dy:dy + H, dx:dx + W] for dy in range(k) for dx in range(k)) / (k * k)


def _jobs(W, count, seed, lo=6, hi=40):
    gaps, imgs = W.serving_jobs(seed, count, lo, hi)
    return gaps, imgs


def _direct(P, ctx, cache, img, seed, k):
    import torch

    px = torch.from_numpy(img.reshape(-1)).cuda()
    ct = ctx.encrypt_cached(cache, px, seed) if cache is not None else ctx.encrypt_pixels(px, seed)
    if k:
        ct = ctx.mean_filter(ct, img.shape[0], img.shape[1], k)
    out = ctx.decrypt_pixels(ct)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(img.shape)


@pytest.mark.parametrize("use_cache,k", [(True, 3), (False, 5), (True, 0)])
def test_alone_vs_mix(env, use_cache, k):
    P, W, ctx, cache = env
    cache = cache if use_cache else None
    _say("[gpu] serving alone vs mix cache=%s k=%d" % (use_cache, k))
    gaps, imgs = _jobs(W, 14, seed=40 + k)
    seeds = [(4, 1000 + i) for i in range(len(imgs))]
    # the mix: arrivals 0.3 ms apart on average, at most 4 jobs on the device
    budget = 3 * max(P.job_bytes(ctx, *im.shape, k, cache) for im in imgs)
    srv = P.Server(ctx, budget, max_inflight=4, filter_k=k, cache=cache)
    ids = {}
    for g, im, sd in zip(gaps, imgs, seeds):
        time.sleep(g * 3e-4)
        ids[srv.submit(im, sd)] = len(ids)
    srv.drain()
    mix = {ids[r["id"]]: r for r in srv.poll(64)}
    st = srv.stats()
    srv.close()
    assert len(mix) == len(imgs) and all(r["status"] == 0 for r in mix.values())
    assert st["peak_inflight_bytes"] <= budget and st["completed"] == len(imgs)
    # alone: one job at a time through a fresh server
    srv = P.Server(ctx, budget, max_inflight=1, filter_k=k, cache=cache)
    for i, (im, sd) in enumerate(zip(imgs, seeds)):
        srv.submit(im, sd)
        srv.drain()
        (r,) = srv.poll(4)
        assert np.array_equal(r["pixels"], mix[i]["pixels"]), "job %d differs alone vs in the mix" % i
    srv.close()
    for i in (0, len(imgs) // 2, len(imgs) - 1):
        d = _direct(P, ctx, cache, imgs[i], seeds[i], k)
        assert np.array_equal(d, mix[i]["pixels"]), "job %d differs from the direct pipeline" % i
    for i, im in enumerate(imgs):
        ref = _box(im, k) if k else im.astype(np.float64)
        err = np.max(np.abs(mix[i]["pixels"] - ref))
        assert err < 2e-3, (i, err)


def test_admission_budget(env):
    P, W, ctx, cache = env
    _say("[gpu] serving admission budget")
    srv = P.Server(ctx, 1 << 20, max_inflight=2, filter_k=3, cache=cache)
    with pytest.raises(P.CkksError) as e:
        srv.submit(np.zeros((64, 64), np.uint8), (1, 2))
    assert e.value.name == "CKKS_ENOMEM_BUDGET"
    srv.close()
    # budget of one largest job: jobs run one at a time although two slots exist
    gaps, imgs = _jobs(W, 8, seed=77, lo=8, hi=24)
    budget = max(P.job_bytes(ctx, *im.shape, 3, cache) for im in imgs)
    srv = P.Server(ctx, budget, max_inflight=2, filter_k=3, cache=cache)
    for i, im in enumerate(imgs):
        srv.submit(im, (4, 2000 + i))
    srv.drain()
    res = srv.poll(64)
    st = srv.stats()
    srv.close()
    assert len(res) == len(imgs) and all(r["status"] == 0 for r in res)
    assert st["peak_inflight_bytes"] <= budget
    assert [r["id"] for r in sorted(res, key=lambda r: r["t_admit_us"])] == sorted(r["id"] for r in res)
    for r in res:
        assert r["t_submit_us"] <= r["t_admit_us"] <= r["t_done_us"] and r["gpu_ms"] > 0


def test_backfilling_keeps_results(env):
    # a large job that waits for arena space lets small ones start ahead of it (at most
    # max_bypass of them); every job's pixels equal the same job run alone
    P, W, ctx, cache = env
    _say("[gpu] serving backfilling")
    big = W.zipf_image(120, 96, 96)
    small = [W.zipf_image(121 + i, 16, 16) for i in range(6)]
    b_big = P.job_bytes(ctx, 96, 96, 3, cache)
    b_small = P.job_bytes(ctx, 16, 16, 3, cache)
    budget = b_big + 3 * b_small  # the first big job leaves room for small ones, not for a second big
    alone = {}
    srv = P.Server(ctx, budget, max_inflight=1, filter_k=3, cache=cache)
    for i, im in enumerate([big, big] + small):
        srv.submit(im, (6, 4000 + i))
        srv.drain()
        alone[i] = srv.poll(4)[0]["pixels"].copy()
    srv.close()
    srv = P.Server(ctx, budget, max_inflight=4, filter_k=3, cache=cache, max_bypass=2)
    ids = [srv.submit(im, (6, 4000 + i)) for i, im in enumerate([big, big] + small)]
    srv.drain()
    res = {r["id"]: r for r in srv.poll(64)}
    st = srv.stats()
    srv.close()
    assert len(res) == 8 and all(r["status"] == 0 for r in res.values())
    for i, jid in enumerate(ids):
        assert np.array_equal(res[jid]["pixels"], alone[i]), i
    assert st["peak_inflight_bytes"] <= budget
    # the second big job waited for space and was overtaken at most twice
    t2 = res[ids[1]]["t_admit_us"]
    assert sum(1 for j in ids[2:] if res[j]["t_admit_us"] < t2) <= 2
    assert st["backfilled"] <= 2  # only the waiting big job is ever overtaken (small jobs are equal)


def test_jobs_overlap(env):
    # jobs submitted together run side by side: each takes milliseconds on the device,
    # far longer than the submissions, and the budget holds three of them
    P, W, ctx, cache = env
    _say("[gpu] serving overlap")
    imgs = [W.zipf_image(90 + i, 64, 64) for i in range(6)]
    budget = 3 * P.job_bytes(ctx, 64, 64, 3, cache)
    srv = P.Server(ctx, budget, max_inflight=4, filter_k=3, cache=cache)
    for i, im in enumerate(imgs):
        srv.submit(im, (4, 3000 + i))
    srv.drain()
    res = srv.poll(16)
    st = srv.stats()
    srv.close()
    assert len(res) == 6 and all(r["status"] == 0 for r in res)
    assert st["peak_inflight_jobs"] >= 2, st
    assert st["peak_inflight_bytes"] <= budget
    # overlapping jobs were admitted before earlier ones finished
    res.sort(key=lambda r: r["t_admit_us"])
    assert any(res[i + 1]["t_admit_us"] < res[i]["t_done_us"] for i in range(len(res) - 1))


def test_mix_sampled_against_oracle(env, oracle_mod):
    P, W, ctx, cache = env
    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen(W.keygen_seed(4))
    cseed = W.cache_seed(4)
    pool = np.stack([o.pool_entry(u, cseed) for u in range(16)])
    entries = {}
    _say("[gpu] serving mix vs oracle")
    gaps, imgs = _jobs(W, 6, seed=91, lo=5, hi=18)
    k = 3
    budget = 2 * max(P.job_bytes(ctx, *im.shape, k, cache) for im in imgs)
    srv = P.Server(ctx, budget, max_inflight=3, filter_k=k, cache=cache)
    ids = {}
    for i, im in enumerate(imgs):
        ids[srv.submit(im, (4, 5000 + i), first_index=7 * i)] = i
    srv.drain()
    res = {ids[r["id"]]: r for r in srv.poll(16)}
    srv.close()
    assert len(res) == len(imgs) and all(r["status"] == 0 for r in res.values())
    R = k // 2
    for i, im in enumerate(imgs):
        H, W_ = im.shape
        seed = (4, 5000 + i)
        for (y, x) in {(0, 0), (H - 1, W_ - 1), (H // 2, W_ // 3)}:
            win = []
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    yy, xx = min(max(y + dy, 0), H - 1), min(max(x + dx, 0), W_ - 1)
                    p = int(im[yy, xx])
                    if p not in entries:
                        entries[p] = o.value_entry(p, cseed)
                    win.append(o.value_encrypt(entries[p], pool, 16, p, seed, 7 * i + yy * W_ + xx))
            ref, sc = o.mean_filter_pixel(np.stack(win), k, k, k, R, R)
            val = o.decrypt(ref, level=2, scale=sc)
            assert abs(res[i]["pixels"][y, x] - val) < 1e-9, (i, y, x)


def _alone(P, ctx, cache, img, seed, k, first_index=0, tile_bytes=0):
    srv = P.Server(ctx, 2 * P.job_bytes(ctx, *img.shape, k, cache, tile_bytes), max_inflight=1, filter_k=k,
                   cache=cache, tile_bytes=tile_bytes)
    srv.submit(img, seed, first_index)
    srv.drain()
    (r,) = srv.poll(4)
    srv.close()
    assert r["status"] == 0
    return r["pixels"]


def test_tiled_jobs_bound_the_footprint(env):
    # row tiles cap a job's device bytes; the result is the untiled one, bit for bit
    P, W, ctx, cache = env
    _say("[gpu] serving tiled jobs")
    img = W.zipf_image(93, 70, 45)
    k = 5
    whole = P.job_bytes(ctx, 70, 45, k, cache)
    cap = whole // 6
    tiled = P.job_bytes(ctx, 70, 45, k, cache, cap)
    assert tiled < whole and tiled <= cap + 70 * 45 * 9 + 4096
    ref = _alone(P, ctx, cache, img, (4, 7000), k)
    got = _alone(P, ctx, cache, img, (4, 7000), k, tile_bytes=cap)
    assert np.array_equal(got, ref)
    one_row = _alone(P, ctx, cache, img, (4, 7000), k, tile_bytes=1)  # at least one row per tile
    assert np.array_equal(one_row, ref)
    assert np.max(np.abs(ref - _box(img, k))) < 2e-3


def test_cancel_before_admission(env):
    P, W, ctx, cache = env
    _say("[gpu] serving cancellation")
    big = W.zipf_image(94, 256, 256)
    small = [W.zipf_image(95 + i, 24, 20) for i in range(3)]
    srv = P.Server(ctx, 4 * P.job_bytes(ctx, 256, 256, 3, cache), max_inflight=1, filter_k=3, cache=cache)
    ja = srv.submit(big, (4, 8000))
    ids = [srv.submit(im, (4, 8001 + i)) for i, im in enumerate(small)]
    srv.cancel(ids[1])  # queued behind the running large job
    with pytest.raises(P.CkksError) as e:
        srv.cancel(ids[1])  # no longer queued
    assert e.value.name == "CKKS_ESTATE"
    with pytest.raises(P.CkksError) as e:
        srv.cancel(10**9)
    assert e.value.name == "CKKS_EINVAL"
    srv.drain()
    res = {r["id"]: r for r in srv.poll(16)}
    st = srv.stats()
    srv.close()
    assert res[ids[1]]["status"] == P.ERRORS_BY_NAME["CKKS_ECANCELED"]
    assert st["canceled"] == 1 and st["completed"] == 3
    assert res[ja]["status"] == 0
    for i in (0, 2):
        assert res[ids[i]]["status"] == 0
        assert np.array_equal(res[ids[i]]["pixels"], _alone(P, ctx, cache, small[i], (4, 8001 + i), 3))


def test_failure_mid_mix_leaves_others_unchanged(env):
    P, W, ctx, cache = env
    _say("[gpu] serving failure injection")
    bigs = [W.zipf_image(110 + i, 200, 200) for i in range(2)]
    smalls = [W.zipf_image(120 + i, 30, 26) for i in range(4)]
    srv = P.Server(ctx, 6 * P.job_bytes(ctx, 200, 200, 3, cache), max_inflight=2, filter_k=3, cache=cache)
    ids = [srv.submit(im, (4, 9000 + i)) for i, im in enumerate(bigs)]
    ids += [srv.submit(im, (4, 9100 + i)) for i, im in enumerate(smalls)]
    srv.inject_failure(ids[3], -4)  # queued behind the two large jobs
    with pytest.raises(P.CkksError):  # only a CKKS_E* code can be injected
        srv.inject_failure(ids[4], 0)
    with pytest.raises(P.CkksError) as e:  # an invalid job inside the mix is refused at submission
        srv.submit(np.zeros((0, 5), np.uint8), (4, 1))
    assert e.value.name == "CKKS_EINVAL"
    srv.drain()
    res = {r["id"]: r for r in srv.poll(16)}
    st = srv.stats()
    srv.close()
    assert res[ids[3]]["status"] == -4 and st["failed"] == 1 and st["completed"] == 5
    for j, (im, sd) in enumerate([(bigs[0], (4, 9000)), (bigs[1], (4, 9001))] +
                                 [(smalls[i], (4, 9100 + i)) for i in range(4)]):
        if j == 3:
            continue
        assert res[ids[j]]["status"] == 0
        assert np.array_equal(res[ids[j]]["pixels"], _alone(P, ctx, cache, im, sd, 3)), j
