"""GPU test of the no-allocation cached encryption (ckks_encrypt_cached_noalloc): called
through the C ABI it must give, bit for bit, what ckks_encrypt_cached gives, on two calls
in a row (the second with fewer pixels, so the shared fixed scratch array still holds the
first call's metadata), for value and radix caches; sizes past its fixed array are
refused before any work is enqueued."""
import ctypes as C
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

    _say("[gpu] no-alloc context N=4096, 3x36-bit")
    ctx = P.Context(12, 3, 36, 30)
    ctx.keygen(W.keygen_seed(1))
    return P, W, ctx


def _noalloc(P, ctx, cache, px, seed, first, out, stream):
    b = out.out_batch()
    rc = P.lib().ckks_encrypt_cached_noalloc(ctx.handle, cache.handle, C.c_void_p(px.data_ptr()), int(px.numel()),
                                              P._seed(seed), int(first), C.byref(b), P._stream(stream))
    return rc, b


@pytest.mark.parametrize("kind", ["topk", "full", "radix"])
def test_noalloc_matches_encrypt_cached(env, kind):
    import torch

    P, W, ctx = env
    img = W.zipf_image(71, 96, 64)
    px = torch.from_numpy(img.reshape(-1)).cuda()
    if kind == "topk":
        cache = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=32, zero_pool=16, scan_px=px, seed=(7, 1))
    elif kind == "full":
        cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=8, seed=(7, 2))
    else:
        cache = ctx.cache_build(P.CKKS_CACHE_RADIX, base=16, digits=2, seed=(7, 3))
    stream = torch.cuda.Stream()
    assert P.lib().ckks_encrypt_cached_noalloc_max_pixels(cache.handle) >= 2_000_000
    for call, (n, seed, first) in enumerate([(px.numel(), (3, 1), 0), (1000, (3, 2), 77)]):
        _say("[gpu] no-alloc %s call %d: %d pixels" % (kind, call, n))
        sub = px[:n]
        out = ctx.empty(n)
        rc, b = _noalloc(P, ctx, cache, sub, seed, first, out, stream)
        assert rc == 0, P.ckks_last_error()
        assert b.count == n and b.level == 3 and b.scale == ctx.scale
        ref = ctx.encrypt_cached(cache, sub, seed, first, stream=stream)
        stream.synchronize()
        assert np.array_equal(out.to_numpy(), ref.to_numpy()), "call %d differs" % call
    cache.close()


def test_noalloc_refuses_past_its_array(env):
    import torch

    P, W, ctx = env
    cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=4, seed=(7, 4))
    cap = int(P.lib().ckks_encrypt_cached_noalloc_max_pixels(cache.handle))
    px = torch.zeros(cap + 1, dtype=torch.uint8, device="cuda")
    out = ctx.empty(1)  # also too small: either check refuses before any launch
    rc, _ = _noalloc(P, ctx, cache, px, (1, 1), 0, out, None)
    assert rc == -3, P.ckks_last_error()  # CKKS_ENOMEM_BUDGET, the size check comes first
    torch.cuda.synchronize()
    cache.close()
