"""GPU tests of the streamed image pipeline (row tiles with recomputed halos, three
overlapped stage streams): its decrypted output must equal, bit for bit, the whole-image
sequence encrypt -> mean filter -> decrypt through the C ABI (whose ciphertexts and
filter the parity tests pin to the CPU oracle), for every cache kind, window, tile
height (including 1 row, a ragged last tile and one tile for the whole image) and
stream count."""
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

    _say("[gpu] pipeline context N=4096, 3x36-bit")
    ctx = P.Context(12, 3, 36, 30)
    ctx.keygen(W.keygen_seed(5))
    img = W.zipf_image(55, 37, 23)
    px = torch.from_numpy(img.reshape(-1)).cuda()
    caches = {
        "plain": None,
        "radix": ctx.cache_build(P.CKKS_CACHE_RADIX, base=16, digits=2, seed=W.cache_seed(5)),
        "value": ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=64, zero_pool=16, scan_px=px, seed=W.cache_seed(5)),
    }
    torch.cuda.synchronize()
    return P, W, ctx, img, px, caches


def _whole(ctx, cache, px, H, W_, seed, first, k):
    import torch

    ct = ctx.encrypt_cached(cache, px, seed, first) if cache is not None else ctx.encrypt_pixels(px, seed, first)
    flt = ctx.mean_filter(ct, H, W_, k)
    out = ctx.decrypt_pixels(flt)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kind", ["plain", "radix", "value"])
@pytest.mark.parametrize("k,tile,streams", [(3, 8, 3), (5, 4, 3), (5, 1, 3), (3, 37, 1), (5, 10, 1), (7, 6, 3)])
def test_pipeline_equals_whole_image(env, kind, k, tile, streams):
    import torch

    P, W, ctx, img, px, caches = env
    H, W_ = img.shape
    cache = caches[kind]
    _say("[gpu] pipeline %s k=%d tile=%d streams=%d" % (kind, k, tile, streams))
    seed, first = (5, 3), 11
    ref = _whole(ctx, cache, px, H, W_, seed, first, k)
    got = ctx.image_pipeline(px, H, W_, seed, k, tile, streams, cache=cache, first_index=first)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), ref)
    R = k // 2
    pad = np.pad(img.astype(np.float64), R, mode="edge")
    box = sum(pad[dy:dy + H, dx:dx + W_] for dy in range(k) for dx in range(k)) / (k * k)
    assert np.max(np.abs(got.cpu().numpy().reshape(H, W_) - box)) < 2e-3


def test_pipeline_errors(env):
    P, W, ctx, img, px, caches = env
    with pytest.raises(P.CkksError):
        ctx.image_pipeline(px, 37, 23, (1, 1), 4, 8, 3)  # even window
    with pytest.raises(P.CkksError):
        ctx.image_pipeline(px, 37, 23, (1, 1), 3, 8, 2)  # 2 streams
    with pytest.raises(P.CkksError):
        ctx.image_pipeline(px, 37, 23, (1, 1), 3, 0, 3)  # empty tiles
