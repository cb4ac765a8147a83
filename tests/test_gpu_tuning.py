"""GPU tests of the tuned settings: the autotuner's launch-shape timings, persistence of
the settings in a tuning file (save, load into a fresh context, other ring shapes kept
apart), and that every launch shape of the HBM-bound kernels gives results bit-identical
to the default shape and to the oracle."""
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

    _say("[gpu] tuning context N=4096, 3x36-bit")
    ctx = P.Context(12, 3, 36, 30)
    ctx.keygen(W.keygen_seed(1))
    return P, W, ctx


def test_autotune_save_and_load(env, tmp_path):
    P, W, ctx = env
    _say("[gpu] autotune with launch shapes")
    rep = ctx.autotune(512)
    assert rep["row_wgs_per_cu"] in (0, 2, 4, 8, 16)
    assert rep["gather_wgs_per_cu"] in (2, 4, 8, 16, 32)
    assert all(v > 0 and np.isfinite(v) for v in rep["row_ms"].values())
    assert all(v > 0 and np.isfinite(v) for v in rep["gather_ms"].values())
    assert ctx.launch_shapes() == (rep["row_wgs_per_cu"], rep["gather_wgs_per_cu"])
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    ctx.tune_save(path)  # replaces its own line
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("ckks-tune-v1 ")
    fresh = P.Context(12, 3, 36, 30)
    fresh.keygen(W.keygen_seed(1))
    fresh.set_launch_shapes(64, 1)
    fresh.set_ntt_width(32)
    assert fresh.tune_load(path)
    assert fresh.launch_shapes() == ctx.launch_shapes()
    assert fresh.ntt_width() == rep["encrypt_width"]
    other = P.Context(12, 2, 36, 30)  # another ring shape: not in the file yet
    assert not other.tune_load(path)
    assert other.launch_shapes() == (0, 8)
    other.set_launch_shapes(4, 16)
    other.tune_save(path)
    assert len(open(path).read().splitlines()) == 2
    assert fresh.tune_load(path) and fresh.launch_shapes() == ctx.launch_shapes()
    assert not P.Context(11, 3, 36, 30).tune_load(str(tmp_path / "absent.txt"))
    with open(path, "a") as f:  # a later line for this shape with an unsupported width
        f.write(lines[0].replace(" enc=%d " % rep["encrypt_width"], " enc=64 ") + "\n")
    with pytest.raises(P.CkksError):
        fresh.tune_load(path)
    other.close()
    fresh.close()


def test_launch_shapes_keep_results(env, oracle_mod):
    import torch

    P, W, ctx = env
    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen(W.keygen_seed(1))
    rng = np.random.default_rng(77)
    px = rng.integers(0, 256, 300).astype(np.uint8)
    px_dev = torch.from_numpy(px).cuda()
    radix = ctx.cache_build(P.CKKS_CACHE_RADIX, base=16, digits=2, seed=(5, 6))
    topk = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=24, zero_pool=4, scan_px=px_dev, seed=(5, 6))
    keep = ctx.launch_shapes()

    def run():
        a = ctx.encrypt_pixels(px_dev[:40], (1, 2))
        b = ctx.encrypt_pixels(px_dev[40:80], (1, 3))
        outs = {"add": ctx.add(a, b), "sub": ctx.sub(a, b), "mulc": ctx.mul_const(a, 0.3)}
        outs["rescale"] = ctx.rescale(outs["mulc"])
        c = ctx.add(a, b)
        ctx.add_const(c, 7.0)
        outs["addc"] = c
        outs["radix"] = ctx.encrypt_cached(radix, px_dev, (8, 9), 100)
        outs["topk"] = ctx.encrypt_cached(topk, px_dev, (8, 9), 100)
        torch.cuda.synchronize()
        flat = lambda c: c.to_numpy().reshape(c.count, -1).copy()
        return {k: flat(v) for k, v in outs.items()}, flat(a), flat(b)

    ctx.set_launch_shapes(0, 8)
    ref, A, B = run()
    for shape in [(2, 2), (16, 32), (64, 1), (1, 64)]:
        _say("[gpu] launch shapes %s" % (shape,))
        ctx.set_launch_shapes(*shape)
        got, _, _ = run()
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (shape, k)
    ctx.set_launch_shapes(*keep)
    for i in range(0, 40, 13):
        assert np.array_equal(ref["add"][i], o.add(A[i], B[i]))
        assert np.array_equal(ref["sub"][i], o.sub(A[i], B[i]))
        m, sc = o.mul_const(A[i], 0.3)
        assert np.array_equal(ref["mulc"][i], m)
        assert np.array_equal(ref["rescale"][i], o.rescale(m, scale=sc)[0])
        assert np.array_equal(ref["addc"][i], o.add_const(o.add(A[i], B[i]), 7.0))
    ent = o.radix_entries(16, 2, (5, 6))
    for t in (0, 1, 150, 299):
        assert np.array_equal(ref["radix"][t], o.radix_encrypt(ent, 16, 2, int(px[t]), (8, 9), 100 + t))
    with pytest.raises(P.CkksError):
        ctx.set_launch_shapes(65, 8)
    with pytest.raises(P.CkksError):
        ctx.set_launch_shapes(0, 0)
    radix.close()
    topk.close()
