"""GPU parity at the ring degrees the benchmark configurations do not use (N = 2^11 and
2^14), for every register blocking the degree allows: keys, encryption and the
relinearized product bit-exact against the oracle, decryption to the pixel values.  At
N = 2^11 with 32 values per thread the workgroup is a single wave, so every NTT exchange
runs without a workgroup barrier; at N = 2^14 the encryption kernel keeps its samples in
registers and runs its inverse transforms one at a time."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RINGS = [(11, 3, 30, 20, (8, 16, 32)), (14, 4, 50, 40, (16, 32))]


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


def _dev(px):
    import torch

    return torch.from_numpy(np.ascontiguousarray(px, dtype=np.uint8).reshape(-1)).cuda()


def _np(cts):
    import torch

    torch.cuda.synchronize()
    return cts.to_numpy().reshape(cts.count, -1)


@pytest.mark.parametrize("log_n,L,bits,log_scale,widths", RINGS)
def test_ring_parity(P, oracle_mod, log_n, L, bits, log_scale, widths):
    px = np.array([0, 1, 7, 64, 128, 200, 254, 255, 33, 99, 150, 77], dtype=np.uint8)
    o = oracle_mod.Oracle(log_n, L, bits, log_scale)
    o.keygen((11, log_n))
    o.relin_keygen((12, log_n))
    ref = o.encrypt_batch(px, (13, log_n), first_index=5)
    prod = [o.mul(ref[i], ref[i + 6]) for i in range(6)]
    for w in widths:
        _say("[gpu] ring N=2^%d width %d" % (log_n, w))
        ctx = P.Context(log_n, L, bits, log_scale)
        ctx.set_ntt_width(w)
        ctx.keygen((11, log_n))
        s, pk = ctx.keys_export()
        assert np.array_equal(s, o.s) and np.array_equal(pk, o.pk), w
        cts = ctx.encrypt_pixels(_dev(px), (13, log_n), first_index=5)
        got = _np(cts)
        assert np.array_equal(got, ref), w
        dec = ctx.decrypt_pixels(cts).cpu().numpy()
        # fresh noise ~ 2^8 per coefficient decodes to ~2^8 sqrt(N/2) / scale (0.008 at
        # N=2^11 and scale 2^20, 2e-8 at N=2^14 and scale 2^40); allow 8 times that
        assert np.max(np.abs(dec - px)) < 8 * 2.0**8 * np.sqrt(2.0**log_n / 2) / 2.0**log_scale, w
        ctx.relin_keygen((12, log_n))
        evk, qP = ctx.relin_keys_export()
        assert qP == o.qP and np.array_equal(evk, o.evk.reshape(evk.shape)), w
        m = _np(ctx.mul(cts[0:6], cts[6:12]))
        for i in range(6):
            assert np.array_equal(m[i], prod[i]), (w, i)
        ctx.close()
