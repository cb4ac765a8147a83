"""Benchmark of the pixel-level CKKS hot path on one MI355X.

One step is one pass of the whole path over one 256x256 image (N = 8192, 4 x 50-bit
primes, scale 2^40, Zipf(1.1) pixels): plain encryption of every pixel, radix-cached
encryption (base 16, 2 digits), value-cached encryption (top-64 values, pool of 256
encrypted zeros), a 3x3 homomorphic mean filter (8 additions, multiply by 1/9, rescale)
and decryption.  Inputs are resident in HBM before the timed region; caches are built
beforehand (their build time is reported separately).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: full-rate FP64 VALU lane-operations per second
PEAK_VALU_OPS = 256 * 64 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=192, help="pixels in the oracle's timed sample (0 = skip)")
    ap.add_argument("--phases", default="plain,radix,value,filter,decrypt")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--ntt-width", type=int, default=0, help="values per NTT thread (16 or 32; 0 = library default)")
    return ap.parse_args()


def ntt_ops_per_ct(log_n, L):
    """Algorithmic FP64 VALU operations of one plain encryption: 3 transforms per limb of
    N/2 log N butterflies (8 ops: a 6-op modular product and the sum and difference) and
    2N pointwise modular products (6 ops) per limb."""
    N = 1 << log_n
    butterflies = L * 3 * (N // 2) * log_n
    pointwise = 2 * L * N
    return 8 * butterflies + 6 * pointwise


def cpu_baseline(cfg, img, sample):
    """The oracle as it stands, on the host cores, over a bounded sample of the same work."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2409_03568_amd import workloads as W

    c = W.CONFIGS[cfg]
    e = c.extras
    o = O.Oracle(c.log_n, c.num_primes, c.prime_bits, c.log_scale)
    o.keygen(W.keygen_seed(cfg))
    H, Wd = img.shape
    px = img.reshape(-1)
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(px.size, size=sample, replace=False))
    threads = O.num_threads()
    job, cseed = W.job_seed(cfg), W.cache_seed(cfg)
    pool = ThreadPoolExecutor(max_workers=threads)
    # cache entries: built once, outside the per-pixel timing (as on the GPU)
    rent = o.radix_entries(e["base"], e["digits"], cseed)
    top = o.topk(o.histogram(px), e["topk"])
    ventries = dict(zip(top, pool.map(lambda v: o.value_entry(v, cseed), top)))
    pool_cts = np.stack(list(pool.map(lambda u: o.pool_entry(u, cseed), range(e["pool"]))))
    t = {}
    t0 = time.perf_counter()
    plain = np.stack(list(pool.map(lambda i: o.encrypt(int(px[i]), job, int(i)), idx)))
    t["plain"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    list(pool.map(lambda i: o.radix_encrypt(rent, e["base"], e["digits"], int(px[i]), job, int(i)), idx))
    t["radix"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    list(pool.map(lambda i: o.value_encrypt(ventries.get(int(px[i])), pool_cts, e["pool"], int(px[i]), job, int(i)),
                  idx))
    t["value"] = time.perf_counter() - t0
    # filter: the oracle sums the k x k ciphertexts around each sampled pixel (taken from
    # the sampled plain ciphertexts, which are of the same size), multiplies and rescales
    k = e["k"]
    patch = np.stack([plain[j % len(plain)] for j in range(k * k)])
    t0 = time.perf_counter()
    list(pool.map(lambda i: o.mean_filter_pixel(patch, k, k, k, k // 2, k // 2), idx))
    t["filter"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    list(pool.map(lambda j: o.decrypt(plain[j]), range(len(idx))))
    t["decrypt"] = time.perf_counter() - t0
    total = sum(t.values())
    return {
        "value": sample / total,
        "unit": "pixel-ciphertexts/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d random pixels of the same image through plain, radix and value encryption, the 3x3 filter "
                  "and decryption (%d host threads, caches prebuilt)" % (sample, threads),
        "phase_s": {k2: round(v, 3) for k2, v in t.items()},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the workload is one GPU's share); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2409_03568_amd as P
    from paper_2409_03568_amd import workloads as W

    cfg = 2
    c = W.CONFIGS[cfg]
    e = c.extras
    img = W.config_image(cfg)
    H, Wd = img.shape
    n = img.size
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.int64, device=dev).fill_(7)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, device=0)
    if args.ntt_width:
        ctx.set_ntt_width(args.ntt_width)
    ctx.keygen(W.keygen_seed(cfg))
    px = torch.from_numpy(img.reshape(-1)).to(dev)
    stream = torch.cuda.Stream(device=dev)
    job = W.job_seed(cfg)
    phases = [p for p in args.phases.split(",") if p]

    with torch.cuda.stream(stream):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        radix = ctx.cache_build(P.CKKS_CACHE_RADIX, base=e["base"], digits=e["digits"], seed=W.cache_seed(cfg),
                                stream=stream)
        ev[1].record(stream)
        value = ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=e["topk"], zero_pool=e["pool"], scan_px=px,
                                seed=W.cache_seed(cfg), stream=stream)
        ev[2].record(stream)
        stream.synchronize()
        cache_ms = {"radix": ev[0].elapsed_time(ev[1]), "value_topk": ev[1].elapsed_time(ev[2])}
        ct = ctx.empty(n)
        flt = ctx.empty(n, c.num_primes - 1)
        dec = torch.empty(n, dtype=torch.float64, device=dev)
        hits = int(np.isin(img, [v for v in value.export()[0]]).sum())

        def step(events=None):
            def mark(i):
                if events is not None:
                    events[i].record(stream)

            mark(0)
            if "plain" in phases:
                ctx.encrypt_pixels(px, job, out=ct, stream=stream)
            mark(1)
            if "radix" in phases:
                ctx.encrypt_cached(radix, px, job, out=ct, stream=stream)
            mark(2)
            if "value" in phases:
                ctx.encrypt_cached(value, px, job, out=ct, stream=stream)
            mark(3)
            if "filter" in phases:
                ctx.mean_filter(ct, H, Wd, e["k"], out=flt, stream=stream)
            mark(4)
            if "decrypt" in phases:
                ctx.decrypt_pixels(flt if "filter" in phases else ct, out=dec, stream=stream)
            mark(5)

        for _ in range(args.warmup):
            step()
        stream.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            step(evs[s])
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    names = ["plain", "radix", "value", "filter", "decrypt"]
    phase_ms = {nm: float(np.mean([evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(args.steps)]))
                for i, nm in enumerate(names)}
    step_ms = float(np.mean([evs[s][0].elapsed_time(evs[s][5]) for s in range(args.steps)]))
    ms_per_step = wall * 1000.0 / args.steps
    S = ctx.ct_bytes()
    # correctness guard on the measured output (decrypted filter vs the plaintext filter)
    ok = None
    if "filter" in phases and "decrypt" in phases:
        R = e["k"] // 2
        pad = np.pad(img.astype(np.float64), R, mode="edge")
        box = sum(pad[dy:dy + H, dx:dx + Wd] for dy in range(e["k"]) for dx in range(e["k"])) / (e["k"] ** 2)
        ok = float(np.max(np.abs(dec.cpu().numpy().reshape(H, Wd) - box)))

    ops = ntt_ops_per_ct(c.log_n, c.num_primes) * n
    t_plain = phase_ms["plain"] / 1e3
    roofline = None
    if t_plain > 0:
        achieved = ops / t_plain / 1e12
        peak = PEAK_VALU_OPS / 1e12
        roofline = {"bound": "alu", "kernel": "k_encrypt<13,5> (fused plain encryption)", "achieved": round(achieved, 3),
                    "peak": round(peak, 3), "unit": "TVALUop/s (FP64)", "frac": round(achieved / peak, 4),
                    "traffic": None}

    def gbs(nbytes, ms):
        return round(nbytes / (ms / 1e3) / 1e9, 1) if ms > 0 else None

    phases_out = {
        "plain": {"ms": round(phase_ms["plain"], 3), "ct_per_s": round(n / (phase_ms["plain"] / 1e3)) if phase_ms["plain"] else None},
        "radix": {"ms": round(phase_ms["radix"], 3), "ct_per_s": round(n / (phase_ms["radix"] / 1e3)) if phase_ms["radix"] else None,
                  "GBps_write": gbs(n * S, phase_ms["radix"])},
        "value": {"ms": round(phase_ms["value"], 3), "ct_per_s": round(n / (phase_ms["value"] / 1e3)) if phase_ms["value"] else None,
                  "hits": hits, "GBps_alg": gbs(n * S + hits * 2 * S, phase_ms["value"])},
        "filter": {"ms": round(phase_ms["filter"], 3), "GBps_alg": gbs(n * S * (1 + (c.num_primes - 1) / c.num_primes),
                                                                        phase_ms["filter"])},
        "decrypt": {"ms": round(phase_ms["decrypt"], 3), "ct_per_s": round(n / (phase_ms["decrypt"] / 1e3)) if phase_ms["decrypt"] else None},
    }
    out = {
        "metric": "pixel ciphertexts/sec (plain vs cached encrypt) + p50/p99 job latency, 1 GPU",
        "value": round(n / (ms_per_step / 1e3), 1),
        "unit": "pixel-ciphertexts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256x256 Zipf(1.1) image, N=8192, 4x50-bit primes, scale 2^40: plain + radix(16,2) + "
                               "value(top-64, pool 256) encryption, 3x3 mean filter, decryption",
                   "pixels": n, "log_n": c.log_n, "primes": c.num_primes, "prime_bits": c.prime_bits,
                   "parallelism": "1 GPU"},
        "phases": phases_out,
        "step_ms_events": round(step_ms, 3),
        "cache_build_ms": {k: round(v, 3) for k, v in cache_ms.items()},
        "filter_decrypt_max_err": ok,
        "roofline": roofline,
    }
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(cfg, img, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
