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
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: full-rate FP64 VALU lane-operations per second
PEAK_VALU_OPS = 256 * 64 * 2.4e9

# Sources of the plain-encryption kernel; the HBM traffic measured with hardware counters
# (profiles/c2_step_hbm_counters.md) is reported only while they are unchanged.
ENC_SOURCES = ["paper_2409_03568_amd/csrc/" + f for f in
               ("k_ntt_impl.hpp", "k_ntt_13_enc.hip", "ntt.hpp", "modarith.hpp", "philox.hpp", "internal.hpp")]
COUNTERS_MD = os.path.join(ROOT, "profiles", "c2_step_hbm_counters.md")


def sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in ENC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(width):
    """(bytes read + written per plain-encryption launch at this workload, source) from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded in profiles/, or (None, why) when they
    were taken at another NTT width or the kernel's sources changed since (the counters
    cannot be read from inside this process)."""
    try:
        text = open(COUNTERS_MD).read()
    except OSError:
        return None, "no counter record"
    m = re.search(r"traffic k_encrypt_plain_c2 width=(\d+) read_bytes=(\d+) write_bytes=(\d+) .* "
                  r"sources_sha256=([0-9a-f]+)", text)
    if not m:
        return None, "no counter record"
    if int(m.group(1)) != width:
        return None, "counters recorded at width %s, this run uses %d" % (m.group(1), width)
    if sources_sha256() != m.group(4):
        return None, "kernel sources changed since the counters were recorded"
    return int(m.group(2)) + int(m.group(3)), ("rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0 (copy-calibrated) "
                                               "from profiles/c2_step_hbm_counters.md, sources sha256 %s" % m.group(4)[:16])


CONVENTION = ("FP64 VALU issue: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s, i.e. 78.6 TFLOP/s / 2 "
              "with an FMA counted as one op; algorithmic ops = 8 per butterfly (6-op exact modular product + sum "
              "+ difference) and 6 per pointwise modular product")


def host_info():
    """CPU model and logical CPU count of the host running the oracle."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def value_phase(ms, n, hits, S, ops_per_ct):
    """Value-cached encryption against its roofline: each hit writes S bytes (its cache entry
    and pool member are read from L2) and each miss is one plain encryption (FP64 VALU).  The
    serial floor adds the two (hits at 8 TB/s, then misses at 39.3 T ops/s); the overlapped
    floor is the larger of the two, what the misses running beside the hit gather can reach."""
    if not ms:
        return {"ms": 0.0}
    misses = n - hits
    t_hbm = hits * S / (PEAK_HBM_GBS * 1e9) * 1e3
    t_alu = misses * ops_per_ct / PEAK_VALU_OPS * 1e3
    return {"ms": round(ms, 3), "ct_per_s": round(n / (ms / 1e3)), "hits": hits, "misses": misses,
            "GBps_write": round(n * S / (ms / 1e3) / 1e9, 1),
            "roofline": {"floor_serial_ms": round(t_hbm + t_alu, 3), "floor_overlapped_ms": round(max(t_hbm, t_alu), 3),
                         "frac_serial": round((t_hbm + t_alu) / ms, 4), "frac_overlapped": round(max(t_hbm, t_alu) / ms, 4),
                         "hbm_part_ms": round(t_hbm, 3), "alu_part_ms": round(t_alu, 3)}}


def c1_bench(P, W, runs):
    """Config 1: 1024 pixels of a 32x32 uniform image at N = 4096, 3 x 36-bit primes, scale
    2^30 -- plain encryption then decryption (the ciphertext output is 201 MB, about 25 us at
    8 TB/s, so this size is bound by launch and ramp-up latency)."""
    import torch

    cfg = 1
    c = W.CONFIGS[cfg]
    img = W.config_image(cfg)
    n = img.size
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, device=0)
    ctx.keygen(W.keygen_seed(cfg))
    stream = torch.cuda.Stream()
    px = torch.from_numpy(img.reshape(-1)).cuda()
    ct = ctx.empty(n)
    dec = torch.empty(n, dtype=torch.float64, device="cuda")
    for _ in range(3):
        ctx.encrypt_pixels(px, W.job_seed(cfg), out=ct, stream=stream)
        ctx.decrypt_pixels(ct, out=dec, stream=stream)
    stream.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(runs)]
    for k in range(runs):
        evs[k][0].record(stream)
        ctx.encrypt_pixels(px, W.job_seed(cfg), out=ct, stream=stream)
        evs[k][1].record(stream)
        ctx.decrypt_pixels(ct, out=dec, stream=stream)
        evs[k][2].record(stream)
    stream.synchronize()
    enc = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    de = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    err = float(np.max(np.abs(dec.cpu().numpy() - img.reshape(-1))))
    ctx.close()
    return {"pixels": n, "encrypt_ms": round(enc, 4), "decrypt_ms": round(de, 4),
            "ct_per_s": round(n / ((enc + de) / 1e3)), "encrypt_ct_per_s": round(n / (enc / 1e3)),
            "max_abs_err": err}


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=6144,
                    help="pixels in the oracle's timed sample of config 2 (configs 1 and 5 scale with it; 0 = skip)")
    ap.add_argument("--c1-runs", type=int, default=20, help="timed runs of config 1 (0 = skip)")
    ap.add_argument("--phases", default="plain,radix,value,filter,decrypt")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--ntt-width", type=int, default=0, help="values per NTT thread (16 or 32; 0 = library default)")
    ap.add_argument("--batched-runs", type=int, default=2,
                    help="timed runs of the 64-image batched workload (0 = skip it)")
    ap.add_argument("--pipeline-runs", type=int, default=5,
                    help="timed runs per variant of the streamed 512x512 pipeline (0 = skip it)")
    ap.add_argument("--matching-runs", type=int, default=5,
                    help="timed runs of the squared-difference image match (0 = skip)")
    ap.add_argument("--serving-jobs", type=int, default=200,
                    help="jobs per load point of the serving measurement (0 = skip it)")
    ap.add_argument("--serving-budget-gb", type=float, default=160.0, help="device bytes the server may hold")
    ap.add_argument("--serving-tile-gb", type=float, default=0.0,
                    help="cap on one job's row-tile buffers in the server (0 = whole images)")
    ap.add_argument("--serving-slots", type=int, default=8, help="jobs the server runs at once (streams)")
    ap.add_argument("--serving-bypass", type=int, default=8,
                    help="younger jobs the server may start ahead of a waiting one (0 = strict arrival order)")
    return ap.parse_args()


def ntt_ops_per_ct(log_n, L):
    """Algorithmic FP64 VALU operations of one plain encryption: 3 transforms per limb of
    N/2 log N butterflies (8 ops: a 6-op modular product and the sum and difference) and
    2N pointwise modular products (6 ops) per limb."""
    N = 1 << log_n
    butterflies = L * 3 * (N // 2) * log_n
    pointwise = 2 * L * N
    return 8 * butterflies + 6 * pointwise


def mul_ops_per_pair(log_n, level):
    """Algorithmic FP64 VALU operations of one relinearized product at `level` limbs:
    5 transforms per limb for the tensor product (4 forward, 1 inverse for d2), in the
    special prime level forward and 2 inverse transforms, in each q_j level - 1 forward
    (digit j's transform comes from the tensor step) and 2 inverse transforms (8 ops per
    butterfly); per element 7 pointwise products per limb (tensor), 2 per digit and
    prime (key switching) and 4 per limb (ModDown), 6 ops each."""
    N = 1 << log_n
    transforms = 5 * level + (level + 2) + level * (level + 1)
    products = 7 * level + 2 * level * (level + 1) + 4 * level
    return 8 * transforms * (N // 2) * log_n + 6 * products * N


def matching_bench(P, W, runs):
    """Image matching by squared differences (Sec. 4.4.3) on two 256x256 images at
    N = 8192, 4 x 50-bit primes: subtraction, relinearized product, rescale and
    decryption of every pixel pair; the client-side square roots and sum give the L1
    distance, checked against the plaintext one."""
    import torch

    cfg = 2
    c = W.CONFIGS[cfg]
    a_img, b_img = W.matching_pair(cfg, 256, 256)
    n = a_img.size
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, device=0)
    ctx.keygen(W.keygen_seed(cfg))
    ctx.relin_keygen((W.keygen_seed(cfg)[0] ^ 0x5E1, cfg))
    tune = ctx.autotune(8192)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = ctx.encrypt_pixels(torch.from_numpy(a_img.reshape(-1)).cuda(), W.job_seed(cfg, 0), stream=stream)
        b = ctx.encrypt_pixels(torch.from_numpy(b_img.reshape(-1)).cuda(), W.job_seed(cfg, 1), stream=stream)
        d = ctx.empty(n)
        sq = ctx.empty(n)
        r = ctx.empty(n, c.num_primes - 1)
        dec = torch.empty(n, dtype=torch.float64, device="cuda")

        def once(ev=None):
            if ev is not None:
                ev[0].record(stream)
            ctx.sub(a, b, out=d, stream=stream)
            if ev is not None:
                ev[1].record(stream)
            ctx.mul(d, d, out=sq, stream=stream)
            if ev is not None:
                ev[2].record(stream)
            ctx.rescale(sq, out=r, stream=stream)
            if ev is not None:
                ev[3].record(stream)
            ctx.decrypt_pixels(r, out=dec, stream=stream)
            if ev is not None:
                ev[4].record(stream)

        once()
        stream.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(runs)]
        for k in range(runs):
            once(evs[k])
        stream.synchronize()
    names = ["sub", "mul", "rescale", "decrypt"]
    ms = {nm: float(np.median([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(runs)]))
          for i, nm in enumerate(names)}
    total = float(np.median([evs[k][0].elapsed_time(evs[k][4]) for k in range(runs)]))
    got = dec.cpu().numpy()
    diff = a_img.astype(np.int64).reshape(-1) - b_img.astype(np.int64).reshape(-1)
    l1 = float(np.sqrt(np.rint(got).clip(0)).sum())
    best = tune["mul_width"]
    ops = mul_ops_per_pair(c.log_n, c.num_primes) * n
    ach = ops / (ms["mul"] / 1e3) / 1e12
    res = {"pairs": int(n), "ms": {k: round(v, 3) for k, v in ms.items()}, "total_ms": round(total, 3),
           "pairs_per_s": round(n / (total / 1e3)),
           "autotune_8192_pairs_ms": {w: {str(k): round(v, 3) for k, v in tune[w + "_ms"].items()}
                                      for w in ("encrypt", "decrypt", "mul")},
           "mul_roofline": {"bound": "alu", "kernel": "k_mul<13, %d, 1> (tensor, key switch, ModDown; %d values "
                                                      "per thread)" % (best.bit_length() - 1, best),
                            "achieved": round(ach, 3), "peak": round(PEAK_VALU_OPS / 1e12, 3),
                            "unit": "TVALUop/s (FP64)", "frac": round(ach * 1e12 / PEAK_VALU_OPS, 4)},
           "max_sq_err": float(np.max(np.abs(got - diff.astype(np.float64) ** 2))),
           "l1": l1, "l1_plain": float(np.abs(diff).sum())}
    ctx.close()
    del a, b, d, sq, r, dec
    torch.cuda.empty_cache()
    return res


def cpu_baseline(cfg, img, sample):
    """The oracle as it stands, on the host cores, over a bounded sample of the same work:
    `sample` random pixels of the workload's image through its steps (plain encryption and
    decryption for the 32x32 image; plain, radix and value encryption, the k x k filter and
    decryption for the 256x256 and 512x512 images), caches prebuilt as on the GPU."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2409_03568_amd import workloads as W

    c = W.CONFIGS[cfg]
    e = c.extras
    o = O.Oracle(c.log_n, c.num_primes, c.prime_bits, c.log_scale)
    o.keygen(W.keygen_seed(cfg))
    px = img.reshape(-1)
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(px.size, size=min(sample, px.size), replace=False))
    threads = O.num_threads()
    job, cseed = W.job_seed(cfg), W.cache_seed(cfg)
    pool = ThreadPoolExecutor(max_workers=threads)
    full = "base" in e
    if full:  # cache entries: built once, outside the per-pixel timing (as on the GPU)
        rent = o.radix_entries(e["base"], e["digits"], cseed)
        top = o.topk(o.histogram(px), e["topk"])
        ventries = dict(zip(top, pool.map(lambda v: o.value_entry(v, cseed), top)))
        pool_cts = np.stack(list(pool.map(lambda u: o.pool_entry(u, cseed), range(e["pool"]))))
    t = {}
    t0 = time.perf_counter()
    plain = np.stack(list(pool.map(lambda i: o.encrypt(int(px[i]), job, int(i)), idx)))
    t["plain"] = time.perf_counter() - t0
    dec_cts, dec_level = plain, c.num_primes
    if full:
        t0 = time.perf_counter()
        list(pool.map(lambda i: o.radix_encrypt(rent, e["base"], e["digits"], int(px[i]), job, int(i)), idx))
        t["radix"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        list(pool.map(lambda i: o.value_encrypt(ventries.get(int(px[i])), pool_cts, e["pool"], int(px[i]), job,
                                                int(i)), idx))
        t["value"] = time.perf_counter() - t0
        # filter: the oracle sums the k x k ciphertexts around each sampled pixel (taken from
        # the sampled plain ciphertexts, which are of the same size), multiplies and rescales
        k = e["k"]
        patch = np.stack([plain[j % len(plain)] for j in range(k * k)])
        t0 = time.perf_counter()
        flt = list(pool.map(lambda i: o.mean_filter_pixel(patch, k, k, k, k // 2, k // 2)[0], idx))
        t["filter"] = time.perf_counter() - t0
        dec_cts, dec_level = flt, c.num_primes - 1
    t0 = time.perf_counter()
    list(pool.map(lambda j: o.decrypt(dec_cts[j], level=dec_level), range(len(idx))))
    t["decrypt"] = time.perf_counter() - t0
    total = sum(t.values())
    steps = "plain, radix and value encryption, the %dx%d filter and decryption" % (e["k"], e["k"]) if full else \
        "plain encryption and decryption"
    return {
        "value": len(idx) / total,
        "unit": "pixel-ciphertexts/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d random pixels of the %dx%d %s image (N=%d, %d primes) through %s (%d host threads, caches "
                  "prebuilt; %.1f s)" % (len(idx), img.shape[0], img.shape[1], e.get("image", "uniform"), 1 << c.log_n,
                                         c.num_primes, steps, threads, total),
        "phase_s": {k2: round(v, 3) for k2, v in t.items()},
    }


def batched_bench(P, W, runs):
    """64 RGB images (sides log-uniform in 32..512) in one flat index space: full value
    cache encryption with each image's brightness fused in, then decryption, through a
    ring buffer of 65536 ciphertexts, replayed as a HIP graph; the NTT blocking is
    autotuned first."""
    import torch

    cfg = 3
    c = W.CONFIGS[cfg]
    e = c.extras
    imgs, b = W.batched_rgb_images(e["seed"], e["count"], e["lo"], e["hi"])
    px = np.concatenate([im.reshape(-1) for im in imgs])
    ends = np.cumsum([im.size for im in imgs]).astype(np.uint64)
    bf = b.astype(np.float64)
    n = px.size
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, device=0)
    ctx.keygen(W.keygen_seed(cfg))
    tune = ctx.autotune(8192)
    cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=e["pool"], seed=W.cache_seed(cfg))
    plan = P.BatchPlan(ctx, cache, 65536, use_graph=True)
    d_px = torch.from_numpy(px).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    plan.run(d_px, ends, bf, W.job_seed(cfg), 0, out=out, stream=stream)  # eager run + graph capture
    stream.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(runs):
        plan.run(d_px, ends, bf, W.job_seed(cfg), 0, out=out, stream=stream)
    ev[1].record(stream)
    stream.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / runs
    ref = px.astype(np.float64) + np.repeat(bf, [im.size for im in imgs])
    err = float(np.max(np.abs(out.cpu().numpy() - ref)))
    S = ctx.ct_bytes()
    res = {"images": len(imgs), "ciphertexts": int(n), "ms": round(ms, 2), "ct_per_s": round(n / (ms / 1e3)),
           "ciphertext_TB_per_run": round(n * S / 1e12, 3), "GBps_write": round(n * S / (ms / 1e3) / 1e9, 1),
           "frac_of_8TBps": round(n * S / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
           "ring_cts": 65536, "graph": True, "max_abs_err": err,
           "autotune": {"encrypt_width": tune["encrypt_width"], "decrypt_width": tune["decrypt_width"],
                        "encrypt_ms": {str(k): round(v, 3) for k, v in tune["encrypt_ms"].items()},
                        "decrypt_ms": {str(k): round(v, 3) for k, v in tune["decrypt_ms"].items()}}}
    plan.close()
    cache.close()
    ctx.close()
    del d_px, out
    torch.cuda.empty_cache()
    return res


def pipeline_bench(P, W, runs):
    """512x512 Zipf image at N=4096 / 3x36-bit: plain, radix and value-cache encryption ->
    5x5 mean filter -> decryption, in tiles of 64 rows on one stream (a ring of encrypted
    rows) and on three overlapped streams (recomputed halos), against the whole image at
    once."""
    import torch

    cfg = 5
    c = W.CONFIGS[cfg]
    e = c.extras
    img = W.config_image(cfg)
    H, Wd = img.shape
    n = img.size
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, device=0)
    ctx.keygen(W.keygen_seed(cfg))
    px = torch.from_numpy(img.reshape(-1)).cuda()
    caches = {"plain": None,
              "radix": ctx.cache_build(P.CKKS_CACHE_RADIX, base=e["base"], digits=e["digits"], seed=W.cache_seed(cfg)),
              "value": ctx.cache_build(P.CKKS_CACHE_VALUE_TOPK, topk=e["topk"], zero_pool=e["pool"], scan_px=px,
                                       seed=W.cache_seed(cfg))}
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    R = e["k"] // 2
    pad = np.pad(img.astype(np.float64), R, mode="edge")
    box = sum(pad[dy:dy + H, dx:dx + Wd] for dy in range(e["k"]) for dx in range(e["k"])) / (e["k"] ** 2)
    T = 64
    ringrows = min(T + 2 * (e["k"] // 2), H)
    res = {"pixels": n, "k": e["k"], "tile_rows": T, "ciphertext_GB": round(n * ctx.ct_bytes() / 1e9, 1),
           # device buffers of the ciphertexts: one stream keeps a ring of T + 2R encrypted rows and T
           # filtered rows; the whole image keeps every encrypted and filtered ciphertext
           "buffer_GB": {"tiles_1_stream": round((ringrows * ctx.ct_bytes() + T * ctx.ct_bytes(c.num_primes - 1))
                                                 * Wd / 1e9, 2),
                         "whole_image": round(n * (ctx.ct_bytes() + ctx.ct_bytes(c.num_primes - 1)) / 1e9, 2)}}
    for name, cache in caches.items():
        row = {}
        for mode, tile, streams in (("overlap_3_streams", 64, 3), ("tiles_1_stream", 64, 1), ("whole_image", H, 1)):
            ctx.image_pipeline(px, H, Wd, W.job_seed(cfg), e["k"], tile, streams, cache=cache, out=out,
                               stream=stream)
            stream.synchronize()
            times = []
            for _ in range(runs):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                ev[0].record(stream)
                ctx.image_pipeline(px, H, Wd, W.job_seed(cfg), e["k"], tile, streams, cache=cache, out=out,
                                   stream=stream)
                ev[1].record(stream)
                stream.synchronize()
                times.append(ev[0].elapsed_time(ev[1]))
            ms = float(np.median(times))
            row[mode] = {"ms_median": round(ms, 2), "ms_min": round(min(times), 2), "px_per_s": round(n / (ms / 1e3))}
        row["max_abs_err"] = float(np.max(np.abs(out.cpu().numpy().reshape(H, Wd) - box)))
        res[name] = row
    for cch in caches.values():
        if cch is not None:
            cch.close()
    ctx.close()
    del px, out
    torch.cuda.empty_cache()
    return res


def serving_bench(P, W, n_jobs, budget_gb, tile_gb, bypass, slots=8):
    """Serving workload: Poisson arrivals of encrypt (full value cache) -> 3x3 mean filter ->
    decrypt jobs on N=8192 / 4x50-bit; each job alone first (its unloaded latency), then
    closed-loop saturation, then open-loop arrivals at 0.5, 0.8 and 0.95 of it; latency =
    host clock from submission to the decrypted pixels being in host memory, slowdown =
    latency over the job's unloaded latency (job sizes span two orders of magnitude, so the
    raw latency percentiles mostly reflect the size mix)."""
    import torch

    cfg = 4
    c = W.CONFIGS[cfg]
    e = c.extras
    ctx = P.Context(c.log_n, c.num_primes, c.prime_bits, c.log_scale, device=0)
    ctx.keygen(W.keygen_seed(cfg))
    cache = ctx.cache_build(P.CKKS_CACHE_VALUE_FULL, zero_pool=e["pool"], seed=W.cache_seed(cfg))
    torch.cuda.synchronize()
    gaps, imgs = W.serving_jobs(e["seed"], n_jobs, e["lo"], e["hi"])
    px_total = int(sum(im.size for im in imgs))
    budget = int(budget_gb * 1e9)
    tile_bytes = int(tile_gb * 1e9)
    max_job = max(P.job_bytes(ctx, *im.shape, e["k"], cache, tile_bytes) for im in imgs)
    max_job_whole = max(P.job_bytes(ctx, *im.shape, e["k"], cache) for im in imgs)
    srv = P.Server(ctx, budget, max_inflight=slots, filter_k=e["k"], cache=cache,
                   max_job_pixels=max(im.size for im in imgs), tile_bytes=tile_bytes, max_bypass=bypass)

    def run(arrivals):
        t0 = time.perf_counter()
        done, ids = [], {}
        for i, im in enumerate(imgs):
            if arrivals is not None:
                while True:
                    dt = t0 + arrivals[i] - time.perf_counter()
                    if dt <= 0:
                        break
                    done += srv.poll(64, 0)
                    time.sleep(min(dt, 5e-4))
            ids[srv.submit(im, W.job_seed(cfg, i))] = i
        srv.drain()
        wall = time.perf_counter() - t0
        done += srv.poll(len(imgs) + 64, 0)
        assert len(done) == len(imgs) and all(r["status"] == 0 for r in done)
        lat = np.zeros(len(imgs))
        for r in done:
            lat[ids[r["id"]]] = (r["t_done_us"] - r["t_submit_us"]) / 1e3
        return wall, lat

    def pct(lat):
        # latency percentiles, and those of the slowdown: a job's latency over its latency alone
        sd = lat / alone
        return {"p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "slowdown_p50": round(float(np.percentile(sd, 50)), 2),
                "slowdown_p99": round(float(np.percentile(sd, 99)), 2)}

    run(None)  # warm-up (pool allocations, pinned staging)
    alone = np.zeros(len(imgs))  # each job by itself on the idle server
    for i, im in enumerate(imgs):
        jid = srv.submit(im, W.job_seed(cfg, i))
        srv.drain()
        r = srv.poll(4, 0)
        assert len(r) == 1 and r[0]["id"] == jid and r[0]["status"] == 0
        alone[i] = (r[0]["t_done_us"] - r[0]["t_submit_us"]) / 1e3
    wall, lat = run(None)
    sat_qps = len(imgs) / wall
    sizes = np.array([im.size for im in imgs], dtype=np.float64)
    out = {"jobs_per_point": len(imgs), "pixels_per_job_mean": round(px_total / len(imgs), 1),
           "job_pixels_p99_over_p50": round(float(np.percentile(sizes, 99) / np.percentile(sizes, 50)), 2),
           "alone_ms": {"p50": round(float(np.percentile(alone, 50)), 2), "p99": round(float(np.percentile(alone, 99)), 2),
                        "p99_over_p50": round(float(np.percentile(alone, 99) / np.percentile(alone, 50)), 2)},
           "max_job_GB": round(max_job / 1e9, 2), "max_job_GB_untiled": round(max_job_whole / 1e9, 2),
           "tile_GB": tile_gb, "budget_GB": round(budget / 1e9, 1), "slots": slots, "max_bypass": bypass,
           "closed_loop": {"qps": round(sat_qps, 2), "px_per_s": round(px_total / wall), **pct(lat)},
           "open_loop": []}
    for load in (0.5, 0.8, 0.95):
        qps = load * sat_qps
        wall, lat = run(np.cumsum(gaps) / qps)
        out["open_loop"].append({"load": load, "qps": round(qps, 2), "px_per_s": round(px_total / wall), **pct(lat)})
    st = srv.stats()
    out["peak_inflight_jobs"] = st["peak_inflight_jobs"]
    out["peak_inflight_GB"] = round(st["peak_inflight_bytes"] / 1e9, 2)
    out["backfilled_jobs"] = st["backfilled"]
    srv.close()
    cache.close()
    ctx.close()
    return out


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
    # a phase left out of --phases reports 0 (its events bracket no work)
    phase_ms = {nm: float(np.mean([evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(args.steps)]))
                if nm in phases else 0.0 for i, nm in enumerate(names)}
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
        width = ctx.ntt_width()
        traffic, traffic_src = measured_traffic(width)
        roofline = {"bound": "alu",
                    "kernel": "k_encrypt<13, %d, 1, 0, false> (fused plain encryption, %d values per thread)"
                              % (width.bit_length() - 1, width),
                    "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TVALUop/s (FP64)",
                    "frac": round(achieved / peak, 4),
                    "traffic": traffic, "traffic_source": traffic_src, "convention": CONVENTION}
    # the HBM-bound kernels against the 8 TB/s peak (algorithmic bytes: radix and value
    # encryption write S per pixel, the filter reads S and writes S (L-1)/L per pixel)
    hbm = {}
    if phase_ms["radix"] > 0:
        hbm["radix_gather"] = {"GBps": round(n * S / (phase_ms["radix"] / 1e3) / 1e9, 1)}
    if phase_ms["filter"] > 0:
        hbm["mean_filter"] = {"GBps": round(n * S * (1 + (c.num_primes - 1) / c.num_primes) / (phase_ms["filter"] / 1e3) / 1e9, 1)}
    for v in hbm.values():
        v["frac_of_8TBps"] = round(v["GBps"] / PEAK_HBM_GBS, 4)

    def gbs(nbytes, ms):
        return round(nbytes / (ms / 1e3) / 1e9, 1) if ms > 0 else None

    phases_out = {
        "plain": {"ms": round(phase_ms["plain"], 3), "ct_per_s": round(n / (phase_ms["plain"] / 1e3)) if phase_ms["plain"] else None},
        "radix": {"ms": round(phase_ms["radix"], 3), "ct_per_s": round(n / (phase_ms["radix"] / 1e3)) if phase_ms["radix"] else None,
                  "GBps_write": gbs(n * S, phase_ms["radix"])},
        "value": value_phase(phase_ms["value"], n, hits, S, ntt_ops_per_ct(c.log_n, c.num_primes)),
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
        "hbm_kernels": hbm,
    }
    del ct, flt, dec, radix, value
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    progress("step: %.3f ms" % ms_per_step)
    if args.c1_runs > 0:
        out["c1"] = c1_bench(P, W, args.c1_runs)
        progress("config 1 done")
    if args.batched_runs > 0:
        out["batched"] = batched_bench(P, W, args.batched_runs)
        progress("batched done")
    if args.pipeline_runs > 0:
        out["pipeline"] = pipeline_bench(P, W, args.pipeline_runs)
        progress("pipeline done")
    if args.matching_runs > 0:
        out["matching"] = matching_bench(P, W, args.matching_runs)
        progress("matching done")
    if args.serving_jobs > 0:
        out["serving"] = serving_bench(P, W, args.serving_jobs, args.serving_budget_gb, args.serving_tile_gb,
                                       args.serving_bypass, args.serving_slots)
        progress("serving done")
    if args.cpu_sample > 0:
        cb = cpu_baseline(cfg, img, args.cpu_sample)
        cb.update(host_info())
        cb["per_config"] = {"c1": cpu_baseline(1, W.config_image(1), min(args.cpu_sample, 1024)),
                            "c5": cpu_baseline(5, W.config_image(5), max(1, args.cpu_sample // 2))}
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
