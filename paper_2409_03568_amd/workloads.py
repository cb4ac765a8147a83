"""Seeded synthetic inputs for the benchmark configurations.

The paper measures on USC-SIPI images (Sec. 4.2), which are not available here; these
generators stand in for them with images of the sizes and pixel statistics the
benchmark configurations specify.  This module holds no CKKS arithmetic: it only draws
pixels, image sizes, arrival times and seeds, and both the GPU path and the CPU oracle
take their inputs from it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KEYGEN_SEED_WORD = 0x240903568
CACHE_SEED_WORD = 0xCAC4E


def keygen_seed(cfg: int) -> tuple[int, int]:
    return (KEYGEN_SEED_WORD, cfg)


def job_seed(cfg: int, job: int = 0) -> tuple[int, int]:
    return (cfg, job)


def cache_seed(cfg: int) -> tuple[int, int]:
    return (CACHE_SEED_WORD, cfg)


def uniform_image(seed: int, H: int, W: int) -> np.ndarray:
    """uint8 pixels uniform on 0..255."""
    return np.random.default_rng(seed).integers(0, 256, (H, W), dtype=np.uint8)


def zipf_pmf(s: float = 1.1) -> np.ndarray:
    """P(v) proportional to (v + 1)^-s over v = 0..255 (a skewed histogram)."""
    v = np.arange(256, dtype=np.float64)
    p = (v + 1.0) ** (-s)
    return p / p.sum()


def zipf_image(seed: int, H: int, W: int, s: float = 1.1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice(256, size=(H, W), p=zipf_pmf(s)).astype(np.uint8)


def log_uniform_sides(rng: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


@dataclass
class Config:
    name: str
    log_n: int
    num_primes: int
    prime_bits: int
    log_scale: int
    sigma: float = 3.2
    extras: dict = field(default_factory=dict)


CONFIGS = {
    1: Config("N=4096, 3x36-bit primes, scale 2^30; 32x32 uniform image, plain encrypt -> decrypt",
              12, 3, 36, 30, extras=dict(H=32, W=32, image="uniform", seed=1)),
    2: Config("N=8192, 4x50-bit primes, scale 2^40; 256x256 Zipf(1.1) image; plain vs radix-cache (base 16, "
              "2 digits) vs value-cache (top-64, pool 256) encrypt; 3x3 mean filter; decrypt",
              13, 4, 50, 40, extras=dict(H=256, W=256, image="zipf", seed=2, base=16, digits=2, topk=64,
                                         pool=256, k=3)),
    3: Config("N=8192, 4x50-bit primes, scale 2^40; 64 RGB images, sides log-uniform in 32..512; full value "
              "cache; brightness +b per image; decrypt", 13, 4, 50, 40,
              extras=dict(count=64, lo=32, hi=512, seed=3, pool=256)),
    4: Config("N=8192, 4x50-bit primes, scale 2^40; Poisson arrivals of encrypt -> 3x3 mean filter -> decrypt "
              "jobs, Zipf(1.1) grayscale images with sides log-uniform in 32..384", 13, 4, 50, 40,
              extras=dict(lo=32, hi=384, seed=4, pool=256, k=3)),
    5: Config("N=4096, 3x36-bit primes, scale 2^30; 512x512 Zipf(1.1) image; plain / radix / value encrypt; "
              "5x5 mean filter", 12, 3, 36, 30,
              extras=dict(H=512, W=512, image="zipf", seed=5, base=16, digits=2, topk=64, pool=256, k=5)),
}


def config_image(cfg: int) -> np.ndarray:
    c = CONFIGS[cfg]
    e = c.extras
    if e["image"] == "uniform":
        return uniform_image(e["seed"], e["H"], e["W"])
    return zipf_image(e["seed"], e["H"], e["W"])


def batched_rgb_images(seed: int = 3, count: int = 64, lo: int = 32, hi: int = 512):
    """RGB images with sides drawn log-uniform in [lo, hi] and a brightness offset b in -40..40 each."""
    rng = np.random.default_rng(seed)
    H = log_uniform_sides(rng, count, lo, hi)
    W = log_uniform_sides(rng, count, lo, hi)
    imgs = [rng.integers(0, 256, (int(h), int(w), 3), dtype=np.uint8) for h, w in zip(H, W)]
    b = rng.integers(-40, 41, count)
    return imgs, b


def matching_pair(seed: int, H: int, W: int, sigma: float = 8.0, s: float = 1.1):
    """A Zipf image and a perturbed copy of it (Gaussian pixel noise, clipped to 0..255)
    for the squared-difference image match."""
    rng = np.random.default_rng(seed)
    a = rng.choice(256, size=(H, W), p=zipf_pmf(s)).astype(np.int64)
    b = np.clip(a + np.rint(rng.normal(0.0, sigma, size=(H, W))).astype(np.int64), 0, 255)
    return a.astype(np.uint8), b.astype(np.uint8)


def serving_jobs(seed: int, count: int, lo: int = 32, hi: int = 384):
    """Unit-rate exponential arrival gaps and grayscale Zipf images with log-uniform sides;
    the arrival times at rate qps are cumsum(gaps) / qps, so every rate sees the same jobs."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, size=count)
    H = log_uniform_sides(rng, count, lo, hi)
    W = log_uniform_sides(rng, count, lo, hi)
    pmf = zipf_pmf()
    imgs = [rng.choice(256, size=(int(h), int(w)), p=pmf).astype(np.uint8) for h, w in zip(H, W)]
    return gaps, imgs


def poisson_arrivals(seed: int, qps: float, count: int, lo: int = 32, hi: int = 384):
    """Job arrival times (exponential gaps) and grayscale Zipf images with log-uniform sides."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps)
    H = log_uniform_sides(rng, count, lo, hi)
    W = log_uniform_sides(rng, count, lo, hi)
    pmf = zipf_pmf()
    imgs = [rng.choice(256, size=(int(h), int(w)), p=pmf).astype(np.uint8) for h, w in zip(H, W)]
    return t, imgs
