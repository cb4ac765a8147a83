"""Python access to the plain CPU CKKS oracle (ckks_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this module.  It neither imports nor is imported by
the product package, and the two share no code.

The oracle follows arXiv 2409.03568 (iCHEETAH): Sec. 2.2.2 for key generation,
encryption and decryption, Sec. 2.2.3 for the homomorphic operations, Sec. 3.2
for radix / scanning / full caching, Sec. 3.3 for the randomness added to cached
ciphertexts and Sec. 4.4 for the image operations.  Conventions are listed in
ckks_oracle.h.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_HDR = os.path.join(_HERE, "ckks_oracle.h")
_LIB = os.path.join(_HERE, "liborc.so")

MAX_LIMBS = 16
MAX_B = 64
TAG_V, TAG_E0, TAG_E1, TAG_AUX, TAG_SK, TAG_EK, TAG_A0 = 1, 2, 3, 4, 16, 17, 32
RADIX_BASE_T, VALUE_BASE_T, POOL_BASE_T = 0, 256, 512


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(
        os.path.getmtime(_SRC), os.path.getmtime(_HDR)
    ):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = [
        "gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
        "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("log_n", C.c_int), ("L", C.c_int), ("log_scale", C.c_int), ("B", C.c_int),
        ("sigma", C.c_double),
        ("q", C.c_uint64 * MAX_LIMBS), ("psi", C.c_uint64 * MAX_LIMBS),
        ("cdt", C.c_uint64 * (2 * MAX_B)),
        ("qP", C.c_uint64), ("psiP", C.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER(_Params)
        u64p, i64p, dp, u8p = (C.POINTER(C.c_uint64), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                               C.POINTER(C.c_uint8))
        ip = C.POINTER(C.c_int)
        sig = {
            "orc_gen_primes": (C.c_int, [C.c_int, C.c_int, C.c_int, u64p]),
            "orc_primitive_2n_root": (C.c_uint64, [C.c_uint64, C.c_int]),
            "orc_cdt_table": (C.c_int, [C.c_double, C.c_int, u64p]),
            "orc_params_init": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, u64p]),
            "orc_philox4x64_10": (None, [u64p, u64p, u64p]),
            "orc_stream_word": (C.c_uint64, [u64p, C.c_uint64, C.c_uint64, C.c_uint64]),
            "orc_ternary": (C.c_int64, [C.c_uint64]),
            "orc_gauss": (C.c_int64, [C.c_uint64, u64p, C.c_int]),
            "orc_sample_ternary": (None, [u64p, C.c_uint64, C.c_uint64, C.c_int, i64p]),
            "orc_sample_gauss": (None, [P, u64p, C.c_uint64, C.c_uint64, i64p]),
            "orc_sample_uniform": (None, [u64p, C.c_uint64, C.c_uint64, C.c_int, C.c_uint64, u64p]),
            "orc_negacyclic_schoolbook": (None, [u64p, u64p, u64p, C.c_int, C.c_uint64]),
            "orc_negacyclic_mul": (None, [u64p, u64p, u64p, C.c_int, C.c_uint64, C.c_uint64]),
            "orc_encode_table": (None, [C.c_int, C.c_int, dp]),
            "orc_encode": (None, [P, C.c_double, i64p]),
            "orc_keygen": (None, [P, u64p, i64p, u64p]),
            "orc_encrypt": (None, [P, u64p, C.c_double, u64p, C.c_uint64, u64p]),
            "orc_decrypt_coeffs": (None, [P, i64p, u64p, C.c_int, u64p]),
            "orc_decode_centered": (C.c_int, [P, u64p, C.c_int, i64p]),
            "orc_decrypt": (C.c_double, [P, i64p, u64p, C.c_int, C.c_double, ip]),
            "orc_add": (None, [P, u64p, u64p, u64p, C.c_int]),
            "orc_sub": (None, [P, u64p, u64p, u64p, C.c_int]),
            "orc_mul_const": (C.c_int, [P, u64p, C.c_int, C.c_double, C.c_double, u64p, dp]),
            "orc_add_const": (C.c_int, [P, u64p, C.c_int, C.c_double, C.c_double]),
            "orc_rescale": (C.c_int, [P, u64p, C.c_int, C.c_double, u64p, dp]),
            "orc_radix_entries": (None, [P, u64p, C.c_int, C.c_int, u64p, u64p]),
            "orc_radix_encrypt": (C.c_int, [P, u64p, C.c_int, C.c_int, C.c_int, u64p, C.c_uint64, u64p]),
            "orc_histogram": (None, [u8p, C.c_uint64, u64p]),
            "orc_topk": (C.c_int, [u64p, C.c_int, ip]),
            "orc_value_entry": (None, [P, u64p, C.c_int, u64p, u64p]),
            "orc_pool_entry": (None, [P, u64p, C.c_int, u64p, u64p]),
            "orc_pool_pick": (C.c_uint32, [u64p, C.c_uint64, C.c_uint32]),
            "orc_value_encrypt": (None, [P, u64p, u64p, u64p, C.c_uint32, C.c_int, u64p, C.c_uint64, u64p]),
            "orc_mean_filter_pixel": (C.c_int, [P, u64p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                               C.c_int, C.c_int, u64p, dp]),
            "orc_encrypt_batch": (None, [P, u64p, u8p, C.c_uint64, u64p, C.c_uint64, u64p]),
            "orc_decrypt_batch": (None, [P, i64p, u64p, C.c_uint64, C.c_int, C.c_double, dp, ip]),
            "orc_num_threads": (C.c_int, []),
            "orc_relin_keygen": (None, [P, i64p, u64p, u64p]),
            "orc_tensor": (None, [P, u64p, u64p, C.c_int, u64p]),
            "orc_key_switch": (None, [P, u64p, u64p, C.c_int, u64p]),
            "orc_mod_down": (None, [P, u64p, C.c_int, u64p]),
            "orc_mul": (None, [P, u64p, u64p, u64p, C.c_int, u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint64))


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


def _seed(seed):
    s = np.array([int(seed[0]) & (2**64 - 1), int(seed[1]) & (2**64 - 1)], dtype=np.uint64)
    return s, s.ctypes.data_as(C.POINTER(C.c_uint64))


# ---------------------------------------------------------------------------
# scalar pieces
# ---------------------------------------------------------------------------
def gen_primes(log_n: int, bits: int, L: int) -> list[int]:
    q = np.zeros(L, dtype=np.uint64)
    n = lib().orc_gen_primes(log_n, bits, L, q.ctypes.data_as(C.POINTER(C.c_uint64)))
    return [int(x) for x in q[:n]]


def primitive_2n_root(q: int, log_n: int) -> int:
    return int(lib().orc_primitive_2n_root(q, log_n))


def cdt_table(sigma: float, B: int) -> np.ndarray:
    T = np.zeros(max(2 * B, 1), dtype=np.uint64)
    rc = lib().orc_cdt_table(sigma, B, T.ctypes.data_as(C.POINTER(C.c_uint64)))
    assert rc == 0
    return T[: 2 * B]


def philox(ctr, key) -> list[int]:
    c, cp = _u64([int(x) & (2**64 - 1) for x in ctr])
    k, kp = _u64([int(x) & (2**64 - 1) for x in key])
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(cp, kp, out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return [int(x) for x in out]


def stream_word(key, t: int, tag: int, j: int) -> int:
    k, kp = _seed(key)
    return int(lib().orc_stream_word(kp, t, tag, j))


def ternary(w: int) -> int:
    return int(lib().orc_ternary(w))


def gauss(w: int, T: np.ndarray, B: int) -> int:
    T, Tp = _u64(T if len(T) else np.zeros(1, dtype=np.uint64))
    return int(lib().orc_gauss(w, Tp, B))


def negacyclic_schoolbook(a, b, q: int) -> np.ndarray:
    a, ap = _u64(a)
    b, bp = _u64(b)
    c = np.zeros(len(a), dtype=np.uint64)
    lib().orc_negacyclic_schoolbook(ap, bp, c.ctypes.data_as(C.POINTER(C.c_uint64)), len(a), q)
    return c


def negacyclic_mul(a, b, q: int, psi: int) -> np.ndarray:
    a, ap = _u64(a)
    b, bp = _u64(b)
    c = np.zeros(len(a), dtype=np.uint64)
    lib().orc_negacyclic_mul(ap, bp, c.ctypes.data_as(C.POINTER(C.c_uint64)), len(a), q, psi)
    return c


def encode_table(log_n: int, log_scale: int) -> np.ndarray:
    T = np.zeros(1 << log_n, dtype=np.float64)
    lib().orc_encode_table(log_n, log_scale, T.ctypes.data_as(C.POINTER(C.c_double)))
    return T


def psnr(mse: float, max_i: float = 255.0) -> float:
    """Peak signal-to-noise ratio, Sec. 4.3.2: 10 log10(MAX^2 / MSE)."""
    import math

    return 10.0 * math.log10(max_i * max_i / mse)


def mse(a, b) -> float:
    """Mean squared error between two images, Sec. 4.3.2."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.mean((a - b) ** 2))


# ---------------------------------------------------------------------------
# a parameter set with its keys
# ---------------------------------------------------------------------------
@dataclass
class Oracle:
    log_n: int
    L: int
    bits: int
    log_scale: int
    sigma: float = 3.2
    B: int | None = None
    primes: list[int] | None = None

    def __post_init__(self):
        if self.B is None:
            self.B = int(6 * self.sigma) if self.sigma > 0 else 0
        self.P = _Params()
        pr = None
        if self.primes is not None:
            pr_arr = np.array(self.primes, dtype=np.uint64)
            self._pr_keep = pr_arr
            pr = pr_arr.ctypes.data_as(C.POINTER(C.c_uint64))
        rc = lib().orc_params_init(C.byref(self.P), self.log_n, self.L, self.bits, self.log_scale,
                                   self.sigma, self.B, pr)
        if rc != 0:
            raise ValueError("orc_params_init failed: %d" % rc)
        self.N = 1 << self.log_n
        self.q = [int(self.P.q[i]) for i in range(self.L)]
        self.psi = [int(self.P.psi[i]) for i in range(self.L)]
        self.B = int(self.P.B)
        self.cdt = np.array([int(self.P.cdt[k]) for k in range(2 * self.B)], dtype=np.uint64)
        self.scale = float(2.0**self.log_scale)
        self.qP = int(self.P.qP)
        self.psiP = int(self.P.psiP)
        self.s = None
        self.pk = None
        self.evk = None

    # -- sizes ---------------------------------------------------------------
    def ct_words(self, level: int | None = None) -> int:
        return 2 * (self.L if level is None else level) * self.N

    @property
    def _p(self):
        return C.byref(self.P)

    # -- sampling --------------------------------------------------------------
    def sample_ternary(self, key, t, tag):
        k, kp = _seed(key)
        out = np.zeros(self.N, dtype=np.int64)
        lib().orc_sample_ternary(kp, t, tag, self.N, out.ctypes.data_as(C.POINTER(C.c_int64)))
        return out

    def sample_gauss(self, key, t, tag):
        k, kp = _seed(key)
        out = np.zeros(self.N, dtype=np.int64)
        lib().orc_sample_gauss(self._p, kp, t, tag, out.ctypes.data_as(C.POINTER(C.c_int64)))
        return out

    def sample_uniform(self, key, t, tag, q):
        k, kp = _seed(key)
        out = np.zeros(self.N, dtype=np.uint64)
        lib().orc_sample_uniform(kp, t, tag, self.N, q, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    # -- CKKS -------------------------------------------------------------------
    def encode(self, value: float) -> np.ndarray:
        m = np.zeros(self.N, dtype=np.int64)
        lib().orc_encode(self._p, float(value), m.ctypes.data_as(C.POINTER(C.c_int64)))
        return m

    def keygen(self, seed):
        k, kp = _seed(seed)
        s = np.zeros(self.N, dtype=np.int64)
        pk = np.zeros(2 * self.L * self.N, dtype=np.uint64)
        lib().orc_keygen(self._p, kp, s.ctypes.data_as(C.POINTER(C.c_int64)),
                         pk.ctypes.data_as(C.POINTER(C.c_uint64)))
        self.s, self.pk = s, pk
        return s, pk

    def set_keys(self, s, pk):
        self.s = np.ascontiguousarray(s, dtype=np.int64)
        self.pk = np.ascontiguousarray(pk, dtype=np.uint64).reshape(-1)

    def encrypt(self, value: float, seed, t: int) -> np.ndarray:
        k, kp = _seed(seed)
        pk, pkp = _u64(self.pk)
        ct = np.zeros(self.ct_words(), dtype=np.uint64)
        lib().orc_encrypt(self._p, pkp, float(value), kp, t, ct.ctypes.data_as(C.POINTER(C.c_uint64)))
        return ct

    def encrypt_batch(self, px, seed, first_index: int = 0) -> np.ndarray:
        px = np.ascontiguousarray(px, dtype=np.uint8).reshape(-1)
        k, kp = _seed(seed)
        pk, pkp = _u64(self.pk)
        out = np.zeros((len(px), self.ct_words()), dtype=np.uint64)
        lib().orc_encrypt_batch(self._p, pkp, px.ctypes.data_as(C.POINTER(C.c_uint8)), len(px), kp,
                                first_index, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    def decrypt_coeffs(self, ct, level: int | None = None) -> np.ndarray:
        level = self.L if level is None else level
        ct, ctp = _u64(ct)
        s, sp = _i64(self.s)
        d = np.zeros(level * self.N, dtype=np.uint64)
        lib().orc_decrypt_coeffs(self._p, sp, ctp, level, d.ctypes.data_as(C.POINTER(C.c_uint64)))
        return d.reshape(level, self.N)

    def decode_centered(self, d, level: int) -> tuple[np.ndarray, int]:
        d, dp = _u64(np.asarray(d).reshape(-1))
        x = np.zeros(self.N, dtype=np.int64)
        rc = lib().orc_decode_centered(self._p, dp, level, x.ctypes.data_as(C.POINTER(C.c_int64)))
        return x, rc

    def decrypt(self, ct, level: int | None = None, scale: float | None = None) -> float:
        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        ct, ctp = _u64(ct)
        s, sp = _i64(self.s)
        err = C.c_int(0)
        v = lib().orc_decrypt(self._p, sp, ctp, level, scale, C.byref(err))
        if err.value:
            raise ArithmeticError("decryption bound violated (limb-0 lift disagrees with CRT)")
        return float(v)

    def decrypt_exact(self, ct, level: int | None = None, scale: float | None = None) -> float:
        """Decryption by its definition (Sec. 2.2.2), without the limb-0 shortcut: the residues
        d_i = c0_i + c1_i s of every limb, their centered integer x in (-Q/2, Q/2] by the
        Chinese remainder theorem over all `level` primes (Python integers), and slot 0 of
        the decoding, sum_j x_j cos(pi j / N) / scale, summed exactly rounded (math.fsum)."""
        import math

        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        d = self.decrypt_coeffs(ct, level)
        qs = self.q[:level]
        Q = math.prod(qs)
        x = [0] * self.N
        for i, qi in enumerate(qs):
            Mi = Q // qi
            ci = Mi * pow(Mi % qi, -1, qi)
            row = [int(v) for v in d[i]]
            for j in range(self.N):
                x[j] += row[j] * ci
        terms = []
        for j in range(self.N):
            xj = x[j] % Q
            if xj > Q // 2:
                xj -= Q
            terms.append(float(xj) * math.cos(math.pi * j / self.N))
        return math.fsum(terms) / scale

    def decrypt_batch(self, cts, level: int | None = None, scale: float | None = None) -> np.ndarray:
        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        cts = np.ascontiguousarray(cts, dtype=np.uint64)
        n = cts.size // (2 * level * self.N)
        s, sp = _i64(self.s)
        out = np.zeros(n, dtype=np.float64)
        nerr = C.c_int(0)
        lib().orc_decrypt_batch(self._p, sp, cts.ctypes.data_as(C.POINTER(C.c_uint64)), n, level, scale,
                                out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nerr))
        if nerr.value:
            raise ArithmeticError("decryption bound violated in %d ciphertexts" % nerr.value)
        return out

    # -- homomorphic operations ---------------------------------------------------
    def add(self, a, b, level=None):
        level = self.L if level is None else level
        a, ap = _u64(a)
        b, bp = _u64(b)
        out = np.zeros_like(a)
        lib().orc_add(self._p, ap, bp, out.ctypes.data_as(C.POINTER(C.c_uint64)), level)
        return out

    def sub(self, a, b, level=None):
        level = self.L if level is None else level
        a, ap = _u64(a)
        b, bp = _u64(b)
        out = np.zeros_like(a)
        lib().orc_sub(self._p, ap, bp, out.ctypes.data_as(C.POINTER(C.c_uint64)), level)
        return out

    def mul_const(self, a, c, level=None, scale=None):
        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        a, ap = _u64(a)
        out = np.zeros_like(a)
        sc = C.c_double(0)
        rc = lib().orc_mul_const(self._p, ap, level, scale, float(c), out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 C.byref(sc))
        if rc:
            raise ValueError("mul_const constant out of range")
        return out, sc.value

    def add_const(self, a, b, level=None, scale=None):
        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        a = np.array(a, dtype=np.uint64, copy=True)
        rc = lib().orc_add_const(self._p, a.ctypes.data_as(C.POINTER(C.c_uint64)), level, scale, float(b))
        if rc:
            raise ValueError("add_const constant out of range")
        return a

    def rescale(self, a, level=None, scale=None):
        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        a, ap = _u64(a)
        out = np.zeros(2 * (level - 1) * self.N, dtype=np.uint64)
        sc = C.c_double(0)
        rc = lib().orc_rescale(self._p, ap, level, scale, out.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(sc))
        if rc:
            raise ValueError("rescale needs level >= 2")
        return out, sc.value

    # -- ciphertext multiplication ------------------------------------------------
    def relin_keygen(self, seed) -> np.ndarray:
        """Key-switching keys of s^2: evk[i][j][2][N] (digit i < L, prime j <= L, j = L is qP)."""
        k, kp = _seed(seed)
        s, sp = _i64(self.s)
        evk = np.zeros(self.L * (self.L + 1) * 2 * self.N, dtype=np.uint64)
        lib().orc_relin_keygen(self._p, sp, kp, evk.ctypes.data_as(C.POINTER(C.c_uint64)))
        self.evk = evk
        return evk.reshape(self.L, self.L + 1, 2, self.N)

    def tensor(self, a, b, level=None) -> np.ndarray:
        level = self.L if level is None else level
        a, ap = _u64(a)
        b, bp = _u64(b)
        d = np.zeros(3 * level * self.N, dtype=np.uint64)
        lib().orc_tensor(self._p, ap, bp, level, d.ctypes.data_as(C.POINTER(C.c_uint64)))
        return d

    def key_switch(self, d2, level=None, evk=None) -> np.ndarray:
        level = self.L if level is None else level
        e, ep = _u64(self.evk if evk is None else evk)
        d2, dp = _u64(d2)
        acc = np.zeros(2 * (level + 1) * self.N, dtype=np.uint64)
        lib().orc_key_switch(self._p, ep, dp, level, acc.ctypes.data_as(C.POINTER(C.c_uint64)))
        return acc

    def mod_down(self, acc, level=None) -> np.ndarray:
        level = self.L if level is None else level
        acc, ap = _u64(acc)
        out = np.zeros(2 * level * self.N, dtype=np.uint64)
        lib().orc_mod_down(self._p, ap, level, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    def mul(self, a, b, level=None, evk=None) -> np.ndarray:
        """Relinearized product of two ciphertexts at one level (scale = product of scales)."""
        level = self.L if level is None else level
        e, ep = _u64(self.evk if evk is None else evk)
        a, ap = _u64(a)
        b, bp = _u64(b)
        out = np.zeros(2 * level * self.N, dtype=np.uint64)
        lib().orc_mul(self._p, ep, ap, bp, level, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    # -- caches -------------------------------------------------------------------
    def radix_entries(self, r: int, D: int, cache_seed) -> np.ndarray:
        k, kp = _seed(cache_seed)
        pk, pkp = _u64(self.pk)
        out = np.zeros((D + 1, self.ct_words()), dtype=np.uint64)
        lib().orc_radix_entries(self._p, pkp, r, D, kp, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    def radix_encrypt(self, entries, r: int, D: int, p: int, job_seed, t: int) -> np.ndarray:
        e, ep = _u64(entries)
        k, kp = _seed(job_seed)
        out = np.zeros(self.ct_words(), dtype=np.uint64)
        rc = lib().orc_radix_encrypt(self._p, ep, r, D, int(p), kp, t, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        if rc:
            raise ValueError("pixel not representable with D digits")
        return out

    @staticmethod
    def histogram(px) -> np.ndarray:
        px = np.ascontiguousarray(px, dtype=np.uint8).reshape(-1)
        h = np.zeros(256, dtype=np.uint64)
        lib().orc_histogram(px.ctypes.data_as(C.POINTER(C.c_uint8)), len(px), h.ctypes.data_as(C.POINTER(C.c_uint64)))
        return h

    @staticmethod
    def topk(h, k: int) -> list[int]:
        h, hp = _u64(h)
        vals = np.zeros(256, dtype=np.int32)
        n = lib().orc_topk(hp, k, vals.ctypes.data_as(C.POINTER(C.c_int)))
        return [int(v) for v in vals[:n]]

    def value_entry(self, value: int, cache_seed) -> np.ndarray:
        k, kp = _seed(cache_seed)
        pk, pkp = _u64(self.pk)
        out = np.zeros(self.ct_words(), dtype=np.uint64)
        lib().orc_value_entry(self._p, pkp, int(value), kp, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    def pool_entry(self, u: int, cache_seed) -> np.ndarray:
        k, kp = _seed(cache_seed)
        pk, pkp = _u64(self.pk)
        out = np.zeros(self.ct_words(), dtype=np.uint64)
        lib().orc_pool_entry(self._p, pkp, int(u), kp, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    @staticmethod
    def pool_pick(job_seed, t: int, npool: int) -> int:
        k, kp = _seed(job_seed)
        return int(lib().orc_pool_pick(kp, t, npool))

    def value_encrypt(self, value_ct, pool, npool: int, p: int, job_seed, t: int) -> np.ndarray:
        """value_ct: the cached Enc(p), or None for a value outside the cache."""
        k, kp = _seed(job_seed)
        pk, pkp = _u64(self.pk)
        if value_ct is None:
            vp = None
        else:
            value_ct, vp = _u64(value_ct)
        pool_arr, pp = _u64(pool if pool is not None else np.zeros(1, dtype=np.uint64))
        out = np.zeros(self.ct_words(), dtype=np.uint64)
        lib().orc_value_encrypt(self._p, pkp, vp, pp, npool, int(p), kp, t, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    # -- image operations -------------------------------------------------------------
    def mean_filter_pixel(self, img_cts, H: int, W: int, k: int, y: int, x: int, level=None, scale=None):
        level = self.L if level is None else level
        scale = self.scale if scale is None else scale
        img, ip = _u64(img_cts)
        out = np.zeros(2 * (level - 1) * self.N, dtype=np.uint64)
        sc = C.c_double(0)
        rc = lib().orc_mean_filter_pixel(self._p, ip, H, W, level, scale, k, y, x,
                                         out.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(sc))
        if rc:
            raise ValueError("mean filter failed: %d" % rc)
        return out, sc.value


def num_threads() -> int:
    return int(lib().orc_num_threads())
