"""Python binding of libckks_mi355x.so, the MI355X (gfx950) pixel-level CKKS library.

Argument marshalling only: every computation runs in the library's HIP kernels, and
PyTorch supplies device memory and streams.  The functions carry the names of the C
ABI in include/ckks_mi355x.h; `Context` bundles them for convenience.  Nothing here
falls back to the CPU: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libckks_mi355x.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ckks_mi355x.h")

CKKS_OK = 0
CKKS_PENDING = 1
ERRORS = {
    -1: "CKKS_EINVAL", -2: "CKKS_ENOMEM", -3: "CKKS_ENOMEM_BUDGET", -4: "CKKS_EDEVICE", -5: "CKKS_ELEVEL",
    -6: "CKKS_ESCALE", -7: "CKKS_ECACHE", -8: "CKKS_EUNSUPPORTED", -9: "CKKS_ESTATE", -10: "CKKS_ECANCELED", -11: "CKKS_EIO",
}
ERRORS_BY_NAME = {v: k for k, v in ERRORS.items()}
CKKS_CACHE_RADIX, CKKS_CACHE_VALUE_TOPK, CKKS_CACHE_VALUE_FULL = 1, 2, 3


class CkksError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "CKKS_E?"), code, message))
        self.code = code
        self.name = ERRORS.get(code, "CKKS_E?")


class ckks_params_t(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("num_primes", C.c_uint32), ("prime_bits", C.c_uint32),
                ("log_scale", C.c_uint32), ("sigma", C.c_double), ("gauss_bound", C.c_uint32),
                ("reserved", C.c_uint32), ("primes", C.POINTER(C.c_uint64))]


class ckks_ct_batch_t(C.Structure):
    _fields_ = [("data", C.c_void_p), ("count", C.c_uint64), ("level", C.c_uint32), ("reserved", C.c_uint32),
                ("scale", C.c_double)]


class ckks_cache_desc_t(C.Structure):
    _fields_ = [("kind", C.c_int32), ("base", C.c_uint32), ("digits", C.c_uint32), ("topk", C.c_uint32),
                ("zero_pool", C.c_uint32)]


class ckks_server_config_t(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_inflight", C.c_uint32), ("filter_k", C.c_uint32),
                ("cache", C.c_void_p), ("max_job_pixels", C.c_uint64), ("tile_bytes", C.c_uint64),
                ("max_bypass", C.c_uint32), ("reserved", C.c_uint32)]


class ckks_job_result_t(C.Structure):
    _fields_ = [("job_id", C.c_uint64), ("status", C.c_int32), ("height", C.c_uint32), ("width", C.c_uint32),
                ("t_submit_us", C.c_double), ("t_admit_us", C.c_double), ("t_done_us", C.c_double),
                ("gpu_ms", C.c_double)]


class ckks_server_stats_t(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("queued", C.c_uint64), ("inflight", C.c_uint64), ("arena_bytes", C.c_uint64),
                ("inflight_bytes", C.c_uint64), ("peak_inflight_bytes", C.c_uint64),
                ("peak_inflight_jobs", C.c_uint32), ("reserved", C.c_uint32), ("canceled", C.c_uint64),
                ("backfilled", C.c_uint64)]


class ckks_tune_report_t(C.Structure):
    _fields_ = [("encrypt_width", C.c_uint32), ("decrypt_width", C.c_uint32), ("trial_cts", C.c_uint32),
                ("mul_width", C.c_uint32), ("encrypt_ms", C.c_double * 3), ("decrypt_ms", C.c_double * 3),
                ("mul_ms", C.c_double * 3), ("row_wgs_per_cu", C.c_uint32), ("gather_wgs_per_cu", C.c_uint32),
                ("row_ms", C.c_double * 5), ("gather_ms", C.c_double * 5)]


class ckks_pipeline_config_t(C.Structure):
    _fields_ = [("tile_rows", C.c_uint32), ("streams", C.c_uint32), ("filter_k", C.c_uint32),
                ("reserved", C.c_uint32)]


class ckks_batch_config_t(C.Structure):
    _fields_ = [("chunk_cts", C.c_uint64), ("use_graph", C.c_uint32), ("reserved", C.c_uint32)]


_lib = None

_SIGS = {
    "ckks_last_error": (C.c_char_p, []),
    "ckks_params_resolve": (C.c_int, [C.POINTER(ckks_params_t), C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)]),
    "ckks_host_cdt_table": (C.c_int, [C.POINTER(ckks_params_t), C.POINTER(C.c_uint64), C.c_uint32]),
    "ckks_host_encode_table": (C.c_int, [C.POINTER(ckks_params_t), C.POINTER(C.c_double), C.c_uint64]),
    "ckks_context_create": (C.c_int, [C.POINTER(ckks_params_t), C.c_int, C.POINTER(C.c_void_p)]),
    "ckks_context_destroy": (None, [C.c_void_p]),
    "ckks_ct_bytes": (C.c_uint64, [C.c_void_p, C.c_uint32]),
    "ckks_context_set_ntt_width": (C.c_int, [C.c_void_p, C.c_uint32]),
    "ckks_context_get_ntt_width": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32)]),
    "ckks_context_set_launch_shapes": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32]),
    "ckks_context_get_launch_shapes": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]),
    "ckks_tune_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "ckks_tune_load": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int)]),
    "ckks_context_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "ckks_keygen": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "ckks_keys_export": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]),
    "ckks_keys_import": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]),
    "ckks_relin_keygen": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "ckks_relin_keys_export": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "ckks_mul": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.POINTER(ckks_ct_batch_t),
                           C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_encrypt_pixels": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64), C.c_uint64,
                                      C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_cache_build": (C.c_int, [C.c_void_p, C.POINTER(ckks_cache_desc_t), C.c_void_p, C.c_uint64,
                                   C.POINTER(C.c_uint64), C.POINTER(C.c_void_p), C.c_void_p]),
    "ckks_cache_destroy": (None, [C.c_void_p]),
    "ckks_cache_entries": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32)]),
    "ckks_cache_export": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_uint64)]),
    "ckks_cache_import": (C.c_int, [C.c_void_p, C.POINTER(ckks_cache_desc_t), C.c_uint32, C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_void_p)]),
    "ckks_encrypt_cached": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64),
                                      C.c_uint64, C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_encrypt_cached_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64),
                                              C.c_uint64, C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_encrypt_cached_noalloc_max_pixels": (C.c_uint64, [C.c_void_p]),
    "ckks_add": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.POINTER(ckks_ct_batch_t),
                           C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_sub": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.POINTER(ckks_ct_batch_t),
                           C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_mul_const": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.c_double, C.POINTER(ckks_ct_batch_t),
                                 C.c_void_p]),
    "ckks_add_const": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.c_void_p, C.c_double, C.c_void_p]),
    "ckks_rescale": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_mean_filter": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.c_uint32, C.c_uint32, C.c_uint32,
                                   C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_decrypt_pixels": (C.c_int, [C.c_void_p, C.POINTER(ckks_ct_batch_t), C.c_void_p, C.c_void_p]),
    "ckks_stream_sync": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ckks_stream_status": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ckks_image_pipeline": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32,
                                      C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(ckks_pipeline_config_t),
                                      C.c_void_p, C.c_void_p]),
    "ckks_autotune": (C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(ckks_tune_report_t)]),
    "ckks_batch_plan_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(ckks_batch_config_t),
                                         C.POINTER(C.c_void_p)]),
    "ckks_batch_run": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                 C.c_uint32, C.POINTER(C.c_uint64), C.c_uint64, C.c_void_p,
                                 C.POINTER(ckks_ct_batch_t), C.c_void_p]),
    "ckks_batch_plan_destroy": (None, [C.c_void_p]),
    "ckks_server_create": (C.c_int, [C.c_void_p, C.POINTER(ckks_server_config_t), C.POINTER(C.c_void_p)]),
    "ckks_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint64),
                                     C.c_uint64, C.c_void_p, C.POINTER(C.c_uint64)]),
    "ckks_server_poll": (C.c_int, [C.c_void_p, C.POINTER(ckks_job_result_t), C.c_uint32, C.POINTER(C.c_uint32),
                                   C.c_int32]),
    "ckks_server_drain": (C.c_int, [C.c_void_p]),
    "ckks_server_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ckks_server_inject_failure": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32]),
    "ckks_job_bytes": (C.c_uint64, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]),
    "ckks_server_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ckks_server_stats_t)]),
    "ckks_server_destroy": (None, [C.c_void_p]),
}


def lib():
    """Load the HIP library (after torch, so both share one HIP runtime).  Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libckks_mi355x.so is not built: run __graft_entry__.build() or "
                              "python paper_2409_03568_amd/build_native.py")
        import torch  # noqa: F401  (loads the HIP runtime first)

        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ckks_last_error() -> str:
    return lib().ckks_last_error().decode()


def _check(rc: int):
    if rc != CKKS_OK:
        raise CkksError(rc, ckks_last_error())


def _seed(seed):
    arr = (C.c_uint64 * 2)(int(seed[0]) & (2**64 - 1), int(seed[1]) & (2**64 - 1))
    return arr


def _stream(stream):
    if stream is None:
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


# ---------------------------------------------------------------------------
# parameters and host-only queries
# ---------------------------------------------------------------------------
def ckks_params(log_n: int, num_primes: int, prime_bits: int, log_scale: int, sigma: float = 3.2,
                gauss_bound: int = 0, primes=None) -> ckks_params_t:
    p = ckks_params_t(log_n, num_primes, prime_bits, log_scale, sigma, gauss_bound, 0, None)
    if primes is not None:
        arr = (C.c_uint64 * len(primes))(*[int(x) for x in primes])
        p._primes_keep = arr
        p.primes = C.cast(arr, C.POINTER(C.c_uint64))
    return p


def ckks_params_resolve(params: ckks_params_t):
    q = (C.c_uint64 * params.num_primes)()
    B = C.c_uint32(0)
    _check(lib().ckks_params_resolve(C.byref(params), q, C.byref(B)))
    return [int(x) for x in q], int(B.value)


def ckks_host_cdt_table(params: ckks_params_t) -> np.ndarray:
    _, B = ckks_params_resolve(params)
    out = np.zeros(max(1, 2 * B), dtype=np.uint64)
    _check(lib().ckks_host_cdt_table(C.byref(params), out.ctypes.data_as(C.POINTER(C.c_uint64)), len(out)))
    return out[: 2 * B]


def ckks_host_encode_table(params: ckks_params_t) -> np.ndarray:
    out = np.zeros(1 << params.log_n, dtype=np.float64)
    _check(lib().ckks_host_encode_table(C.byref(params), out.ctypes.data_as(C.POINTER(C.c_double)), len(out)))
    return out


# ---------------------------------------------------------------------------
# ciphertext batches in torch device memory
# ---------------------------------------------------------------------------
@dataclass
class Ciphertexts:
    """count ciphertexts [count][2][level][N] as uint64 residues (stored in an int64 tensor)."""

    data: "object"  # torch.Tensor, int64, on the context's device
    level: int
    scale: float

    @property
    def count(self) -> int:
        return int(self.data.shape[0])

    def batch(self) -> ckks_ct_batch_t:
        return ckks_ct_batch_t(self.data.data_ptr() if self.count else None, self.count, self.level, 0, self.scale)

    def out_batch(self) -> ckks_ct_batch_t:
        """Descriptor of this tensor as an output buffer: its real capacity (rows of the
        tensor's own level), which the library checks against the result's size."""
        d = self.data
        if d.dim() != 4 or not d.is_contiguous():
            raise ValueError("an output tensor must be a contiguous [count][2][level][N] tensor")
        return ckks_ct_batch_t(d.data_ptr() if d.shape[0] else None, int(d.shape[0]), int(d.shape[2]), 0, self.scale)

    def to_numpy(self) -> np.ndarray:
        return self.data.cpu().numpy().view(np.uint64)

    def __getitem__(self, idx) -> "Ciphertexts":
        d = self.data[idx]
        if d.dim() == 3:
            d = d.unsqueeze(0)
        return Ciphertexts(d, self.level, self.scale)


class Context:
    """A parameter set on one GPU with its keys (wraps ckks_context_create)."""

    def __init__(self, log_n: int, num_primes: int, prime_bits: int, log_scale: int, sigma: float = 3.2,
                 gauss_bound: int = 0, primes=None, device: int = 0):
        import torch

        self.params = ckks_params(log_n, num_primes, prime_bits, log_scale, sigma, gauss_bound, primes)
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        _check(lib().ckks_context_create(C.byref(self.params), device, C.byref(h)))
        self.handle = h
        self.N = 1 << log_n
        self.L = num_primes
        self.scale = float(2.0**log_scale)
        q = (C.c_uint64 * num_primes)()
        _check(lib().ckks_context_info(self.handle, None, None, None, q))
        self.q = [int(x) for x in q]

    def close(self):
        if getattr(self, "handle", None):
            lib().ckks_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning -------------------------------------------------------------
    def set_ntt_width(self, values_per_thread: int):
        _check(lib().ckks_context_set_ntt_width(self.handle, values_per_thread))

    def ntt_width(self) -> int:
        v = C.c_uint32(0)
        _check(lib().ckks_context_get_ntt_width(self.handle, C.byref(v)))
        return int(v.value)

    # -- memory -------------------------------------------------------------
    def ct_bytes(self, level: int | None = None) -> int:
        return int(lib().ckks_ct_bytes(self.handle, self.L if level is None else level))

    def empty(self, n: int, level: int | None = None) -> Ciphertexts:
        import torch

        level = self.L if level is None else level
        return Ciphertexts(torch.empty((n, 2, level, self.N), dtype=torch.int64, device=self.device), level,
                           self.scale)

    def from_numpy(self, arr, level: int | None = None, scale: float | None = None) -> Ciphertexts:
        import torch

        level = self.L if level is None else level
        a = np.ascontiguousarray(arr, dtype=np.uint64).reshape(-1, 2, level, self.N).view(np.int64)
        return Ciphertexts(torch.from_numpy(a.copy()).to(self.device), level, self.scale if scale is None else scale)

    # -- keys ---------------------------------------------------------------
    def keygen(self, seed):
        _check(lib().ckks_keygen(self.handle, _seed(seed)))

    def keys_export(self):
        s = np.zeros(self.N, dtype=np.int64)
        pk = np.zeros(2 * self.L * self.N, dtype=np.uint64)
        _check(lib().ckks_keys_export(self.handle, s.ctypes.data_as(C.POINTER(C.c_int64)),
                                      pk.ctypes.data_as(C.POINTER(C.c_uint64))))
        return s, pk

    def keys_import(self, s, pk):
        s = np.ascontiguousarray(s, dtype=np.int64)
        pk = np.ascontiguousarray(pk, dtype=np.uint64).reshape(-1)
        _check(lib().ckks_keys_import(self.handle, s.ctypes.data_as(C.POINTER(C.c_int64)),
                                      pk.ctypes.data_as(C.POINTER(C.c_uint64))))

    def relin_keygen(self, seed):
        _check(lib().ckks_relin_keygen(self.handle, _seed(seed)))

    def relin_keys_export(self):
        """(evk[L][L+1][2][N] as uint64, the special prime qP)."""
        evk = np.zeros(self.L * (self.L + 1) * 2 * self.N, dtype=np.uint64)
        qP = C.c_uint64(0)
        _check(lib().ckks_relin_keys_export(self.handle, evk.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(qP)))
        return evk.reshape(self.L, self.L + 1, 2, self.N), int(qP.value)

    # -- encryption -------------------------------------------------------------
    def encrypt_pixels(self, px, seed, first_index: int = 0, out: Ciphertexts | None = None,
                       stream=None) -> Ciphertexts:
        n = int(px.numel())
        out = self.empty(n) if out is None else out
        b = out.out_batch()
        _check(lib().ckks_encrypt_pixels(self.handle, _ptr(px), n, _seed(seed), first_index, C.byref(b),
                                         _stream(stream)))
        out.level, out.scale = int(b.level), float(b.scale)
        return out

    def cache_import(self, kind: int, values, entries, pool=None, base: int = 0, digits: int = 0, topk: int = 0,
                     zero_pool: int = 0) -> "Cache":
        """Install a cache from host arrays laid out as Cache.export returns them."""
        vals = np.ascontiguousarray(values, dtype=np.uint32)
        ent = np.ascontiguousarray(entries, dtype=np.uint64).reshape(-1)
        pl = None if pool is None else np.ascontiguousarray(pool, dtype=np.uint64).reshape(-1)
        if ent.size != vals.size * 2 * self.L * self.N:
            raise ValueError("entries must hold len(values) ciphertexts of level L")
        if pl is not None and pl.size != zero_pool * 2 * self.L * self.N:
            raise ValueError("pool must hold zero_pool ciphertexts of level L")
        desc = ckks_cache_desc_t(kind, base, digits, topk, zero_pool)
        h = C.c_void_p()
        _check(lib().ckks_cache_import(self.handle, C.byref(desc), vals.size, vals.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       ent.ctypes.data_as(C.POINTER(C.c_uint64)),
                                       None if pl is None else pl.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(h)))
        return Cache(h, self, kind)

    def cache_build(self, kind: int, base: int = 0, digits: int = 0, topk: int = 0, zero_pool: int = 0,
                    scan_px=None, seed=(0, 0), stream=None) -> "Cache":
        desc = ckks_cache_desc_t(kind, base, digits, topk, zero_pool)
        h = C.c_void_p()
        n_scan = 0 if scan_px is None else int(scan_px.numel())
        _check(lib().ckks_cache_build(self.handle, C.byref(desc), _ptr(scan_px), n_scan, _seed(seed), C.byref(h),
                                      _stream(stream)))
        return Cache(h, self, kind)

    def encrypt_cached(self, cache: "Cache", px, seed, first_index: int = 0, out: Ciphertexts | None = None,
                       stream=None) -> Ciphertexts:
        n = int(px.numel())
        out = self.empty(n) if out is None else out
        b = out.out_batch()
        _check(lib().ckks_encrypt_cached(self.handle, cache.handle, _ptr(px), n, _seed(seed), first_index,
                                         C.byref(b), _stream(stream)))
        out.level, out.scale = int(b.level), float(b.scale)
        return out

    # -- homomorphic operations ---------------------------------------------------
    def _binary(self, fn, a: Ciphertexts, b: Ciphertexts, out, stream):
        out = self.empty(a.count, a.level) if out is None else out
        ba, bb, bo = a.batch(), b.batch(), out.out_batch()
        _check(fn(self.handle, C.byref(ba), C.byref(bb), C.byref(bo), _stream(stream)))
        out.level, out.scale = int(bo.level), float(bo.scale)
        return out

    def add(self, a, b, out=None, stream=None) -> Ciphertexts:
        return self._binary(lib().ckks_add, a, b, out, stream)

    def sub(self, a, b, out=None, stream=None) -> Ciphertexts:
        return self._binary(lib().ckks_sub, a, b, out, stream)

    def mul(self, a, b, out=None, stream=None) -> Ciphertexts:
        return self._binary(lib().ckks_mul, a, b, out, stream)

    def mul_const(self, a: Ciphertexts, c: float, out=None, stream=None) -> Ciphertexts:
        out = self.empty(a.count, a.level) if out is None else out
        ba, bo = a.batch(), out.out_batch()
        _check(lib().ckks_mul_const(self.handle, C.byref(ba), float(c), C.byref(bo), _stream(stream)))
        out.level, out.scale = int(bo.level), float(bo.scale)
        return out

    def add_const(self, a: Ciphertexts, b=0.0, per_ct=None, stream=None) -> Ciphertexts:
        ba = a.batch()
        _check(lib().ckks_add_const(self.handle, C.byref(ba), _ptr(per_ct), float(b), _stream(stream)))
        return a

    def rescale(self, a: Ciphertexts, out=None, stream=None) -> Ciphertexts:
        out = self.empty(a.count, a.level - 1) if out is None else out
        ba, bo = a.batch(), out.out_batch()
        _check(lib().ckks_rescale(self.handle, C.byref(ba), C.byref(bo), _stream(stream)))
        out.level, out.scale = int(bo.level), float(bo.scale)
        return out

    def mean_filter(self, img: Ciphertexts, H: int, W: int, k: int, out=None, stream=None) -> Ciphertexts:
        out = self.empty(img.count, img.level - 1) if out is None else out
        bi, bo = img.batch(), out.out_batch()
        _check(lib().ckks_mean_filter(self.handle, C.byref(bi), H, W, k, C.byref(bo), _stream(stream)))
        out.level, out.scale = int(bo.level), float(bo.scale)
        return out

    def decrypt_pixels(self, cts: Ciphertexts, out=None, stream=None):
        import torch

        out = torch.empty(cts.count, dtype=torch.float64, device=self.device) if out is None else out
        b = cts.batch()
        _check(lib().ckks_decrypt_pixels(self.handle, C.byref(b), _ptr(out), _stream(stream)))
        return out

    def stream_sync(self, stream=None):
        _check(lib().ckks_stream_sync(self.handle, _stream(stream)))

    def stream_done(self, stream=None) -> bool:
        """Non-blocking: True when the stream's work has completed (ckks_stream_status)."""
        rc = lib().ckks_stream_status(self.handle, _stream(stream))
        if rc == CKKS_PENDING:
            return False
        _check(rc)
        return True

    def image_pipeline(self, px, H: int, W: int, seed, k: int, tile_rows: int, streams: int = 1,
                       cache: "Cache | None" = None, first_index: int = 0, out=None, stream=None):
        """Encrypt -> k x k mean filter -> decrypt of an H x W image in row tiles (streams=1: a
        ring of encrypted rows on the caller's stream; 3: three stage streams with recomputed
        halos); returns the decrypted filtered pixels (H*W doubles on the device)."""
        import torch

        out = torch.empty(H * W, dtype=torch.float64, device=px.device) if out is None else out
        cfg = ckks_pipeline_config_t(int(tile_rows), int(streams), int(k), 0)
        _check(lib().ckks_image_pipeline(self.handle, cache.handle if cache is not None else None, _ptr(px), H, W,
                                         _seed(seed), int(first_index), C.byref(cfg), _ptr(out), _stream(stream)))
        return out

    def autotune(self, trial_cts: int = 4096) -> dict:
        """Time the NTT register blockings for encryption, decryption and (with
        key-switching keys) the product, and the launch shapes of the row-wise kernels and
        the value-cache gather; keep the fastest of each (ckks_autotune)."""
        r = ckks_tune_report_t()
        _check(lib().ckks_autotune(self.handle, int(trial_cts), C.byref(r)))
        out = {"encrypt_width": r.encrypt_width, "decrypt_width": r.decrypt_width, "trial_cts": r.trial_cts,
               "encrypt_ms": {8: r.encrypt_ms[0], 16: r.encrypt_ms[1], 32: r.encrypt_ms[2]},
               "decrypt_ms": {8: r.decrypt_ms[0], 16: r.decrypt_ms[1], 32: r.decrypt_ms[2]},
               "row_wgs_per_cu": r.row_wgs_per_cu, "gather_wgs_per_cu": r.gather_wgs_per_cu,
               "row_ms": dict(zip((0, 2, 4, 8, 16), list(r.row_ms))),
               "gather_ms": dict(zip((2, 4, 8, 16, 32), list(r.gather_ms)))}
        if r.mul_width:
            out["mul_width"] = r.mul_width
            out["mul_ms"] = {8: r.mul_ms[0], 16: r.mul_ms[1], 32: r.mul_ms[2]}
        return out

    def set_launch_shapes(self, row_wgs: int, gather_wgs: int):
        _check(lib().ckks_context_set_launch_shapes(self.handle, int(row_wgs), int(gather_wgs)))

    def launch_shapes(self) -> tuple:
        """(row_wgs, gather_wgs): workgroups per compute unit of the row-wise kernels (0: one
        per row) and of the value-cache gather."""
        r, g = C.c_uint32(0), C.c_uint32(0)
        _check(lib().ckks_context_get_launch_shapes(self.handle, C.byref(r), C.byref(g)))
        return r.value, g.value

    def tune_save(self, path: str):
        """Store this context's tuned settings in the tuning file at path (ckks_tune_save)."""
        _check(lib().ckks_tune_save(self.handle, os.fsencode(path)))

    def tune_load(self, path: str) -> bool:
        """Apply the tuning file's settings for this device and ring shape; False if none."""
        found = C.c_int(0)
        _check(lib().ckks_tune_load(self.handle, os.fsencode(path), C.byref(found)))
        return bool(found.value)


class Cache:
    def __init__(self, handle, ctx: Context, kind: int):
        self.handle = handle
        self.ctx = ctx
        self.kind = kind

    def entries(self) -> int:
        n = C.c_uint32(0)
        _check(lib().ckks_cache_entries(self.handle, C.byref(n)))
        return int(n.value)

    def export(self, pool_size: int = 0):
        """(values[n], entries[n][2][L][N], pool[pool_size][2][L][N]) as numpy arrays."""
        n = self.entries()
        S = 2 * self.ctx.L * self.ctx.N
        vals = np.zeros(max(n, 1), dtype=np.uint32)
        ent = np.zeros(max(n, 1) * S, dtype=np.uint64)
        pool = np.zeros(max(pool_size, 1) * S, dtype=np.uint64)
        _check(lib().ckks_cache_export(self.handle, vals.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       ent.ctypes.data_as(C.POINTER(C.c_uint64)),
                                       pool.ctypes.data_as(C.POINTER(C.c_uint64)) if pool_size else None))
        return vals[:n], ent[: n * S].reshape(n, S), pool[: pool_size * S].reshape(pool_size, S)

    def close(self):
        if getattr(self, "handle", None):
            lib().ckks_cache_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Batched images: flat pixels, per-image brightness, decrypted values; ciphertexts go
    through a ring buffer of chunk_cts ciphertexts; optional HIP-graph replay."""

    def __init__(self, ctx: Context, cache: "Cache | None", chunk_cts: int, use_graph: bool = False):
        cfg = ckks_batch_config_t(int(chunk_cts), 1 if use_graph else 0, 0)
        h = C.c_void_p()
        _check(lib().ckks_batch_plan_create(ctx.handle, cache.handle if cache is not None else None, C.byref(cfg),
                                            C.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.cache = cache

    def run(self, px, seg_end, seg_b, seed, first_index: int = 0, out=None, stream=None,
            cts_out: "Ciphertexts | None" = None):
        """Decrypted pixel + brightness values; with cts_out (n ciphertexts of level L) every
        brightened ciphertext is also kept there."""
        import torch

        n = px.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=px.device)
        se = np.ascontiguousarray(seg_end, dtype=np.uint64)
        sb = np.ascontiguousarray(seg_b, dtype=np.float64)
        cb = cts_out.out_batch() if cts_out is not None else None
        _check(lib().ckks_batch_run(self.handle, _ptr(px), n, se.ctypes.data_as(C.POINTER(C.c_uint64)),
                                    sb.ctypes.data_as(C.POINTER(C.c_double)), len(se), _seed(seed), int(first_index),
                                    _ptr(out), C.byref(cb) if cb is not None else None, _stream(stream)))
        if cts_out is not None:
            cts_out.level, cts_out.scale = int(cb.level), float(cb.scale)
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().ckks_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_bytes(ctx: Context, H: int, W: int, filter_k: int, cache: "Cache | None" = None, tile_bytes: int = 0) -> int:
    """Arena bytes a server job of H x W pixels takes (ckks_job_bytes): pixels, decrypted
    values and one row tile's buffers, as the server's admission counts them."""
    return int(lib().ckks_job_bytes(ctx.handle, cache.handle if cache is not None else None, int(H), int(W),
                                    int(filter_k), int(tile_bytes)))


class Server:
    """Serving runtime over a context: jobs of encrypt -> k x k mean filter -> decrypt,
    admitted in arrival order by device bytes into an arena of `hbm_budget_bytes` (younger
    jobs may start ahead of a waiting one, at most `max_bypass` times per job), at most
    `max_inflight` running at once, each on its own stream."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_inflight: int = 4, filter_k: int = 3,
                 cache: "Cache | None" = None, max_job_pixels: int = 0, tile_bytes: int = 0, max_bypass: int = 0):
        cfg = ckks_server_config_t(int(hbm_budget_bytes), int(max_inflight), int(filter_k),
                                   cache.handle if cache is not None else None, int(max_job_pixels), int(tile_bytes),
                                   int(max_bypass), 0)
        h = C.c_void_p()
        _check(lib().ckks_server_create(ctx.handle, C.byref(cfg), C.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.cache = cache
        self.filter_k = int(filter_k)
        self.tile_bytes = int(tile_bytes)
        self._outputs = {}  # job id -> (pixels copy owner, output array): kept alive until polled

    def job_bytes(self, H: int, W: int) -> int:
        return job_bytes(self.ctx, H, W, self.filter_k, self.cache, self.tile_bytes)

    def cancel(self, job_id: int):
        """Cancel a queued job (ckks_server_cancel); it is polled with status CKKS_ECANCELED."""
        _check(lib().ckks_server_cancel(self.handle, int(job_id)))

    def inject_failure(self, job_id: int, status: int = -4):
        """Make a queued job fail when admitted (ckks_server_inject_failure), for failure tests."""
        _check(lib().ckks_server_inject_failure(self.handle, int(job_id), int(status)))

    def submit(self, img, seed, first_index: int = 0) -> int:
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W = img.shape
        out = np.empty(H * W, dtype=np.float64)
        jid = C.c_uint64(0)
        _check(lib().ckks_server_submit(self.handle, img.ctypes.data, H, W, _seed(seed), int(first_index),
                                        out.ctypes.data, C.byref(jid)))
        self._outputs[int(jid.value)] = out
        return int(jid.value)

    def poll(self, max_results: int = 64, wait_ms: int = 0):
        """List of finished jobs: dicts with id, status, times (us) and the decrypted pixels."""
        buf = (ckks_job_result_t * max(1, max_results))()
        n = C.c_uint32(0)
        _check(lib().ckks_server_poll(self.handle, buf, max_results, C.byref(n), int(wait_ms)))
        res = []
        for r in buf[: n.value]:
            out = self._outputs.pop(int(r.job_id))
            res.append({"id": int(r.job_id), "status": int(r.status), "H": int(r.height), "W": int(r.width),
                        "t_submit_us": r.t_submit_us, "t_admit_us": r.t_admit_us, "t_done_us": r.t_done_us,
                        "gpu_ms": r.gpu_ms, "pixels": out.reshape(r.height, r.width)})
        return res

    def drain(self):
        _check(lib().ckks_server_drain(self.handle))

    def stats(self) -> dict:
        st = ckks_server_stats_t()
        _check(lib().ckks_server_stats_get(self.handle, C.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in ckks_server_stats_t._fields_ if f != "reserved"}

    def close(self):
        if getattr(self, "handle", None):
            lib().ckks_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
