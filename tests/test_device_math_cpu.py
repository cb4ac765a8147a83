"""CPU checks of the HIP library's device arithmetic, run through a host emulation.

The library's FP64 modular arithmetic, Philox samplers and per-pass NTT functions are
host-callable; tests/native/device_math_emulation.cpp drives them for one emulated
workgroup.  Results are compared with the CPU oracle and with Python big integers.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "device_math_emulation.cpp")
LIB = os.path.join(HERE, "native", "libdevice_math_emulation.so")
DEPS = [SRC] + [os.path.join(ROOT, "paper_2409_03568_amd", "csrc", f) for f in
                ("host_math.cpp", "host_math.hpp", "ntt.hpp", "modarith.hpp", "philox.hpp")]


def _build():
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in DEPS):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-ffp-contract=off", "-o", tmp, SRC, os.path.join(ROOT, "paper_2409_03568_amd", "csrc", "host_math.cpp")]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    L = C.CDLL(_build())
    u64p, i64p = C.POINTER(C.c_uint64), C.POINTER(C.c_int64)
    L.emu_negacyclic.argtypes = [i64p, u64p, u64p, C.c_int, C.c_uint64, C.c_uint64, C.c_int, C.c_int, C.c_int]
    L.emu_negacyclic.restype = C.c_int
    L.emu_max_abs.restype = C.c_double
    L.emu_lds_bijective.restype = C.c_int
    L.emu_wave_local_ok.restype = C.c_int
    L.emu_wave_local_count.restype = C.c_int
    for f in ("emu_mulmod",):
        getattr(L, f).argtypes = [C.c_double, C.c_double, C.c_double]
        getattr(L, f).restype = C.c_double
    for f in ("emu_reduce", "emu_canon", "emu_center"):
        getattr(L, f).argtypes = [C.c_double, C.c_double]
        getattr(L, f).restype = C.c_double
    L.emu_mul_shoup.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
    L.emu_mul_shoup.restype = C.c_uint64
    L.emu_mod_i64.argtypes = [C.c_int64, C.c_uint64]
    L.emu_mod_i64.restype = C.c_uint64
    L.emu_residue_of_double.argtypes = [C.c_double, C.c_uint64]
    L.emu_residue_of_double.restype = C.c_uint64
    L.emu_philox.argtypes = [u64p, u64p, u64p]
    L.emu_ternary.argtypes = [C.c_uint64]
    L.emu_ternary.restype = C.c_int
    L.emu_gauss.argtypes = [C.c_uint64, C.c_double, C.c_int]
    L.emu_gauss.restype = C.c_int
    L.emu_fwd_mask.argtypes = [C.c_int, C.c_double, C.c_double]
    L.emu_fwd_mask.restype = C.c_uint32
    L.emu_inv_mask.argtypes = [C.c_int, C.c_double, C.c_double]
    L.emu_inv_mask.restype = C.c_uint32
    return L


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


@pytest.mark.parametrize("log_n,bits,logr", [(11, 30, 5), (12, 36, 5), (12, 36, 4), (12, 36, 3), (13, 50, 5),
                                            (13, 50, 4), (13, 50, 3), (13, 40, 4), (14, 50, 5), (14, 50, 4),
                                            (11, 49, 4), (11, 49, 3)])
def test_emulated_ntt_product_matches_oracle(emu, oracle_mod, log_n, bits, logr):
    N = 1 << log_n
    rng = np.random.default_rng(log_n * 100 + bits)
    rc = 0 if bits <= 40 else 1
    for q in oracle_mod.gen_primes(log_n, bits, 2):
        psi = oracle_mod.primitive_2n_root(q, log_n)
        cases = [
            ("ternary x uniform", rng.integers(-1, 2, N).astype(np.int64), rng.integers(0, q, N, dtype=np.uint64), 1),
            ("uniform x uniform", rng.integers(0, q, N, dtype=np.uint64).astype(np.int64),
             rng.integers(0, q, N, dtype=np.uint64), 0),
            ("all q-1", np.full(N, q - 1, dtype=np.int64), np.full(N, q - 1, dtype=np.uint64), 0),
            ("all -1 x all q-1", np.full(N, -1, dtype=np.int64), np.full(N, q - 1, dtype=np.uint64), 1),
        ]
        for name, a, b, small in cases:
            emu.emu_reset_max()
            c = np.zeros(N, dtype=np.uint64)
            st = emu.emu_negacyclic(a.ctypes.data_as(C.POINTER(C.c_int64)), _u64(b).ctypes.data_as(C.POINTER(C.c_uint64)),
                                    c.ctypes.data_as(C.POINTER(C.c_uint64)), log_n, q, psi, small, logr, rc)
            assert st == 0
            a_res = np.array([int(x) % q for x in a], dtype=np.uint64)
            ref = oracle_mod.negacyclic_mul(a_res, b, q, psi)
            assert np.array_equal(c, ref), (name, q)
            assert emu.emu_max_abs() < 2.0**52, name
            assert emu.emu_lds_bijective() == 1
            # exchanges run without a workgroup barrier keep every wave on its own LDS slots
            assert emu.emu_wave_local_ok() == 1
            if (log_n, logr) == (13, 3):
                assert emu.emu_wave_local_count() == 6  # 2 of the 4 exchanges in each of 3 transforms


def test_reduction_schedules(emu):
    # 36-bit primes never need a reduction inside a forward transform; 50-bit primes do
    assert emu.emu_fwd_mask(13, 2.0**36, 1.0) == 0
    assert emu.emu_inv_mask(13, 2.0**36, 2.0**36 + 4) == 0
    assert emu.emu_fwd_mask(13, 2.0**50, 2.0**50) != 0
    assert emu.emu_inv_mask(13, 2.0**50, 2.0**50 + 4) != 0
    # a schedule derived for a larger modulus reduces at least where a smaller one needs to
    for log_n in (11, 12, 13, 14):
        for small, big in ((2.0**36, 2.0**40), (2.0**45, 2.0**50)):
            for f, inb in ((emu.emu_fwd_mask, lambda q: 1.0), (emu.emu_fwd_mask, lambda q: q),
                           (emu.emu_inv_mask, lambda q: q + 4)):
                m_small, m_big = f(log_n, small, inb(small)), f(log_n, big, inb(big))
                # every prefix of stages of the big schedule has at least as many reductions
                order = range(log_n) if f is emu.emu_fwd_mask else range(log_n - 1, -1, -1)
                cs = cb = 0
                for s in order:
                    cs += (m_small >> s) & 1
                    cb += (m_big >> s) & 1
                    assert cb >= cs


def test_fp64_modular_arithmetic_exact(emu, oracle_mod):
    rng = np.random.default_rng(7)
    for bits in (20, 36, 49, 50):
        q = oracle_mod.gen_primes(12, bits, 1)[0]
        # forward-transform values reach 2^52 - 2^48 (the product precondition |a w / q| < 2^51)
        A = [0, 1, -1, q - 1, -(q - 1), 2**51 - 1, -(2**51 - 1), q // 2, -(q // 2), 2**52 - 2**48, -(2**52 - 2**48)]
        A += [int(x) for x in rng.integers(-(2**52) + 2**48, 2**52 - 2**48, 300)]
        W = [0, 1, -1, q // 2, -(q // 2), (q - 1) // 2]
        W += [int(x) for x in rng.integers(-(q // 2), q // 2 + 1, 30)]
        for a in A:
            for w in W[:12]:
                r = emu.emu_mulmod(float(a), float(w), float(q))
                assert r == int(r)
                assert (int(r) - a * w) % q == 0
                assert abs(r) <= q / 2 + abs(a * w) * 2.0**-52 + 1
        for x in A + [2**52 - 1, -(2**52 - 1)]:
            r = emu.emu_reduce(float(x), float(q))
            assert (int(r) - x) % q == 0 and abs(r) <= q / 2 + 1
        for x in [2**53 - 1, -(2**53 - 1), 2**53 - q, 2**52 + 12345] + [int(v) for v in rng.integers(2**52, 2**53, 50)]:
            r = emu.emu_reduce(float(x), float(q))  # exact integers below 2^53
            assert (int(r) - x) % q == 0 and abs(r) <= q / 2 + 2
            c = emu.emu_canon(float(x), float(q))
            assert c == x % q
            z = emu.emu_center(float(x), float(q))
            assert (int(z) - x) % q == 0 and -q / 2 < z <= q / 2


def test_integer_helpers(emu, oracle_mod):
    rng = np.random.default_rng(8)
    for bits in (36, 50):
        q = oracle_mod.gen_primes(13, bits, 1)[0]
        for _ in range(200):
            a = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
            w = int(rng.integers(0, q))
            assert emu.emu_mul_shoup(a, w, q) == (a * w) % q
            x = int(rng.integers(-(2**61), 2**61))
            assert emu.emu_mod_i64(x, q) == x % q
        for x in (0.0, 1.0, -1.0, 2.0**52 + 2, -(2.0**70) - 2.0**30, 2.0**100, 12345678912345.0, -987654321.0):
            assert emu.emu_residue_of_double(x, q) == int(x) % q


def test_device_philox_and_samplers_match_oracle(emu, oracle_mod):
    rng = np.random.default_rng(9)
    B = 19
    T = oracle_mod.cdt_table(3.2, B)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        out = np.zeros(4, dtype=np.uint64)
        emu.emu_philox(_u64(ctr).ctypes.data_as(C.POINTER(C.c_uint64)), _u64(key).ctypes.data_as(C.POINTER(C.c_uint64)),
                       out.ctypes.data_as(C.POINTER(C.c_uint64)))
        assert [int(x) for x in out] == oracle_mod.philox(ctr, key)
        for w in out:
            w = int(w)
            assert emu.emu_ternary(w) == oracle_mod.ternary(w)
            assert emu.emu_gauss(w, 3.2, B) == oracle_mod.gauss(w, T, B)
    edges = [0, 1, 2**64 - 1] + [int(t) + d for t in T for d in (-1, 0, 1)]
    for w in edges:
        w %= 2**64
        assert emu.emu_gauss(w, 3.2, B) == oracle_mod.gauss(w, T, B)
    for w in (0x5555555555555555, 0x5555555555555556, 0xAAAAAAAAAAAAAAAA, 0xAAAAAAAAAAAAAAAB):
        assert emu.emu_ternary(w) == oracle_mod.ternary(w)
