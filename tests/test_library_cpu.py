"""CPU checks of the C-ABI library: it loads, exports every declared entry point, and its
host-side setup (primes, Gaussian table, encoding table, validation) agrees with the
oracle.  No compute call is made: no GPU is needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "ckks_mi355x.h")


@pytest.fixture(scope="module")
def pkg():
    import paper_2409_03568_amd as P

    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libckks_mi355x.so is not built (run __graft_entry__.build())")
    P.lib()
    return P


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ckks_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(pkg):
    names = _declared_functions()
    assert len(names) >= 20
    raw = C.CDLL(pkg.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert set(names) <= set(pkg._SIGS), set(names) - set(pkg._SIGS)


CONFIGS = [(12, 3, 36, 30), (13, 4, 50, 40), (11, 2, 30, 20), (14, 2, 50, 40)]


@pytest.mark.parametrize("log_n,L,bits,log_scale", CONFIGS)
def test_primes_match_oracle(pkg, oracle_mod, log_n, L, bits, log_scale):
    p = pkg.ckks_params(log_n, L, bits, log_scale)
    q, B = pkg.ckks_params_resolve(p)
    assert q == oracle_mod.gen_primes(log_n, bits, L)
    assert B == 19


@pytest.mark.parametrize("sigma,B", [(3.2, 0), (3.2, 12), (1.5, 0), (0.0, 0)])
def test_cdt_table_matches_oracle_bitwise(pkg, oracle_mod, sigma, B):
    p = pkg.ckks_params(13, 2, 50, 40, sigma=sigma, gauss_bound=B)
    T = pkg.ckks_host_cdt_table(p)
    Bref = (B or int(6 * sigma)) if sigma > 0 else 0
    assert np.array_equal(T, oracle_mod.cdt_table(sigma, Bref))


@pytest.mark.parametrize("log_n,log_scale", [(12, 30), (13, 40), (11, 25)])
def test_encode_table_matches_oracle_bitwise(pkg, oracle_mod, log_n, log_scale):
    p = pkg.ckks_params(log_n, 2, 50 if log_scale > 30 else 36, log_scale)
    assert np.array_equal(pkg.ckks_host_encode_table(p), oracle_mod.encode_table(log_n, log_scale))


def test_parameter_validation(pkg, oracle_mod):
    def code(**kw):
        args = dict(log_n=13, num_primes=4, prime_bits=50, log_scale=40)
        args.update(kw)
        try:
            pkg.ckks_params_resolve(pkg.ckks_params(**args))
            return 0
        except pkg.CkksError as e:
            return e.code

    assert code() == 0
    assert code(log_n=10) == -8 and code(log_n=15) == -8
    assert code(prime_bits=51) == -8 and code(prime_bits=19) == -8
    assert code(num_primes=0) == -1 and code(num_primes=17) == -1
    assert code(log_scale=54) == -1  # 256 * 2^(54+1-13) = 2^50: pixel coefficients would not fit below q
    assert code(log_scale=52) == 0
    assert code(sigma=-1.0) == -1
    assert code(gauss_bound=64) == -1
    good = oracle_mod.gen_primes(13, 50, 6)
    assert code(primes=good[2:6]) == 0
    assert code(primes=[good[0], good[0], good[1], good[2]]) == -1  # repeated
    assert code(primes=[good[0] + 2] + good[1:4]) == -1  # not prime / not 1 mod 2N
    assert code(primes=oracle_mod.gen_primes(13, 36, 4)) == -1  # wrong bit length


def test_error_message_is_reported(pkg):
    with pytest.raises(pkg.CkksError) as ei:
        pkg.ckks_params_resolve(pkg.ckks_params(10, 2, 36, 30))
    assert "log_n" in str(ei.value)
    assert "log_n" in pkg.ckks_last_error()


def test_header_is_plain_c_and_cpp(tmp_path):
    """The ABI header compiles on its own as strict C99 and as C++11 (no torch or HIP
    types in the signatures)."""
    import subprocess

    src = tmp_path / "use_header.c"
    src.write_text('#include "ckks_mi355x.h"\n'
                   "int main(void) {\n"
                   "  ckks_params p;\n"
                   "  ckks_ct_batch b;\n"
                   "  (void)p; (void)b;\n"
                   "  return ckks_ct_bytes(0, 1) == 0 ? 0 : 1;\n"
                   "}\n")
    inc = os.path.join(ROOT, "include")
    for cmd in (["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only", "-I", inc, str(src)],
                ["g++", "-std=c++11", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only", "-x", "c++", "-I", inc,
                 str(src)]):
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
