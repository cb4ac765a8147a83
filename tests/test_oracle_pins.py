"""Pins of the CPU oracle against values the paper and the mathematics fix.

None of these checks re-types an oracle formula and compares it with itself:
each one ties an oracle function to something independent of it -- a published
known-answer vector, numpy's own Philox, sympy primality / NTT convolution /
CRT, mpmath's exact Gaussian weights, a numpy solve of the canonical embedding,
big-integer schoolbook products, closed-form identities, or numbers printed in
the paper.  A dropped term, a wrong sign or index, or a transposed operand in
the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

sympy = pytest.importorskip("sympy")
mpmath = pytest.importorskip("mpmath")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# Philox4x64-10
# ---------------------------------------------------------------------------
def test_philox_known_answer(oracle_mod):
    kat = json.load(open(os.path.join(GOLDEN, "philox4x64_10_kat.json")))
    out = oracle_mod.philox([int(x, 16) for x in kat["counter"]], [int(x, 16) for x in kat["key"]])
    assert out == [int(x, 16) for x in kat["output"]]


def test_philox_matches_numpy(oracle_mod):
    # numpy's Philox bit generator is Philox4x64-10; random_raw() first
    # increments its 256-bit counter (carrying across words) and then emits
    # the block for the incremented counter.
    rng = np.random.default_rng(12345)
    for trial in range(40):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        if trial % 4 == 0:
            ctr[0] = 0  # exercise the carry into word 1
        big = sum(c << (64 * i) for i, c in enumerate(ctr))
        prev = (big - 1) % (1 << 256)
        prev_words = [(prev >> (64 * i)) & M64 for i in range(4)]
        g = np.random.Philox(counter=np.array(prev_words, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
        assert [int(x) for x in g.random_raw(4)] == oracle_mod.philox(ctr, key)


def test_stream_word_layout(oracle_mod):
    # word j of stream (key, t, tag) is word j % 4 of the block with counter (t, tag, j // 4, 0)
    key = (0xABCDEF, 0x123)
    for t, tag, j in [(0, 1, 0), (5, 2, 7), (1023, 3, 4095), (7, 4, 1)]:
        blk = oracle_mod.philox([t, tag, j // 4, 0], key)
        assert oracle_mod.stream_word(key, t, tag, j) == blk[j % 4]


# ---------------------------------------------------------------------------
# parameters: primes and roots
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("log_n,bits,L", [(12, 36, 3), (13, 50, 4), (5, 20, 3), (11, 30, 2)])
def test_primes_are_the_largest_ntt_primes(oracle_mod, log_n, bits, L):
    q = oracle_mod.gen_primes(log_n, bits, L)
    m = 2 << log_n
    assert len(q) == L
    assert q == sorted(q, reverse=True)
    for x in q:
        assert sympy.isprime(x)
        assert x % m == 1
        assert x.bit_length() == bits
    # no skipped candidate: every c = 1 mod 2N between 2^bits and q[-1] that is not listed is composite
    c = ((1 << bits) - 2) // m * m + 1
    while c >= q[-1]:
        assert sympy.isprime(c) == (c in q)
        c -= m


@pytest.mark.parametrize("log_n,bits", [(12, 36), (13, 50), (4, 20)])
def test_primitive_root(oracle_mod, log_n, bits):
    N = 1 << log_n
    for q in oracle_mod.gen_primes(log_n, bits, 2):
        psi = oracle_mod.primitive_2n_root(q, log_n)
        assert pow(psi, N, q) == q - 1
        assert pow(psi, 2 * N, q) == 1


# ---------------------------------------------------------------------------
# samplers
# ---------------------------------------------------------------------------
def _exact_cdt(sigma, B, dps=60):
    mpmath.mp.dps = dps
    rho = [mpmath.e ** (-mpmath.mpf(y * y) / (2 * mpmath.mpf(sigma) ** 2)) for y in range(-B, B + 1)]
    Z = mpmath.fsum(rho)
    out, cum = [], mpmath.mpf(0)
    for k in range(2 * B):
        cum += rho[k]
        out.append(int(mpmath.floor(cum / Z * mpmath.mpf(2) ** 64)))
    return out, [r / Z for r in rho]


@pytest.mark.parametrize("sigma,B", [(3.2, 19), (1.0, 6), (3.2, 12)])
def test_cdt_table_against_exact(oracle_mod, sigma, B):
    T = [int(x) for x in oracle_mod.cdt_table(sigma, B)]
    exact, _ = _exact_cdt(sigma, B)
    assert all(T[i] < T[i + 1] for i in range(len(T) - 1))
    for a, b in zip(T, exact):
        # a double-precision cumulative sum is within a few ulps of 1 of the exact CDF
        assert abs(a - b) <= 2**14, (a, b)


def test_gauss_distribution(oracle_mod):
    o = oracle_mod.Oracle(14, 1, 30, 20, sigma=3.2)
    _, pmf = _exact_cdt(3.2, o.B)
    draws = np.concatenate([o.sample_gauss((77, 88), t, 2) for t in range(64)])  # 1,048,576 draws
    assert draws.min() >= -o.B and draws.max() <= o.B
    counts = np.bincount(draws + o.B, minlength=2 * o.B + 1)
    n = draws.size
    expected = np.array([float(p) * n for p in pmf])
    keep = expected > 20
    chi2 = float(np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep]))
    dof = int(keep.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)
    var_exact = float(sum(p * (y - o.B) ** 2 for y, p in enumerate(pmf)))
    assert abs(draws.mean()) < 6 * math.sqrt(var_exact / n)
    assert abs(draws.var() - var_exact) < 0.01 * var_exact


def test_gauss_inverse_cdf_at_thresholds(oracle_mod):
    # inversion sampling: a word w maps to the smallest y with w < 2^64 F(y), so the
    # sample steps from k-B to k-B+1 exactly at the table entry T[k]
    B = 19
    T = oracle_mod.cdt_table(3.2, B)
    for k in range(2 * B):
        assert oracle_mod.gauss(int(T[k]) - 1, T, B) == k - B
        assert oracle_mod.gauss(int(T[k]), T, B) == k - B + 1
    assert oracle_mod.gauss(0, T, B) == -B and oracle_mod.gauss(M64, T, B) == B


def test_ternary_distribution(oracle_mod):
    o = oracle_mod.Oracle(14, 1, 30, 20)
    draws = np.concatenate([o.sample_ternary((5, 6), t, 1) for t in range(32)])
    assert set(np.unique(draws)) <= {-1, 0, 1}
    counts = np.bincount(draws + 1, minlength=3)
    exp = draws.size / 3
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    assert chi2 < 2 + 6 * 2, chi2
    # the mapping floor(3w/2^64) - 1 at the thirds of the word range
    third = -(-(1 << 64) // 3)  # ceil(2^64/3): the first word mapped to 0
    assert oracle_mod.ternary(0) == -1 and oracle_mod.ternary(third - 1) == -1
    assert oracle_mod.ternary(third) == 0 and oracle_mod.ternary(M64) == 1


def test_uniform_mod_q(oracle_mod):
    o = oracle_mod.Oracle(14, 1, 30, 20)
    q = o.q[0]
    a = o.sample_uniform((1, 2), 0, 32, q)
    assert a.max() < q
    # top 4 bits of a/q are uniform
    bins = np.floor(a.astype(np.float64) / q * 16).astype(int)
    counts = np.bincount(bins, minlength=16)
    exp = a.size / 16
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    assert chi2 < 15 + 6 * math.sqrt(30), chi2


def test_uniform_rejection_order(oracle_mod):
    # modulus just above 2^63: about half of all words are rejected, so the
    # retry over words and blocks is exercised; every output must be the first
    # accepted word in the order (block j words 0..3, block N+j, ...).
    o = oracle_mod.Oracle(4, 1, 20, 10)
    q = (1 << 63) + 29
    limit = q * ((1 << 64) // q)
    key = (31, 41)
    a = o.sample_uniform(key, 3, 32, q)
    for j in range(o.N):
        first = None
        blk = j
        while first is None:
            g = np.random.Philox(counter=np.array([2, 32, blk, 0], dtype=np.uint64) , key=np.array(key, dtype=np.uint64))
            for w in (int(x) for x in g.random_raw(4)):
                if w < limit:
                    first = w % q
                    break
            blk += o.N
        assert int(a[j]) == first


# ---------------------------------------------------------------------------
# negacyclic product
# ---------------------------------------------------------------------------
def _schoolbook(a, b, q):
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            if i + j < N:
                c[i + j] += int(a[i]) * int(b[j])
            else:
                c[i + j - N] -= int(a[i]) * int(b[j])
    return [x % q for x in c]


@pytest.mark.parametrize("log_n,bits", [(3, 20), (4, 30), (5, 36), (6, 50)])
def test_negacyclic_ntt_vs_bigint_schoolbook(oracle_mod, log_n, bits):
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    for q in oracle_mod.gen_primes(log_n, bits, 2):
        psi = oracle_mod.primitive_2n_root(q, log_n)
        a = [int(x) % q for x in rng.integers(0, 2**63, N, dtype=np.uint64)]
        b = [int(x) % q for x in rng.integers(0, 2**63, N, dtype=np.uint64)]
        ref = _schoolbook(a, b, q)
        assert [int(x) for x in oracle_mod.negacyclic_mul(a, b, q, psi)] == ref
        assert [int(x) for x in oracle_mod.negacyclic_schoolbook(a, b, q)] == ref


def test_negacyclic_vs_sympy_convolution(oracle_mod):
    from sympy.discrete.convolutions import convolution_ntt

    N = 64
    q = 998244353  # 119 * 2^23 + 1
    psi = oracle_mod.primitive_2n_root(q, 6)
    rng = np.random.default_rng(9)
    a = [int(x) for x in rng.integers(0, q, N)]
    b = [int(x) for x in rng.integers(0, q, N)]
    full = convolution_ntt(a, b, prime=q) + [0] * 2
    ref = [(full[k] - full[k + N]) % q for k in range(N)]
    assert [int(x) for x in oracle_mod.negacyclic_mul(a, b, q, psi)] == ref


def test_negacyclic_config_sizes(oracle_mod):
    # N = 4096 with a 36-bit config prime: the NTT route against the O(N^2) schoolbook route
    o = oracle_mod.Oracle(10, 1, 36, 30)
    rng = np.random.default_rng(3)
    q = o.q[0]
    a = rng.integers(0, q, o.N, dtype=np.uint64)
    b = rng.integers(0, q, o.N, dtype=np.uint64)
    assert np.array_equal(oracle_mod.negacyclic_mul(a, b, q, o.psi[0]), oracle_mod.negacyclic_schoolbook(a, b, q))


# ---------------------------------------------------------------------------
# encoding: the canonical embedding with the pixel in slot 0
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("log_n", [3, 4, 5])
def test_encode_matches_canonical_embedding(oracle_mod, log_n):
    N = 1 << log_n
    log_scale = 20
    o = oracle_mod.Oracle(log_n, 1, 30, log_scale)
    w = np.exp(1j * np.pi / N)  # primitive 2N-th root of unity
    pts = [w ** (pow(5, k, 2 * N)) for k in range(N // 2)]
    pts = pts + [np.conj(p) for p in pts]
    V = np.array([[p**c for c in range(N)] for p in pts])
    for value in [0, 1, 37, 128, 255]:
        z = np.zeros(N // 2, dtype=complex)
        z[0] = value
        rhs = np.concatenate([z, np.conj(z)]) * 2.0**log_scale
        m = np.linalg.solve(V, rhs)
        assert np.max(np.abs(m.imag)) < 1e-6
        ref = np.rint(m.real).astype(np.int64)
        frac = np.abs(m.real - np.floor(m.real) - 0.5)
        ok = frac > 1e-6  # skip coefficients within 1e-6 of a rounding tie
        got = o.encode(value)
        assert np.array_equal(got[ok], ref[ok])
        # decoding slot 0 (evaluation at w) gives the value back up to rounding
        assert abs(np.polyval(got[::-1], w) / 2.0**log_scale - value) < N * 2.0 ** -(log_scale - 1)


def test_cos_identity(oracle_mod):
    # sum_j cos^2(pi j / N) = N / 2, so decode(encode(p)) = p before rounding
    for log_n in (4, 12, 13):
        T = oracle_mod.encode_table(log_n, log_n - 1)  # (2/N) * 2^(n-1) = 1: T_j = cos(pi j/N)
        assert abs(float(np.sum(T * T)) - (1 << log_n) / 2) < 1e-9 * (1 << log_n)


# ---------------------------------------------------------------------------
# key generation and encryption against big-integer schoolbook products
# ---------------------------------------------------------------------------
def test_keygen_and_encrypt_schoolbook(oracle_mod):
    o = oracle_mod.Oracle(4, 2, 30, 20, sigma=3.2)
    seed, job = (11, 22), (33, 44)
    s, pk = o.keygen(seed)
    N, L = o.N, o.L
    e = o.sample_gauss(seed, 0, oracle_mod.TAG_EK)
    assert np.array_equal(s, o.sample_ternary(seed, 0, oracle_mod.TAG_SK))
    pk = pk.reshape(2, L, N)
    for i, q in enumerate(o.q):
        a = o.sample_uniform(seed, 0, oracle_mod.TAG_A0 + i, q)
        as_ = _schoolbook(a, [int(x) % q for x in s], q)
        assert [int(x) for x in pk[0, i]] == [(-as_[j] + int(e[j])) % q for j in range(N)]
        assert np.array_equal(pk[1, i], a)
    t = 9
    ct = o.encrypt(200, job, t).reshape(2, L, N)
    v = o.sample_ternary(job, t, oracle_mod.TAG_V)
    e0 = o.sample_gauss(job, t, oracle_mod.TAG_E0)
    e1 = o.sample_gauss(job, t, oracle_mod.TAG_E1)
    m = o.encode(200)
    for i, q in enumerate(o.q):
        vq = [int(x) % q for x in v]
        p0 = _schoolbook(vq, pk[0, i], q)
        p1 = _schoolbook(vq, pk[1, i], q)
        assert [int(x) for x in ct[0, i]] == [(p0[j] + int(e0[j]) + int(m[j])) % q for j in range(N)]
        assert [int(x) for x in ct[1, i]] == [(p1[j] + int(e1[j])) % q for j in range(N)]


@pytest.mark.parametrize("log_n,L,bits,log_scale", [(5, 2, 30, 20), (12, 3, 36, 30)])
def test_noiseless_roundtrip_is_exact(oracle_mod, log_n, L, bits, log_scale):
    # sigma = 0: e = e0 = e1 = 0, so c0 + c1*s = v*(-a*s) + m + v*a*s = m exactly
    o = oracle_mod.Oracle(log_n, L, bits, log_scale, sigma=0.0)
    o.keygen((1, 2))
    for t, value in enumerate([0, 1, 100, 255]):
        ct = o.encrypt(value, (3, 4), t)
        d = o.decrypt_coeffs(ct)
        x, rc = o.decode_centered(d, L)
        assert rc == 0
        assert np.array_equal(x, o.encode(value))


def test_decrypt_limb0_equals_crt(oracle_mod):
    from sympy.ntheory.modular import crt

    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen((0x240903568, 1))
    ct = o.encrypt(173, (1, 0), 77)
    d = o.decrypt_coeffs(ct)
    x, rc = o.decode_centered(d, 3)
    assert rc == 0
    Q = math.prod(o.q)
    for j in range(0, o.N, 97):
        v, _ = crt(o.q, [int(d[i, j]) for i in range(3)])
        v = int(v)
        if v > Q // 2:
            v -= Q
        assert v == int(x[j])
    # fresh-noise error is far below the 1e-4 pixel bound at these parameters
    assert abs(o.decrypt(ct) - 173) < 1e-4


def test_decode_detects_out_of_bound_value(oracle_mod):
    # plant a coefficient whose CRT value is q0 (limb 0 reads 0): the limb-0 lift is wrong and must be flagged
    o = oracle_mod.Oracle(4, 3, 30, 20)
    d = np.zeros((3, o.N), dtype=np.uint64)
    d[1, 5] = o.q[0] % o.q[1]
    d[2, 5] = o.q[0] % o.q[2]
    _, rc = o.decode_centered(d, 3)
    assert rc == -1


def test_decrypt_exact_is_the_crt_decoding(oracle_mod):
    # the all-limb decryption equals the limb-0 decoding while the bound holds, and its CRT
    # integers are sympy's
    from sympy.ntheory.modular import crt

    o = oracle_mod.Oracle(8, 3, 30, 20)
    o.keygen((4, 4))
    for t, value in enumerate([0, 3, 128, 255]):
        ct = o.encrypt(value, (2, 2), t)
        assert abs(o.decrypt_exact(ct) - o.decrypt(ct)) < 1e-12 * max(1.0, value)
    d = o.decrypt_coeffs(ct)
    Q = math.prod(o.q)
    xs = []
    for j in range(o.N):
        v, _ = crt(o.q, [int(d[i, j]) for i in range(3)])
        v = int(v)
        xs.append(v - Q if v > Q // 2 else v)
    ref = math.fsum(float(x) * math.cos(math.pi * j / o.N) for j, x in enumerate(xs)) / o.scale
    assert o.decrypt_exact(ct) == ref


def test_decrypt_exact_recovers_a_sum_past_the_limb0_bound(oracle_mod):
    # 300 pixels of 255 at N = 4096, scale 2^30: the summed coefficients reach 300*255*2^19,
    # past q0/2 ~ 2^35, so limb 0 alone no longer decodes (and says so) while the CRT does
    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen((0x240903568, 1))
    cts = o.encrypt_batch(np.full(300, 255, dtype=np.uint8), (9, 9))
    acc = cts[0]
    for c in cts[1:]:
        acc = o.add(acc, c)
    with pytest.raises(ArithmeticError):
        o.decrypt(acc)
    assert abs(o.decrypt_exact(acc) - 300 * 255) < 3e-3
    m, sc = o.mul_const(cts[0], 300)
    with pytest.raises(ArithmeticError):
        o.decrypt(m)
    assert abs(o.decrypt_exact(m) - 300 * 255) < 3e-2


def _accepted_radix_pairs():
    pairs = []
    for r in range(2, 257):
        for D in range(1, 9):
            if r ** (D - 1) <= 255 and r ** D >= 256:
                pairs.append((r, D))
    return pairs


def test_radix_randomness_for_every_digit_count(oracle_mod):
    # Sec. 3.3 draws one randomness bit per radix above the lowest.  For every base with two or
    # more digits (what the library accepts), two encryptions of one pixel value whose bits differ
    # are different ciphertexts that decrypt to the same value; with a single digit (base 256,
    # which the library refuses) equal pixels always give the same ciphertext.
    o = oracle_mod.Oracle(5, 2, 30, 20)
    o.keygen((6, 6))
    job = (2, 3)
    words = [oracle_mod.stream_word(job, t, oracle_mod.TAG_AUX, 1) for t in range(64)]
    for r, D in _accepted_radix_pairs():
        E = o.radix_entries(r, D, (0xCAC4E, r))
        mask = (1 << (D - 1)) - 1
        if D == 1:
            a, b = o.radix_encrypt(E, r, D, 200, job, 0), o.radix_encrypt(E, r, D, 200, job, 1)
            assert np.array_equal(a, b), (r, D)
            continue
        t1 = 0
        t2 = next(t for t in range(1, 64) if (words[t] & mask) != (words[t1] & mask))
        a, b = o.radix_encrypt(E, r, D, 200, job, t1), o.radix_encrypt(E, r, D, 200, job, t2)
        assert not np.array_equal(a, b), (r, D)
        qs = np.array(o.q, dtype=object)[:, None]
        da, db = o.decrypt_coeffs(a).astype(object), o.decrypt_coeffs(b).astype(object)
        # both are 200 times Enc(1) plus encryptions of zero: their difference decrypts to noise only
        diff = (da - db) % qs
        diff = np.where(diff > qs // 2, diff - qs, diff)
        assert np.max(np.abs(diff.astype(float))) < 1e6, (r, D)
    assert (256, 1) in _accepted_radix_pairs() and all(D >= 2 for r, D in _accepted_radix_pairs() if r < 256)


# ---------------------------------------------------------------------------
# homomorphic operations
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_oracle(oracle_mod):
    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen((0x240903568, 1))
    return o


def test_linearity_is_exact(oracle_mod, c1_oracle):
    o = c1_oracle
    a = o.encrypt(10, (5, 5), 1)
    b = o.encrypt(250, (5, 5), 2)
    da, db = o.decrypt_coeffs(a).astype(object), o.decrypt_coeffs(b).astype(object)
    qs = np.array(o.q, dtype=object)[:, None]
    assert np.array_equal(o.decrypt_coeffs(o.add(a, b)).astype(object), (da + db) % qs)
    assert np.array_equal(o.decrypt_coeffs(o.sub(a, b)).astype(object), (da - db) % qs)
    k3, sc = o.mul_const(a, 3)
    assert sc == o.scale
    assert np.array_equal(o.decrypt_coeffs(k3).astype(object), (3 * da) % qs)
    km, sc = o.mul_const(a, -7)
    assert np.array_equal(o.decrypt_coeffs(km).astype(object), (-7 * da) % qs)
    assert abs(o.decrypt(o.add(a, b)) - 260) < 1e-4
    assert abs(o.decrypt(o.sub(a, b)) + 240) < 1e-4


def test_rescale_is_rounded_division_of_crt_value(oracle_mod, c1_oracle):
    from sympy.ntheory.modular import crt

    o = c1_oracle
    rng = np.random.default_rng(4)
    ct = np.concatenate([rng.integers(0, q, o.N, dtype=np.uint64) for q in o.q] * 2)
    out, sc = o.rescale(ct)
    ql = o.q[-1]
    ct = ct.reshape(2, 3, o.N)
    out = out.reshape(2, 2, o.N)
    for poly in range(2):
        for j in range(0, o.N, 61):
            x, _ = crt(o.q, [int(ct[poly, i, j]) for i in range(3)])
            y = (int(x) + ql // 2) // ql
            assert [int(out[poly, i, j]) for i in range(2)] == [y % o.q[0], y % o.q[1]]
    assert sc == o.scale / ql


def test_mul_const_fraction_then_rescale(oracle_mod, c1_oracle):
    o = c1_oracle
    a = o.encrypt(180, (6, 6), 3)
    m, sc = o.mul_const(a, 1.0 / 9.0)
    assert sc == o.scale * o.q[-1]
    assert np.array_equal(o.decrypt_coeffs(m).astype(object),
                          (o.decrypt_coeffs(a).astype(object) * round(o.q[-1] / 9.0))
                          % np.array(o.q, dtype=object)[:, None])
    r, sc2 = o.rescale(m, level=3, scale=sc)
    assert sc2 == o.scale  # Delta * q / q is exact in double precision
    assert abs(o.decrypt(r, level=2, scale=sc2) - 20.0) < 1e-4


def test_add_const(oracle_mod, c1_oracle):
    # adding the slot-0 encoding of b shifts the decrypted coefficients by exactly encode(b)
    o = c1_oracle
    a = o.encrypt(100, (7, 7), 4)
    qs = np.array(o.q, dtype=object)[:, None]
    for b, expect in [(-37.0, 63.0), (50.0, 150.0), (0.5, 100.5)]:
        c = o.add_const(a, b)
        diff = (o.decrypt_coeffs(c).astype(object) - o.decrypt_coeffs(a).astype(object)) % qs
        assert np.array_equal(diff, o.encode(b).astype(object)[None, :] % qs)
        assert abs(o.decrypt(c) - expect) < 1e-4


def test_residue_of_large_constants(oracle_mod, c1_oracle):
    # mul_const at a scale of Delta * q: K = rint(c * q_last) of any size reduces exactly mod q_i
    o = c1_oracle
    a = o.encrypt(9, (7, 7), 5)
    qs = np.array(o.q, dtype=object)[:, None]
    for c in (1e9 + 0.5, -3.0e12 + 0.25):
        m, sc = o.mul_const(a, c)
        K = int(np.rint(c * float(o.q[-1])))  # exact: every double above 2^53 is an integer
        assert np.array_equal(o.decrypt_coeffs(m).astype(object), (o.decrypt_coeffs(a).astype(object) * K) % qs)
    big = 2.0**70 + 2.0**20
    m, _ = o.mul_const(a, big)
    assert np.array_equal(o.decrypt_coeffs(m).astype(object), (o.decrypt_coeffs(a).astype(object) * int(big)) % qs)


# ---------------------------------------------------------------------------
# caching (Sec. 3.2) and randomness (Sec. 3.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("r,D", [(16, 2), (2, 8)])
def test_radix_cache_decrypts_every_pixel(oracle_mod, c1_oracle, r, D):
    o = c1_oracle
    E = o.radix_entries(r, D, (0xCAC4E, 1))
    job = (1, 99)
    vals = list(range(0, 256, 5)) + [255]
    got = np.array([o.decrypt(o.radix_encrypt(E, r, D, p, job, t)) for t, p in enumerate(vals)])
    # a wrong digit, index or sign shifts the decoded value by a multiple of r^i
    assert np.max(np.abs(got - np.array(vals))) < 3e-3


def test_radix_randomness_example(oracle_mod, c1_oracle):
    # Sec. 3.3 example with r = 2, i = 5: Ctxt (+) Enc(2^5) (-) 2 x Enc(2^4) still decrypts to Ctxt's value
    o = c1_oracle
    E = o.radix_entries(2, 8, (0xCAC4E, 2))
    ctxt = o.encrypt(77, (8, 8), 0)
    rnd = o.sub(o.sub(o.add(ctxt, E[1 + 5]), E[1 + 4]), E[1 + 4])
    assert abs(o.decrypt(rnd) - 77) < 1e-3
    assert not np.array_equal(rnd, ctxt)


def test_radix_randomness_changes_ciphertexts(oracle_mod, c1_oracle):
    o = c1_oracle
    E = o.radix_entries(16, 2, (0xCAC4E, 1))
    cts = [o.radix_encrypt(E, 16, 2, 200, (1, 5), t) for t in range(8)]
    bits = [o.stream_word((1, 5), t, oracle_mod.TAG_AUX, 1) & 1 if hasattr(o, "stream_word") else
            oracle_mod.stream_word((1, 5), t, oracle_mod.TAG_AUX, 1) & 1 for t in range(8)]
    # pixels whose randomness bit differs give different ciphertexts (P(identical bits for 8) = 2^-7)
    assert len(set(bits)) == 2
    distinct = {cts[t].tobytes() for t in range(8)}
    assert len(distinct) == 2


def test_topk_ranking(oracle_mod):
    rng = np.random.default_rng(5)
    px = rng.integers(0, 40, 5000).astype(np.uint8)
    px[:30] = 200
    h = oracle_mod.Oracle.histogram(px)
    assert np.array_equal(h, np.bincount(px, minlength=256))
    for k in (1, 10, 64):
        got = oracle_mod.Oracle.topk(h, k)
        order = np.lexsort((np.arange(256), -h.astype(np.int64)))  # count desc, then value asc
        ref = [int(v) for v in order if h[v] > 0][:k]
        assert got == ref


def test_pool_pick_is_multiply_high(oracle_mod):
    # u = floor(n w / 2^64): for n = 2^31 it is the top 31 bits of the word, for n = 1 always 0
    key = (1, 7)
    for t in range(20):
        w = oracle_mod.stream_word(key, t, oracle_mod.TAG_AUX, 0)
        assert oracle_mod.Oracle.pool_pick(key, t, 1 << 31) == w >> 33
        assert oracle_mod.Oracle.pool_pick(key, t, 1) == 0
        assert oracle_mod.Oracle.pool_pick(key, t, 256) == w >> 56


def test_value_cache_and_pool(oracle_mod, c1_oracle):
    o = c1_oracle
    cache_seed, job = (0xCAC4E, 1), (1, 7)
    npool = 8
    pool = np.stack([o.pool_entry(u, cache_seed) for u in range(npool)])
    C77 = o.value_entry(77, cache_seed)
    qs = np.array(o.q, dtype=object)[:, None]
    outs = []
    for t in range(6):
        c = o.value_encrypt(C77, pool, npool, 77, job, t)
        u = o.pool_pick(job, t, npool)
        assert 0 <= u < npool
        # c_{p,final} = c_p + c_z exactly (Sec. 3.3)
        assert np.array_equal(o.decrypt_coeffs(c).astype(object),
                              (o.decrypt_coeffs(C77).astype(object) + o.decrypt_coeffs(pool[u]).astype(object)) % qs)
        assert abs(o.decrypt(c) - 77) < 2e-4
        outs.append((u, c.tobytes()))
    # identical pixels with different pool picks give different ciphertexts
    picks = {u for u, _ in outs}
    assert len({c for _, c in outs}) == len(picks) > 1
    # a value outside the cache is a plain encryption with the pixel's own stream
    miss = o.value_encrypt(None, pool, npool, 12, job, 4)
    assert np.array_equal(miss, o.encrypt(12, job, 4))


# ---------------------------------------------------------------------------
# mean filter (Sec. 4.4.1)
# ---------------------------------------------------------------------------
def test_mean_filter_matches_plaintext(oracle_mod):
    o = oracle_mod.Oracle(10, 3, 36, 30)
    o.keygen((3, 3))
    H, W = 5, 6
    img = np.random.default_rng(8).integers(0, 256, (H, W)).astype(np.uint8)
    cts = o.encrypt_batch(img.reshape(-1), (3, 0))
    for k in (1, 3, 5):
        R = k // 2
        pad = np.pad(img.astype(np.float64), R, mode="edge")
        ref = np.zeros((H, W))
        for dy in range(k):
            for dx in range(k):
                ref += pad[dy:dy + H, dx:dx + W]
        ref /= k * k
        for (y, x) in [(0, 0), (2, 3), (H - 1, W - 1), (0, W - 1)]:
            out, sc = o.mean_filter_pixel(cts, H, W, k, y, x)
            assert sc == o.scale
            assert abs(o.decrypt(out, level=2, scale=sc) - ref[y, x]) < 1e-3


# ---------------------------------------------------------------------------
# image-quality metrics printed in the paper
# ---------------------------------------------------------------------------
def test_paper_psnr_values(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "paper_image_metrics.json")))
    mf = g["mean_filter"]
    assert abs(oracle_mod.psnr(mf["mse"]) - mf["psnr_db"]) < 0.01
    rows = [r for r in g["table2"] if r["consistent"]]
    assert len(rows) == 3
    for r in rows:
        assert abs(oracle_mod.psnr(r["mse"]) - r["psnr_db"]) < 0.05
    assert abs(np.mean([r["mse"] for r in g["table2"]]) - g["average"]["mse"]) < 1e-3
    assert abs(oracle_mod.mse([0, 10], [3, 14]) - 12.5) < 1e-12


# ---------------------------------------------------------------------------
# ciphertext multiplication: tensor product, key switching, ModDown (Sec. 2.2.3)
# ---------------------------------------------------------------------------
def _negacyclic_int(a, b):
    """Negacyclic product of two integer sequences over Z (Python integers)."""
    N = len(a)
    c = [0] * N
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            k = i + j
            if k < N:
                c[k] += x * y
            else:
                c[k - N] -= x * y
    return c


def _crt(res, mods):
    return int(sympy.ntheory.modular.crt(mods, [int(r) for r in res])[0])


@pytest.fixture(scope="module")
def tiny_mul_oracle(oracle_mod):
    o = oracle_mod.Oracle(4, 3, 30, 12)  # N = 16, three 30-bit primes
    o.keygen((5, 6))
    o.relin_keygen((7, 8))
    return o


def test_special_prime_is_the_next_ntt_prime(oracle_mod, tiny_mul_oracle):
    o = tiny_mul_oracle
    four = oracle_mod.gen_primes(o.log_n, 30, 4)
    assert o.q == four[:3] and o.qP == four[3]
    assert sympy.isprime(o.qP) and (o.qP - 1) % (2 * o.N) == 0
    assert pow(o.psiP, o.N, o.qP) == o.qP - 1


@pytest.mark.parametrize("level", [3, 2, 1])
def test_key_switch_decrypts_to_qP_d2_s2_plus_small(tiny_mul_oracle, level):
    # With s, the key-switched digits decrypt (mod qP * Q_level) exactly to
    # qP * D2 * s^2 + sum_i d2_i * e_i, where D2 is the CRT value of the digits and e_i
    # the keys' error streams: the key carries qP s^2 in limb i only, all keys share the
    # secret, and each digit is lifted as the integer it is.
    o = tiny_mul_oracle
    N = o.N
    rng = np.random.default_rng(level)
    d2 = np.concatenate([rng.integers(0, q, N, dtype=np.uint64) for q in o.q[:level]])
    acc = o.key_switch(d2, level).reshape(2, level + 1, N)
    mods = o.q[:level] + [o.qP]
    M = math.prod(mods)
    s = [int(x) for x in o.s]
    B = [_crt(acc[0, :, c], mods) for c in range(N)]
    A = [_crt(acc[1, :, c], mods) for c in range(N)]
    As = _negacyclic_int(A, s)
    dec = [(B[c] + As[c]) % M for c in range(N)]
    digits = [[int(x) for x in d2[i * N:(i + 1) * N]] for i in range(level)]
    D2 = [_crt([digits[i][c] for i in range(level)], o.q[:level]) for c in range(N)]
    want = [o.qP * v for v in _negacyclic_int(D2, _negacyclic_int(s, s))]
    for i in range(level):
        e = [int(x) for x in o.sample_gauss((7, 8), 0, 48 + i)]
        for c, v in enumerate(_negacyclic_int(digits[i], e)):
            want[c] += v
    assert dec == [w % M for w in want]


def test_mod_down_is_rounded_division_by_qP(tiny_mul_oracle):
    o = tiny_mul_oracle
    N = o.N
    rng = np.random.default_rng(11)
    for level in (3, 1):
        mods = o.q[:level] + [o.qP]
        acc = np.stack([np.stack([rng.integers(0, m, N, dtype=np.uint64) for m in mods]) for _ in range(2)])
        out = o.mod_down(acc.reshape(-1), level).reshape(2, level, N)
        for k in range(2):
            for c in range(N):
                x = _crt(acc[k, :, c], mods)
                r = x % o.qP
                if r > o.qP // 2:
                    r -= o.qP
                y = (x - r) // o.qP  # exact; |y - x/qP| <= 1/2
                assert abs(y - x / o.qP) <= 0.5 + 1e-9
                for j in range(level):
                    assert int(out[k, j, c]) == y % o.q[j]


def test_tensor_is_the_product_of_the_decryptions(tiny_mul_oracle):
    # d0 + d1 s + d2 s^2 = (a0 + a1 s)(b0 + b1 s) in each R_q
    o = tiny_mul_oracle
    N, L = o.N, o.L
    a = o.encrypt(37.0, (1, 1), 3)
    b = o.encrypt(201.0, (1, 1), 4)
    d = o.tensor(a, b).reshape(3, L, N)
    a2, b2 = a.reshape(2, L, N), b.reshape(2, L, N)
    s = [int(x) for x in o.s]
    for j, q in enumerate(o.q):
        lhs = [0] * N
        for k, poly in enumerate((d[0, j], d[1, j], d[2, j])):
            term = [int(x) for x in poly]
            for _ in range(k):
                term = _negacyclic_int(term, s)
            lhs = [x + y for x, y in zip(lhs, term)]
        da = [int(x) + y for x, y in zip(a2[0, j], _negacyclic_int([int(v) for v in a2[1, j]], s))]
        db = [int(x) + y for x, y in zip(b2[0, j], _negacyclic_int([int(v) for v in b2[1, j]], s))]
        rhs = _negacyclic_int(da, db)
        assert [x % q for x in lhs] == [x % q for x in rhs]


@pytest.fixture(scope="module")
def c1_mul_oracle(oracle_mod):
    o = oracle_mod.Oracle(12, 3, 36, 30)
    o.keygen((0x240903568, 1))
    o.relin_keygen((0x240903568, 99))
    return o


def test_product_decrypts_to_the_product_of_pixels(c1_mul_oracle):
    # CKKS multiplication: (p1 * p2) at scale Delta^2, rescaled once (Sec. 2.2.3)
    o = c1_mul_oracle
    for p1, p2 in ((0, 255), (17, 23), (255, 255), (128, 3)):
        a = o.encrypt(p1, (2, 2), p1)
        b = o.encrypt(p2, (2, 2), 1000 + p2)
        m = o.mul(a, b)
        r, sc = o.rescale(m, level=3, scale=o.scale * o.scale)
        assert sc == o.scale * o.scale / o.q[2]
        got = o.decrypt(r, level=2, scale=sc)
        assert abs(got - p1 * p2) < 0.05, (p1, p2, got)


def test_squared_difference_gives_the_l1_distance(c1_mul_oracle):
    # image matching (Sec. 4.4.3): per pixel (I1 - I2)^2 in encrypted form; the client
    # decrypts and sums the square roots, which is the L1 distance
    o = c1_mul_oracle
    rng = np.random.default_rng(3)
    i1 = rng.integers(0, 256, 6)
    i2 = rng.integers(0, 256, 6)
    total = 0.0
    for t, (x, y) in enumerate(zip(i1, i2)):
        d = o.sub(o.encrypt(float(x), (4, 4), t), o.encrypt(float(y), (4, 5), t))
        sq, sc = o.rescale(o.mul(d, d), level=3, scale=o.scale * o.scale)
        v = o.decrypt(sq, level=2, scale=sc)
        assert abs(v - (int(x) - int(y)) ** 2) < 0.05
        total += math.sqrt(max(v, 0.0))
    assert abs(total - np.abs(i1.astype(int) - i2.astype(int)).sum()) < 0.05
