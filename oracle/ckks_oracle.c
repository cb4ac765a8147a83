/*
 * ckks_oracle.c -- plain, slow CPU reference of pixel-level CKKS (arXiv 2409.03568).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU-baseline
 * timing.  It is written for a reader checking it against the paper, not for speed:
 * every modular product is a 128-bit multiply followed by '%', the negacyclic
 * product is the textbook twisted cyclic NTT, and each function follows the
 * definition it cites.  See ckks_oracle.h for the conventions.
 */
#include "ckks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* scalar modular arithmetic                                                 */
/* ------------------------------------------------------------------------ */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
  a %= q;
  b %= q;
  return a >= b ? a - b : a + (q - b);
}
static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}
/* inverse by Fermat's little theorem (q prime) */
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }
/* signed integer -> residue in [0, q) */
static uint64_t residue(int64_t x, uint64_t q) {
  int64_t r = x % (int64_t)q;
  return (uint64_t)(r < 0 ? r + (int64_t)q : r);
}
/* integer-valued double of any magnitude -> residue in [0, q):
 * |x| = M * 2^e with M < 2^53, so x mod q = (M mod q)(2^e mod q). */
static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q);
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q);
static uint64_t residue_dbl(double x, uint64_t q) {
  if (fabs(x) < 9.0e18) return residue((int64_t)x, q);
  int e;
  const double m = frexp(fabs(x), &e);
  const uint64_t M = (uint64_t)ldexp(m, 53);
  const uint64_t r = mulmod(M % q, powmod(2, (uint64_t)(e - 53), q), q);
  return (x < 0 && r) ? q - r : r;
}

/* ------------------------------------------------------------------------ */
/* parameters: Sec. 4.2 (N = 2^12, Q ~ 2^109, ternary secret); RNS primes    */
/* q_i = 1 mod 2N so X^N+1 splits and the NTT exists (Sec. 2.2.1 ring R_q).  */
/* ------------------------------------------------------------------------ */
static int is_prime_trial(uint64_t n) {
  if (n < 2) return 0;
  if (n % 2 == 0) return n == 2;
  for (uint64_t d = 3; d <= n / d; d += 2)
    if (n % d == 0) return 0;
  return 1;
}

/* The L largest primes below 2^bits that are = 1 mod 2N, in descending order,
 * each with exactly `bits` bits.  Returns the number found. */
int orc_gen_primes(int log_n, int bits, int L, uint64_t *q) {
  const uint64_t m = 2ULL << log_n;
  const uint64_t top = 1ULL << bits, bottom = 1ULL << (bits - 1);
  uint64_t c = ((top - 2) / m) * m + 1; /* largest c = 1 mod 2N with c < 2^bits */
  int found = 0;
  while (found < L && c > bottom) {
    if (is_prime_trial(c)) q[found++] = c;
    c -= m;
  }
  return found;
}

/* Some psi with psi^N = -1 (mod q): then psi has order exactly 2N, as 2N is a
 * power of two. */
uint64_t orc_primitive_2n_root(uint64_t q, int log_n) {
  const uint64_t N = 1ULL << log_n;
  for (uint64_t x = 2; x < q; x++) {
    uint64_t psi = powmod(x, (q - 1) / (2 * N), q);
    if (powmod(psi, N, q) == q - 1) return psi;
  }
  return 0;
}

/* Cumulative table of the discrete Gaussian on [-B, B] with weights
 * rho(y) = exp(-y^2 / (2 sigma^2)).  The paper only says the errors are
 * Gaussian (Sec. 2.2.1); the table is defined by this exact double-precision
 * procedure: rho in order y = -B..B, Z = running sum of all rho, and
 * T[k] = floor(2^64 * (rho(-B) + ... + rho(k-B)) / Z) for k = 0..2B-1.
 * A sample from word w is -B + #{k : w >= T[k]}. */
int orc_cdt_table(double sigma, int B, uint64_t *T) {
  if (B <= 0) return 0;
  if (B > ORC_MAX_B) return -1;
  double rho[2 * ORC_MAX_B + 1];
  for (int y = -B; y <= B; y++) rho[y + B] = exp(-(double)(y * y) / (2.0 * sigma * sigma));
  double Z = 0.0;
  for (int i = 0; i <= 2 * B; i++) Z += rho[i];
  double cum = 0.0;
  for (int k = 0; k < 2 * B; k++) {
    cum += rho[k];
    double f = cum / Z;
    T[k] = (f >= 1.0) ? UINT64_MAX : (uint64_t)ldexp(f, 64);
  }
  return 0;
}

int orc_params_init(orc_params *P, int log_n, int L, int bits, int log_scale, double sigma, int B,
                    const uint64_t *primes) {
  memset(P, 0, sizeof(*P));
  if (L < 1 || L > ORC_MAX_LIMBS || log_n < 1 || log_n > 17 || bits < 4 || bits > 61) return -1;
  P->log_n = log_n;
  P->L = L;
  P->log_scale = log_scale;
  P->sigma = sigma;
  P->B = (sigma > 0.0) ? B : 0;
  if (primes) {
    for (int i = 0; i < L; i++) P->q[i] = primes[i];
  } else if (orc_gen_primes(log_n, bits, L, P->q) != L) {
    return -2;
  }
  for (int i = 0; i < L; i++) {
    if ((P->q[i] - 1) % (2ULL << log_n) != 0) return -3;
    P->psi[i] = orc_primitive_2n_root(P->q[i], log_n);
    if (!P->psi[i]) return -3;
  }
  /* special prime of key switching: the largest prime of the same form (bits, 1 mod 2N)
     that is not a ciphertext prime */
  {
    uint64_t cand[ORC_MAX_LIMBS + 1];
    const int n = orc_gen_primes(log_n, bits, L + 1, cand);
    P->qP = 0;
    for (int k = 0; k < n && !P->qP; k++) {
      int used = 0;
      for (int i = 0; i < L; i++) used |= (cand[k] == P->q[i]);
      if (!used) P->qP = cand[k];
    }
    if (P->qP) P->psiP = orc_primitive_2n_root(P->qP, log_n);
  }
  if (orc_cdt_table(sigma, P->B, P->cdt) != 0) return -4;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128 multiplies with a   */
/* Weyl-sequence key schedule.                                               */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    u128 p0 = (u128)M0 * x0, p1 = (u128)M1 * x2;
    uint64_t y0 = (uint64_t)(p1 >> 64) ^ x1 ^ k0;
    uint64_t y1 = (uint64_t)p1;
    uint64_t y2 = (uint64_t)(p0 >> 64) ^ x3 ^ k1;
    uint64_t y3 = (uint64_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint64_t orc_stream_word(const uint64_t key[2], uint64_t t, uint64_t tag, uint64_t j) {
  uint64_t ctr[4] = {t, tag, j / 4, 0}, out[4];
  orc_philox4x64_10(ctr, key, out);
  return out[j % 4];
}

/* ternary in {-1, 0, 1}, each with probability 1/3 up to 2^-64: floor(3w/2^64) - 1
 * (secret key and encryption randomness: Sec. 4.2 "uniform ternary"). */
int64_t orc_ternary(uint64_t w) { return (int64_t)(((u128)w * 3) >> 64) - 1; }

int64_t orc_gauss(uint64_t w, const uint64_t *T, int B) {
  int64_t c = 0;
  for (int k = 0; k < 2 * B; k++)
    if (w >= T[k]) c++;
  return c - B;
}

void orc_sample_ternary(const uint64_t key[2], uint64_t t, uint64_t tag, int N, int64_t *out) {
  for (int j = 0; j < N; j++) out[j] = orc_ternary(orc_stream_word(key, t, tag, (uint64_t)j));
}

void orc_sample_gauss(const orc_params *P, const uint64_t key[2], uint64_t t, uint64_t tag, int64_t *out) {
  const int N = 1 << P->log_n;
  for (int j = 0; j < N; j++) out[j] = orc_gauss(orc_stream_word(key, t, tag, (uint64_t)j), P->cdt, P->B);
}

/* Uniform residues mod q by rejection: coefficient j tries the words of block j,
 * then of block N+j, 2N+j, ..., accepting the first w < q*floor(2^64/q). */
void orc_sample_uniform(const uint64_t key[2], uint64_t t, uint64_t tag, int N, uint64_t q, uint64_t *out) {
  const uint64_t limit = (uint64_t)((((u128)1 << 64) / q) * q); /* q*floor(2^64/q) < 2^64 */
  for (int j = 0; j < N; j++) {
    int done = 0;
    for (uint64_t a = 0; !done; a++) {
      uint64_t ctr[4] = {t, tag, a * (uint64_t)N + (uint64_t)j, 0}, w[4];
      orc_philox4x64_10(ctr, key, w);
      for (int k = 0; k < 4 && !done; k++) {
        if (w[k] < limit) {
          out[j] = w[k] % q;
          done = 1;
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* negacyclic product in Z_q[X]/(X^N+1) (Sec. 2.2, the ciphertext ring)      */
/* ------------------------------------------------------------------------ */
/* Definition: c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j. */
void orc_negacyclic_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *c, int N, uint64_t q) {
  for (int k = 0; k < N; k++) c[k] = 0;
  for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
      uint64_t p = mulmod(a[i], b[j], q);
      if (i + j < N)
        c[i + j] = addmod(c[i + j], p, q);
      else
        c[i + j - N] = submod(c[i + j - N], p, q);
    }
}

static void bit_reverse_permute(uint64_t *a, int N) {
  for (int i = 1, j = 0; i < N; i++) {
    int bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      uint64_t t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
}

/* Textbook iterative radix-2 cyclic NTT: A_k = sum_j a_j omega^{jk}. */
static void cyclic_ntt(uint64_t *a, int N, uint64_t omega, uint64_t q) {
  bit_reverse_permute(a, N);
  for (int len = 2; len <= N; len <<= 1) {
    uint64_t wl = powmod(omega, (uint64_t)(N / len), q);
    for (int i = 0; i < N; i += len) {
      uint64_t w = 1;
      for (int j = 0; j < len / 2; j++) {
        uint64_t u = a[i + j], v = mulmod(a[i + j + len / 2], w, q);
        a[i + j] = addmod(u, v, q);
        a[i + j + len / 2] = submod(u, v, q);
        w = mulmod(w, wl, q);
      }
    }
  }
}

/* Negacyclic product as a twisted cyclic convolution: with psi^N = -1,
 * a(X)b(X) mod X^N+1 = psi^{-k} * cyclic(a_j psi^j, b_j psi^j)_k. */
void orc_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *c, int N, uint64_t q, uint64_t psi) {
  uint64_t *A = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *Bv = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t pw = 1;
  for (int j = 0; j < N; j++) {
    A[j] = mulmod(a[j] % q, pw, q);
    Bv[j] = mulmod(b[j] % q, pw, q);
    pw = mulmod(pw, psi, q);
  }
  const uint64_t omega = mulmod(psi, psi, q);
  cyclic_ntt(A, N, omega, q);
  cyclic_ntt(Bv, N, omega, q);
  for (int j = 0; j < N; j++) A[j] = mulmod(A[j], Bv[j], q);
  cyclic_ntt(A, N, invmod(omega, q), q); /* inverse transform up to the factor N */
  const uint64_t ninv = invmod((uint64_t)N % q, q), psi_inv = invmod(psi, q);
  pw = ninv;
  for (int j = 0; j < N; j++) {
    c[j] = mulmod(A[j], pw, q);
    pw = mulmod(pw, psi_inv, q);
  }
  free(A);
  free(Bv);
}

/* ------------------------------------------------------------------------ */
/* encoding (Sec. 2.2: C^{N/2} <-> Z_Q[X]/(X^N+1)), one pixel per plaintext  */
/* ------------------------------------------------------------------------ */
/* The pixel sits in slot 0 and every other slot is 0.  Inverting the canonical
 * embedding for that vector gives the closed form
 *   m_j = rint(value * (2 Delta / N) cos(pi j / N)),
 * because only the evaluation points exp(+-i pi/N) carry the value. */
void orc_encode_table(int log_n, int log_scale, double *T) {
  const int N = 1 << log_n;
  for (int j = 0; j < N; j++) T[j] = ldexp(cos(M_PI * (double)j / (double)N), log_scale + 1 - log_n);
}

void orc_encode(const orc_params *P, double value, int64_t *m) {
  const int N = 1 << P->log_n;
  double *T = (double *)malloc(sizeof(double) * (size_t)N);
  orc_encode_table(P->log_n, P->log_scale, T);
  for (int j = 0; j < N; j++) m[j] = (int64_t)rint(value * T[j]);
  free(T);
}

/* ------------------------------------------------------------------------ */
/* key generation (Sec. 2.2.2, steps 1-2): s ternary, e Gaussian, a uniform  */
/* per limb; pk0 = -a*s + e, pk1 = a.  Layout pk[2][L][N].                   */
/* ------------------------------------------------------------------------ */
void orc_keygen(const orc_params *P, const uint64_t seed[2], int64_t *s, uint64_t *pk) {
  const int N = 1 << P->log_n, L = P->L;
  int64_t *e = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *si = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *as = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  orc_sample_ternary(seed, 0, ORC_TAG_SK, N, s);
  orc_sample_gauss(P, seed, 0, ORC_TAG_EK, e);
  for (int i = 0; i < L; i++) {
    const uint64_t q = P->q[i];
    orc_sample_uniform(seed, 0, (uint64_t)(ORC_TAG_A0 + i), N, q, a);
    for (int j = 0; j < N; j++) si[j] = residue(s[j], q);
    orc_negacyclic_mul(a, si, as, N, q, P->psi[i]);
    uint64_t *pk0 = pk + (size_t)i * N, *pk1 = pk + ((size_t)L + i) * N;
    for (int j = 0; j < N; j++) {
      pk0[j] = addmod(submod(0, as[j], q), residue(e[j], q), q);
      pk1[j] = a[j];
    }
  }
  free(e);
  free(a);
  free(si);
  free(as);
}

/* ------------------------------------------------------------------------ */
/* encryption (Sec. 2.2.2): c0 = v*pk0 + e0 + m, c1 = v*pk1 + e1 (mod q_i).  */
/* v, e0, e1 come from the streams (seed, t, tag 1/2/3).  ct[2][L][N].       */
/* ------------------------------------------------------------------------ */
void orc_encrypt(const orc_params *P, const uint64_t *pk, double value, const uint64_t seed[2], uint64_t t,
                 uint64_t *ct) {
  const int N = 1 << P->log_n, L = P->L;
  int64_t *v = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  int64_t *e0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  int64_t *e1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  int64_t *m = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  uint64_t *vi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *prod = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  orc_sample_ternary(seed, t, ORC_TAG_V, N, v);
  orc_sample_gauss(P, seed, t, ORC_TAG_E0, e0);
  orc_sample_gauss(P, seed, t, ORC_TAG_E1, e1);
  orc_encode(P, value, m);
  for (int i = 0; i < L; i++) {
    const uint64_t q = P->q[i];
    for (int j = 0; j < N; j++) vi[j] = residue(v[j], q);
    const uint64_t *pk0 = pk + (size_t)i * N, *pk1 = pk + ((size_t)L + i) * N;
    uint64_t *c0 = ct + (size_t)i * N, *c1 = ct + ((size_t)L + i) * N;
    orc_negacyclic_mul(vi, pk0, prod, N, q, P->psi[i]);
    for (int j = 0; j < N; j++) c0[j] = addmod(addmod(prod[j], residue(e0[j], q), q), residue(m[j], q), q);
    orc_negacyclic_mul(vi, pk1, prod, N, q, P->psi[i]);
    for (int j = 0; j < N; j++) c1[j] = addmod(prod[j], residue(e1[j], q), q);
  }
  free(v);
  free(e0);
  free(e1);
  free(m);
  free(vi);
  free(prod);
}

/* ------------------------------------------------------------------------ */
/* decryption (Sec. 2.2.2): m' = c0 + c1*s, then decode slot 0.              */
/* ------------------------------------------------------------------------ */
/* d[level][N] = c0 + c1*s mod q_i for a ciphertext of the given level. */
void orc_decrypt_coeffs(const orc_params *P, const int64_t *s, const uint64_t *ct, int level, uint64_t *d) {
  const int N = 1 << P->log_n;
  uint64_t *si = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *prod = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  for (int i = 0; i < level; i++) {
    const uint64_t q = P->q[i];
    for (int j = 0; j < N; j++) si[j] = residue(s[j], q);
    const uint64_t *c0 = ct + (size_t)i * N, *c1 = ct + ((size_t)level + i) * N;
    orc_negacyclic_mul(c1, si, prod, N, q, P->psi[i]);
    for (int j = 0; j < N; j++) d[(size_t)i * N + j] = addmod(c0[j], prod[j], q);
  }
  free(si);
  free(prod);
}

/* Centered integer x_j with |x_j| < q_0/2 and x_j = d_0j (mod q_0).  This is the
 * CRT lift whenever the true value is below q_0/2 in magnitude; returns -1 if
 * another limb disagrees (the limb-0 lift is then not the CRT value). */
int orc_decode_centered(const orc_params *P, const uint64_t *d, int level, int64_t *x) {
  const int N = 1 << P->log_n;
  const uint64_t q0 = P->q[0];
  int bad = 0;
  for (int j = 0; j < N; j++) {
    uint64_t r = d[j];
    x[j] = (r > q0 / 2) ? (int64_t)r - (int64_t)q0 : (int64_t)r;
    for (int i = 1; i < level; i++)
      if (residue(x[j], P->q[i]) != d[(size_t)i * N + j]) bad = 1;
  }
  return bad ? -1 : 0;
}

/* Slot 0 of the canonical embedding, real part: sum_j x_j cos(pi j/N) / scale,
 * accumulated with Neumaier compensated summation. */
double orc_decrypt(const orc_params *P, const int64_t *s, const uint64_t *ct, int level, double scale, int *err) {
  const int N = 1 << P->log_n;
  uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N * (size_t)level);
  int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  orc_decrypt_coeffs(P, s, ct, level, d);
  int rc = orc_decode_centered(P, d, level, x);
  double sum = 0.0, comp = 0.0;
  for (int j = 0; j < N; j++) {
    double term = (double)x[j] * cos(M_PI * (double)j / (double)N);
    double tsum = sum + term;
    if (fabs(sum) >= fabs(term))
      comp += (sum - tsum) + term;
    else
      comp += (term - tsum) + sum;
    sum = tsum;
  }
  free(d);
  free(x);
  if (err) *err = rc;
  return (sum + comp) / scale;
}

/* ------------------------------------------------------------------------ */
/* homomorphic operations (Sec. 2.2.3)                                       */
/* ------------------------------------------------------------------------ */
/* addition: residue-wise (the add of Sec. 2.2.3) */
void orc_add(const orc_params *P, const uint64_t *a, const uint64_t *b, uint64_t *out, int level) {
  const int N = 1 << P->log_n;
  for (int poly = 0; poly < 2; poly++)
    for (int i = 0; i < level; i++)
      for (int j = 0; j < N; j++) {
        size_t o = ((size_t)poly * level + i) * N + j;
        out[o] = addmod(a[o], b[o], P->q[i]);
      }
}

/* subtraction (the (-) of Sec. 3.3) */
void orc_sub(const orc_params *P, const uint64_t *a, const uint64_t *b, uint64_t *out, int level) {
  const int N = 1 << P->log_n;
  for (int poly = 0; poly < 2; poly++)
    for (int i = 0; i < level; i++)
      for (int j = 0; j < N; j++) {
        size_t o = ((size_t)poly * level + i) * N + j;
        out[o] = submod(a[o], b[o], P->q[i]);
      }
}

/* Residue-wise product by the integer K (any integer-valued double). */
static void mul_by_integer(const orc_params *P, const uint64_t *a, int level, double K, uint64_t *out) {
  const int N = 1 << P->log_n;
  for (int poly = 0; poly < 2; poly++)
    for (int i = 0; i < level; i++) {
      const uint64_t k = residue_dbl(K, P->q[i]);
      for (int j = 0; j < N; j++) {
        size_t o = ((size_t)poly * level + i) * N + j;
        out[o] = mulmod(a[o], k, P->q[i]);
      }
    }
}

/* Multiply by a plaintext constant c.  An integer-valued c multiplies exactly
 * and keeps the scale; any other c is represented as K = rint(c * q_{level-1}) at
 * scale * q_{level-1}, so that a following rescale (division by q_{level-1})
 * restores the scale (Sec. 2.2.3, rescaling). */
int orc_mul_const(const orc_params *P, const uint64_t *a, int level, double scale, double c, uint64_t *out,
                  double *out_scale) {
  double K;
  double new_scale = scale;
  if (c == rint(c)) {
    K = c;
  } else {
    K = rint(c * (double)P->q[level - 1]);
    new_scale = scale * (double)P->q[level - 1];
  }
  if (!isfinite(K)) return -1;
  mul_by_integer(P, a, level, K, out);
  if (out_scale) *out_scale = new_scale;
  return 0;
}

/* Add a plaintext constant b to the encrypted pixel (brightness, Sec. 4.4.2;
 * watermark, Sec. 4.4.4).  b is encoded like a pixel -- slot 0, every other slot
 * 0 -- at the ciphertext's scale: m_j = rint(f cos(pi j/N)) with
 * f = (b * scale) * 2^(1 - log N), and added to c0 limb by limb. */
int orc_add_const(const orc_params *P, uint64_t *a, int level, double scale, double b) {
  const int N = 1 << P->log_n;
  const double f = ldexp(b * scale, 1 - P->log_n);
  if (!isfinite(f)) return -1;
  for (int j = 0; j < N; j++) {
    const double mj = rint(f * cos(M_PI * (double)j / (double)N));
    for (int i = 0; i < level; i++) {
      uint64_t *c0 = a + (size_t)i * N;
      c0[j] = addmod(c0[j], residue_dbl(mj, P->q[i]), P->q[i]);
    }
  }
  return 0;
}

/* Rescale (Sec. 2.2.3): divide by the last prime q = q_{level-1} with rounding,
 * floor((x + floor(q/2)) / q), and drop that limb.  In RNS:
 * r = (c_last + h) mod q, c'_i = (c_i + h - r) * q^{-1} mod q_i. */
int orc_rescale(const orc_params *P, const uint64_t *in, int level, double scale, uint64_t *out,
                double *out_scale) {
  if (level < 2) return -1;
  const int N = 1 << P->log_n, nl = level - 1;
  const uint64_t q = P->q[level - 1], h = q / 2;
  uint64_t qinv[ORC_MAX_LIMBS];
  for (int i = 0; i < nl; i++) qinv[i] = invmod(q % P->q[i], P->q[i]);
  for (int poly = 0; poly < 2; poly++) {
    const uint64_t *clast = in + ((size_t)poly * level + (level - 1)) * N;
    for (int j = 0; j < N; j++) {
      const uint64_t r = addmod(clast[j], h, q);
      for (int i = 0; i < nl; i++) {
        const uint64_t qi = P->q[i];
        const uint64_t ci = in[((size_t)poly * level + i) * N + j];
        const uint64_t num = submod(addmod(ci, h % qi, qi), r % qi, qi);
        out[((size_t)poly * nl + i) * N + j] = mulmod(num, qinv[i], qi);
      }
    }
  }
  if (out_scale) *out_scale = scale / (double)q;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* radix-based caching (Sec. 3.2) with radix randomness (Sec. 3.3)           */
/* ------------------------------------------------------------------------ */
/* entries[0] = Enc(0), entries[1+i] = Enc(r^i) for i < D, under the cache seed
 * with t = 0 and t = 1+i. */
void orc_radix_entries(const orc_params *P, const uint64_t *pk, int r, int D, const uint64_t cache_seed[2],
                       uint64_t *entries) {
  const size_t S = 2 * (size_t)P->L << P->log_n;
  orc_encrypt(P, pk, 0.0, cache_seed, ORC_RADIX_BASE_T, entries);
  double pw = 1.0;
  for (int i = 0; i < D; i++) {
    orc_encrypt(P, pk, pw, cache_seed, (uint64_t)(ORC_RADIX_BASE_T + 1 + i), entries + (size_t)(1 + i) * S);
    pw *= r;
  }
}

/* c = Enc(0) (+) digit_i copies of Enc(r^i) for every base-r digit of p; then for
 * i = 1..D-1, if bit i-1 of the auxiliary word is set, add Enc(r^i) and subtract
 * Enc(r^{i-1}) r times (Sec. 3.3: Ctxt (+) radixes[i] (-) r x radixes[i-1]). */
int orc_radix_encrypt(const orc_params *P, const uint64_t *entries, int r, int D, int p,
                      const uint64_t job_seed[2], uint64_t t, uint64_t *out) {
  const size_t S = 2 * (size_t)P->L << P->log_n;
  const int L = P->L;
  int rem = p;
  memcpy(out, entries, S * sizeof(uint64_t));
  for (int i = 0; i < D; i++) {
    int digit = rem % r;
    rem /= r;
    for (int k = 0; k < digit; k++) orc_add(P, out, entries + (size_t)(1 + i) * S, out, L);
  }
  if (rem != 0) return -1; /* p >= r^D: not representable with D digits */
  const uint64_t aux = orc_stream_word(job_seed, t, ORC_TAG_AUX, 1);
  for (int i = 1; i < D; i++) {
    if ((aux >> (i - 1)) & 1) {
      orc_add(P, out, entries + (size_t)(1 + i) * S, out, L);
      for (int k = 0; k < r; k++) orc_sub(P, out, entries + (size_t)i * S, out, L);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* scanning-based / full caching (Sec. 3.2) with a randomness pool (Sec. 3.3) */
/* ------------------------------------------------------------------------ */
void orc_histogram(const uint8_t *px, uint64_t n, uint64_t *h) {
  for (int v = 0; v < 256; v++) h[v] = 0;
  for (uint64_t i = 0; i < n; i++) h[px[i]]++;
}

/* The most frequent values, ranked by count (descending) then value
 * (ascending); values that never occur are not cached.  Returns how many. */
int orc_topk(const uint64_t *h, int k, int *values) {
  int used[256] = {0}, cnt = 0;
  while (cnt < k) {
    int best = -1;
    for (int v = 0; v < 256; v++) {
      if (used[v] || h[v] == 0) continue;
      if (best < 0 || h[v] > h[best]) best = v;
    }
    if (best < 0) break;
    used[best] = 1;
    values[cnt++] = best;
  }
  return cnt;
}

void orc_value_entry(const orc_params *P, const uint64_t *pk, int value, const uint64_t cache_seed[2],
                     uint64_t *ct) {
  orc_encrypt(P, pk, (double)value, cache_seed, (uint64_t)(ORC_VALUE_BASE_T + value), ct);
}

void orc_pool_entry(const orc_params *P, const uint64_t *pk, int u, const uint64_t cache_seed[2], uint64_t *ct) {
  orc_encrypt(P, pk, 0.0, cache_seed, (uint64_t)(ORC_POOL_BASE_T + u), ct);
}

/* The pool member for pixel t: floor(npool * w / 2^64), w = auxiliary word 0. */
uint32_t orc_pool_pick(const uint64_t job_seed[2], uint64_t t, uint32_t npool) {
  const uint64_t w = orc_stream_word(job_seed, t, ORC_TAG_AUX, 0);
  return (uint32_t)(((u128)w * npool) >> 64);
}

/* Cached pixel: c_p + c_z (Sec. 3.3, c_{p,final} = c_p + c_{zi}); value_ct is the
 * cached Enc(p) or NULL for a value that is not cached, which is then encrypted
 * in full with the pixel's own stream. */
void orc_value_encrypt(const orc_params *P, const uint64_t *pk, const uint64_t *value_ct, const uint64_t *pool,
                       uint32_t npool, int p, const uint64_t job_seed[2], uint64_t t, uint64_t *out) {
  if (!value_ct) {
    orc_encrypt(P, pk, (double)p, job_seed, t, out);
    return;
  }
  const size_t S = 2 * (size_t)P->L << P->log_n;
  const uint32_t u = orc_pool_pick(job_seed, t, npool);
  orc_add(P, value_ct, pool + (size_t)u * S, out, P->L);
}

/* ------------------------------------------------------------------------ */
/* mean filter (Sec. 4.4.1): I'(y,x) = (1/k^2) sum over the k x k window,    */
/* borders clamped to the edge; the ciphertext sum is followed by a          */
/* multiplication by 1/k^2 (scaled by the last prime) and a rescale.         */
/* ------------------------------------------------------------------------ */
int orc_mean_filter_pixel(const orc_params *P, const uint64_t *img, int H, int W, int level, double scale,
                          int k, int y, int x, uint64_t *out, double *out_scale) {
  if (k < 1 || (k % 2) == 0 || level < 2) return -1;
  const size_t S = 2 * (size_t)level << P->log_n;
  const int R = k / 2;
  uint64_t *acc = (uint64_t *)calloc(S, sizeof(uint64_t));
  uint64_t *tmp = (uint64_t *)malloc(S * sizeof(uint64_t));
  for (int dy = -R; dy <= R; dy++)
    for (int dx = -R; dx <= R; dx++) {
      int yy = y + dy, xx = x + dx;
      yy = yy < 0 ? 0 : (yy >= H ? H - 1 : yy);
      xx = xx < 0 ? 0 : (xx >= W ? W - 1 : xx);
      orc_add(P, acc, img + ((size_t)yy * W + xx) * S, acc, level);
    }
  /* the factor 1/k^2 always takes the scaled representation rint(q_{level-1} / k^2) at
   * scale * q_{level-1}, so the rescale restores the scale for every k (also k = 1) */
  const double ql = (double)P->q[level - 1];
  mul_by_integer(P, acc, level, rint((1.0 / (double)(k * k)) * ql), tmp);
  int rc = orc_rescale(P, tmp, level, scale * ql, out, out_scale);
  free(acc);
  free(tmp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* batches                                                                   */
/* ------------------------------------------------------------------------ */
void orc_encrypt_batch(const orc_params *P, const uint64_t *pk, const uint8_t *px, uint64_t n,
                       const uint64_t seed[2], uint64_t first_index, uint64_t *out) {
  const size_t S = 2 * (size_t)P->L << P->log_n;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < (int64_t)n; i++)
    orc_encrypt(P, pk, (double)px[i], seed, first_index + (uint64_t)i, out + (size_t)i * S);
}

void orc_decrypt_batch(const orc_params *P, const int64_t *s, const uint64_t *cts, uint64_t n, int level,
                       double scale, double *out, int *nerr) {
  const size_t S = 2 * (size_t)level << P->log_n;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int64_t i = 0; i < (int64_t)n; i++) {
    int e = 0;
    out[i] = orc_decrypt(P, s, cts + (size_t)i * S, level, scale, &e);
    if (e) bad++;
  }
  if (nerr) *nerr = bad;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* ciphertext multiplication (Sec. 2.2.3): tensor product, relinearization   */
/* by hybrid key switching with the special prime qP, one digit per limb.   */
/* ------------------------------------------------------------------------ */
static uint64_t prime_at(const orc_params *P, int j) { return j < P->L ? P->q[j] : P->qP; }
static uint64_t root_at(const orc_params *P, int j) { return j < P->L ? P->psi[j] : P->psiP; }

void orc_relin_keygen(const orc_params *P, const int64_t *s, const uint64_t seed[2], uint64_t *evk) {
  const int N = 1 << P->log_n, L = P->L;
  int64_t *e = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  uint64_t *si = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *s2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *as = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  for (int i = 0; i < L; i++) {
    orc_sample_gauss(P, seed, 0, (uint64_t)(ORC_TAG_RK_E0 + i), e);
    for (int j = 0; j <= L; j++) {
      const uint64_t p = prime_at(P, j), psi = root_at(P, j);
      uint64_t *b = evk + (((size_t)i * (L + 1) + j) * 2) * N, *a = b + N;
      orc_sample_uniform(seed, 0, (uint64_t)(ORC_TAG_RK_A0 + 32 * i + j), N, p, a);
      for (int k = 0; k < N; k++) si[k] = residue(s[k], p);
      orc_negacyclic_mul(a, si, as, N, p, psi);
      for (int k = 0; k < N; k++) b[k] = addmod(submod(0, as[k], p), residue(e[k], p), p);
      if (j == i) { /* + (qP mod q_i) * s^2 */
        orc_negacyclic_mul(si, si, s2, N, p, psi);
        const uint64_t pm = P->qP % p;
        for (int k = 0; k < N; k++) b[k] = addmod(b[k], mulmod(pm, s2[k], p), p);
      }
    }
  }
  free(e);
  free(si);
  free(s2);
  free(as);
}

void orc_tensor(const orc_params *P, const uint64_t *a, const uint64_t *b, int level, uint64_t *d) {
  const int N = 1 << P->log_n;
  uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  for (int j = 0; j < level; j++) {
    const uint64_t q = P->q[j], psi = P->psi[j];
    const uint64_t *a0 = a + (size_t)j * N, *a1 = a + ((size_t)level + j) * N;
    const uint64_t *b0 = b + (size_t)j * N, *b1 = b + ((size_t)level + j) * N;
    uint64_t *d0 = d + (size_t)j * N, *d1 = d + ((size_t)level + j) * N, *d2 = d + ((size_t)2 * level + j) * N;
    orc_negacyclic_mul(a0, b0, d0, N, q, psi);
    orc_negacyclic_mul(a0, b1, d1, N, q, psi);
    orc_negacyclic_mul(a1, b0, t, N, q, psi);
    for (int k = 0; k < N; k++) d1[k] = addmod(d1[k], t[k], q);
    orc_negacyclic_mul(a1, b1, d2, N, q, psi);
  }
  free(t);
}

void orc_key_switch(const orc_params *P, const uint64_t *evk, const uint64_t *d2, int level, uint64_t *acc) {
  const int N = 1 << P->log_n, L = P->L;
  uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
  for (int jj = 0; jj <= level; jj++) {
    const int j = jj < level ? jj : L; /* key index of the prime */
    const uint64_t p = prime_at(P, j), psi = root_at(P, j);
    uint64_t *acc0 = acc + (size_t)jj * N, *acc1 = acc + ((size_t)(level + 1) + jj) * N;
    memset(acc0, 0, sizeof(uint64_t) * (size_t)N);
    memset(acc1, 0, sizeof(uint64_t) * (size_t)N);
    for (int i = 0; i < level; i++) {
      const uint64_t *di = d2 + (size_t)i * N;
      for (int k = 0; k < N; k++) x[k] = di[k] % p; /* the digit as an integer in [0, q_i) */
      const uint64_t *kb = evk + (((size_t)i * (L + 1) + j) * 2) * N, *ka = kb + N;
      orc_negacyclic_mul(x, kb, t, N, p, psi);
      for (int k = 0; k < N; k++) acc0[k] = addmod(acc0[k], t[k], p);
      orc_negacyclic_mul(x, ka, t, N, p, psi);
      for (int k = 0; k < N; k++) acc1[k] = addmod(acc1[k], t[k], p);
    }
  }
  free(x);
  free(t);
}

void orc_mod_down(const orc_params *P, const uint64_t *acc, int level, uint64_t *out) {
  const int N = 1 << P->log_n;
  const uint64_t qP = P->qP;
  for (int k = 0; k < 2; k++) {
    const uint64_t *aP = acc + ((size_t)k * (level + 1) + level) * N;
    for (int j = 0; j < level; j++) {
      const uint64_t q = P->q[j], pinv = invmod(qP % q, q);
      const uint64_t *aj = acc + ((size_t)k * (level + 1) + j) * N;
      uint64_t *o = out + ((size_t)k * level + j) * N;
      for (int c = 0; c < N; c++) {
        /* centered residue of x mod qP, reduced mod q */
        const uint64_t xp = aP[c];
        const uint64_t xp_q = xp > qP / 2 ? submod(0, (qP - xp) % q, q) : xp % q;
        o[c] = mulmod(submod(aj[c], xp_q, q), pinv, q);
      }
    }
  }
}

void orc_mul(const orc_params *P, const uint64_t *evk, const uint64_t *a, const uint64_t *b, int level,
             uint64_t *out) {
  const int N = 1 << P->log_n;
  uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)3 * level * N);
  uint64_t *acc = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)2 * (level + 1) * N);
  uint64_t *ks = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)2 * level * N);
  orc_tensor(P, a, b, level, d);
  orc_key_switch(P, evk, d + (size_t)2 * level * N, level, acc);
  orc_mod_down(P, acc, level, ks);
  for (int k = 0; k < 2; k++)
    for (int j = 0; j < level; j++) {
      const uint64_t q = P->q[j];
      for (int c = 0; c < N; c++) {
        const size_t idx = ((size_t)k * level + j) * N + c;
        out[idx] = addmod(d[idx], ks[idx], q);
      }
    }
  free(d);
  free(acc);
  free(ks);
}
