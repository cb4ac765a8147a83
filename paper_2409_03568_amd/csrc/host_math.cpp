#include "host_math.hpp"

#include <math.h>

#include <algorithm>

#include "../../include/ckks_mi355x.h"

namespace ckks {
namespace host {

typedef unsigned __int128 u128;

uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = mul_mod(r, b, q);
    b = mul_mod(b, b, q);
  }
  return r;
}

uint64_t inv_mod(uint64_t a, uint64_t q) {
  // extended Euclid on signed 128-bit values
  __int128 t = 0, nt = 1, r = q, nr = a % q;
  while (nr != 0) {
    __int128 quo = r / nr, tmp;
    tmp = t - quo * nt; t = nt; nt = tmp;
    tmp = r - quo * nr; r = nr; nr = tmp;
  }
  if (t < 0) t += q;
  return (uint64_t)t;
}

uint64_t shoup_companion(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// Deterministic Miller-Rabin for 64-bit integers (the first twelve primes as bases
// are a proven witness set below 3.3e24).
bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; s++; }
  for (uint64_t a : small) {
    uint64_t x = pow_mod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s && comp; i++) {
      x = mul_mod(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

// A primitive 2N-th root: g^((q-1)/2N) for the first g whose power has order 2N
// (its N-th power is -1).
static uint64_t find_psi(uint64_t q, int log_n) {
  const uint64_t twoN = 2ULL << log_n;
  for (uint64_t g = 3; g < q; g += 2) {
    const uint64_t c = pow_mod(g, (q - 1) / twoN, q);
    if (pow_mod(c, twoN >> 1, q) == q - 1) return c;
  }
  return 0;
}

std::string resolve(uint32_t log_n, uint32_t L, uint32_t bits, uint32_t log_scale, double sigma, uint32_t gauss_bound,
                    const uint64_t *primes, Resolved *out, int *code) {
  *code = CKKS_EINVAL;
  if (log_n < 11 || log_n > 14) {
    *code = CKKS_EUNSUPPORTED;
    return "log_n must be in [11, 14]";
  }
  if (L < 1 || L > (uint32_t)kMaxLimbs) return "num_primes must be in [1, 16]";
  if (bits < 20 || bits > 50) {
    *code = CKKS_EUNSUPPORTED;
    return "prime_bits must be in [20, 50] (exact FP64 modular arithmetic)";
  }
  if (!(sigma >= 0.0) || sigma > 64.0) return "sigma must be in [0, 64]";
  int B = 0;
  if (sigma > 0.0) {
    B = gauss_bound ? (int)gauss_bound : (int)floor(6.0 * sigma);
    if (B < 1 || B > kMaxGaussBound) return "gauss_bound must be in [1, 63]";
  }
  const uint64_t twoN = 2ULL << log_n;
  std::vector<uint64_t> q;
  if (primes) {
    for (uint32_t i = 0; i < L; i++) {
      const uint64_t p = primes[i];
      if ((p >> (bits - 1)) != 1 || p % twoN != 1 || !is_prime(p)) return "caller prime is not a prime of prime_bits bits = 1 mod 2N";
      for (uint64_t r : q)
        if (r == p) return "caller primes must be distinct";
      q.push_back(p);
    }
  } else {
    // the L largest primes = 1 (mod 2N) below 2^bits
    const uint64_t lo = 1ULL << (bits - 1);
    uint64_t c = (((1ULL << bits) - 2) / twoN) * twoN + 1;
    while (q.size() < L && c > lo) {
      if (is_prime(c)) q.push_back(c);
      c -= twoN;
    }
    if (q.size() < L) return "not enough primes of the requested size";
  }
  const uint64_t qmin = *std::min_element(q.begin(), q.end());
  // pixel coefficients 255 * 2^(log_scale + 1 - log_n) must stay below the smallest prime
  if ((int)log_scale + 1 - (int)log_n + 8 >= 63 || (256.0 * ldexp(1.0, (int)log_scale + 1 - (int)log_n)) >= (double)qmin) {
    return "log_scale too large for the primes (256 * 2^(log_scale+1-log_n) must be < q_min)";
  }
  out->log_n = (int)log_n;
  out->L = (int)L;
  out->bits = (int)bits;
  out->log_scale = (int)log_scale;
  out->sigma = sigma;
  out->B = B;
  out->q = q;
  out->psi.clear();
  for (uint64_t p : q) {
    const uint64_t psi = find_psi(p, (int)log_n);
    if (!psi) return "no primitive root found";
    out->psi.push_back(psi);
  }
  out->qP = 0;
  out->psiP = 0;
  {
    const uint64_t lo = 1ULL << (bits - 1);
    for (uint64_t c = (((1ULL << bits) - 2) / twoN) * twoN + 1; c > lo && !out->qP; c -= twoN) {
      if (std::find(q.begin(), q.end(), c) == q.end() && is_prime(c)) out->qP = c;
    }
    if (out->qP) out->psiP = find_psi(out->qP, (int)log_n);
    if (!out->psiP) out->qP = 0;
  }
  *code = CKKS_OK;
  return "";
}

// The discrete Gaussian's cumulative thresholds: weights exp(-y^2 / (2 sigma^2)) for
// y = -B..B summed in that order, T[k] = floor(2^64 * (prefix sum through k-B) / total).
std::vector<uint64_t> cdt_table(double sigma, int B, int slots) {
  std::vector<uint64_t> T((size_t)slots, ~0ULL);
  if (B <= 0) return T;
  std::vector<double> w((size_t)(2 * B + 1));
  for (int i = 0; i <= 2 * B; i++) {
    const int y = i - B;
    w[(size_t)i] = exp(-(double)(y * y) / (2.0 * sigma * sigma));
  }
  double total = 0.0;
  for (double v : w) total += v;
  double run = 0.0;
  for (int k = 0; k < 2 * B; k++) {
    run += w[(size_t)k];
    const double f = run / total;
    T[(size_t)k] = f >= 1.0 ? ~0ULL : (uint64_t)ldexp(f, 64);
  }
  return T;
}

std::vector<double> encode_table(int log_n, int log_scale) {
  const int N = 1 << log_n;
  std::vector<double> T((size_t)N);
  for (int j = 0; j < N; j++) T[(size_t)j] = ldexp(cos(M_PI * (double)j / (double)N), log_scale + 1 - log_n);
  return T;
}

std::vector<double> cos_table(int log_n) {
  const int N = 1 << log_n;
  std::vector<double> T((size_t)N);
  for (int j = 0; j < N; j++) T[(size_t)j] = cos(M_PI * (double)j / (double)N);
  return T;
}

double centered(uint64_t r, uint64_t q) { return r > q / 2 ? -(double)(q - r) : (double)r; }

static uint32_t bit_reverse(uint32_t x, int bits) {
  uint32_t y = 0;
  for (int i = 0; i < bits; i++) y |= ((x >> i) & 1u) << (bits - 1 - i);
  return y;
}

void twiddles(uint64_t q, uint64_t psi, int log_n, std::vector<double> &fwd, std::vector<double> &inv) {
  const int N = 1 << log_n;
  const uint64_t psi_inv = inv_mod(psi, q);
  std::vector<uint64_t> pw((size_t)N), ipw((size_t)N);
  pw[0] = ipw[0] = 1;
  for (int i = 1; i < N; i++) {
    pw[(size_t)i] = mul_mod(pw[(size_t)i - 1], psi, q);
    ipw[(size_t)i] = mul_mod(ipw[(size_t)i - 1], psi_inv, q);
  }
  fwd.resize((size_t)N);
  inv.resize((size_t)N);
  for (int k = 0; k < N; k++) {
    const uint32_t b = bit_reverse((uint32_t)k, log_n);
    fwd[(size_t)k] = centered(pw[b], q);
    inv[(size_t)k] = centered(ipw[b], q);
  }
}

}  // namespace host
}  // namespace ckks
