// Host-side setup arithmetic: parameter resolution and the tables a context uploads.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace ckks {
namespace host {

constexpr int kMaxLimbs = 16;
constexpr int kMaxGaussBound = 63;  // a sample plus B fits 7 bits of the packed sample word

struct Resolved {
  int log_n = 0;
  int L = 0;
  int bits = 0;
  int log_scale = 0;
  double sigma = 0;
  int B = 0;
  std::vector<uint64_t> q;    // descending
  std::vector<uint64_t> psi;  // primitive 2N-th roots
  // special prime of key switching (ciphertext multiplication): the largest prime with
  // prime_bits bits, = 1 mod 2N, that is not one of q; 0 if there is none
  uint64_t qP = 0;
  uint64_t psiP = 0;
};

// Returns an empty string on success, else the reason (and sets *code to a CKKS_E* value).
std::string resolve(uint32_t log_n, uint32_t L, uint32_t bits, uint32_t log_scale, double sigma, uint32_t gauss_bound,
                    const uint64_t *primes, Resolved *out, int *code);

bool is_prime(uint64_t n);
uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t q);
uint64_t inv_mod(uint64_t a, uint64_t q);
uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t q);
uint64_t shoup_companion(uint64_t w, uint64_t q);  // floor(w * 2^64 / q)

// Gaussian cumulative table (2B entries) padded with all-ones to `slots` entries.
std::vector<uint64_t> cdt_table(double sigma, int B, int slots);
// T_j = 2^(log_scale + 1 - log_n) cos(pi j / N) and cos(pi j / N).
std::vector<double> encode_table(int log_n, int log_scale);
std::vector<double> cos_table(int log_n);

// Twiddles for the merged-psi transforms, stored as centered doubles:
// fwd[k] = psi^brv(k), inv[k] = psi^-brv(k), k < N.
void twiddles(uint64_t q, uint64_t psi, int log_n, std::vector<double> &fwd, std::vector<double> &inv);

// Centered double representative of a residue.
double centered(uint64_t r, uint64_t q);

}  // namespace host
}  // namespace ckks
