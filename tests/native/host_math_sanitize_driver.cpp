// Runs the library's host-side setup arithmetic (parameter resolution, primes, roots,
// Gaussian and encoding tables, twiddles) for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py), checking a few invariants:
// every twiddle times its inverse is 1, psi^N = -1, the tables have their sizes; invalid
// parameter sets are refused without touching memory out of bounds.  Prints "OK".
#include <stdio.h>
#include <stdlib.h>

#include <cmath>

#include "../../paper_2409_03568_amd/csrc/host_math.hpp"

using namespace ckks::host;

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__); \
      exit(1);                                                 \
    }                                                          \
  } while (0)

static uint64_t from_centered(double x, uint64_t q) {
  const long long v = (long long)x;
  return v < 0 ? (uint64_t)(v + (long long)q) : (uint64_t)v;
}

int main() {
  const unsigned sets[][4] = {{11, 2, 30, 20}, {12, 3, 36, 30}, {13, 4, 50, 40}, {14, 2, 50, 40}, {12, 8, 36, 30}};
  for (auto &p : sets) {
    Resolved r;
    int code = 0;
    const std::string why = resolve(p[0], p[1], p[2], p[3], 3.2, 0, nullptr, &r, &code);
    CHECK(why.empty() && code == 0);
    CHECK((int)r.q.size() == (int)p[1] && r.B == 19);
    const uint64_t N = 1ull << p[0];
    for (int i = 0; i < r.L; i++) {
      const uint64_t q = r.q[(size_t)i];
      CHECK(is_prime(q) && q % (2 * N) == 1);
      CHECK(pow_mod(r.psi[(size_t)i], N, q) == q - 1);
      std::vector<double> f, iv;
      twiddles(q, r.psi[(size_t)i], (int)p[0], f, iv);
      CHECK(f.size() == N && iv.size() == N);
      for (uint64_t k = 0; k < N; k += 7)
        CHECK(mul_mod(from_centered(f[k], q), from_centered(iv[k], q), q) == 1);
      CHECK(mul_mod(inv_mod(12345 % q, q), 12345 % q, q) == 1);
      (void)shoup_companion(q - 1, q);
    }
    CHECK(cdt_table(3.2, r.B, 128).size() == 128);
    const std::vector<double> T = encode_table((int)p[0], (int)p[3]), C = cos_table((int)p[0]);
    CHECK(T.size() == N && C.size() == N && C[0] == 1.0);
  }
  // refused parameter sets
  const unsigned bad[][4] = {{10, 2, 30, 20}, {15, 2, 30, 20}, {12, 0, 36, 30}, {12, 17, 36, 30},
                             {12, 3, 19, 10}, {12, 3, 51, 30}, {12, 3, 36, 40}};
  for (auto &p : bad) {
    Resolved r;
    int code = 0;
    const std::string why = resolve(p[0], p[1], p[2], p[3], 3.2, 0, nullptr, &r, &code);
    CHECK(!why.empty() && code != 0);
  }
  {
    Resolved r;
    int code = 0;
    const uint64_t not_ntt[2] = {1000003, 1000033};
    CHECK(!resolve(12, 2, 20, 10, 3.2, 0, not_ntt, &r, &code).empty() && code != 0);
    CHECK(!resolve(12, 2, 36, 30, 3.2, 64, nullptr, &r, &code).empty());  // Gaussian bound above 63
  }
  printf("OK\n");
  return 0;
}
