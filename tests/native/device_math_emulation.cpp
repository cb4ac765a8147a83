// Host emulation of the library's device arithmetic for CPU tests.
//
// The per-pass NTT functions, the FP64 modular arithmetic and the Philox samplers of
// the HIP library are host-callable; this file runs them for one emulated workgroup,
// thread by thread between the LDS exchanges, so the transforms, their layouts and
// their lazy-reduction schedule can be checked against the oracle without a GPU.
#include <math.h>
#include <stdint.h>

#include <vector>

#include "../../paper_2409_03568_amd/csrc/host_math.hpp"
#include "../../paper_2409_03568_amd/csrc/ntt.hpp"
#include "../../paper_2409_03568_amd/csrc/philox.hpp"

using namespace ckks;

namespace {

double g_max_abs = 0;

template <int LOGR>
void track(const std::vector<std::vector<double>> &X) {
  for (auto &v : X)
    for (double d : v) g_max_abs = fmax(g_max_abs, fabs(d));
}

template <int LOGN, int LOGR>
void fwd(std::vector<std::vector<double>> &X, const double *tw, double q, double qinv, uint32_t mask) {
  using S = NttShape<LOGN, LOGR>;
  std::vector<double> lds(S::N);
  double x[S::R];
  for (int t = 0; t < S::T; t++) {
    for (int r = 0; r < S::R; r++) x[r] = X[t][r];
    fwd_pass<LOGN, LOGR, 0>(x, t, tw, q, qinv, mask);
    for (int r = 0; r < S::R; r++) X[t][r] = x[r];
  }
  track<LOGR>(X);
  auto step = [&](auto pass_c) {
    constexpr int P = decltype(pass_c)::value;
    if constexpr (P >= 1 && P < S::NPASS) {
      for (int t = 0; t < S::T; t++) {
        for (int r = 0; r < S::R; r++) x[r] = X[t][r];
        lds_store<LOGN, LOGR, P - 1>(lds.data(), x, t);
      }
      for (int t = 0; t < S::T; t++) {
        lds_load<LOGN, LOGR, P>(lds.data(), x, t);
        fwd_pass<LOGN, LOGR, P>(x, t, tw, q, qinv, mask);
        for (int r = 0; r < S::R; r++) X[t][r] = x[r];
      }
      track<LOGR>(X);
    }
  };
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 3>{});
}

template <int LOGN, int LOGR>
void inv(std::vector<std::vector<double>> &X, const double *itw, double q, double qinv, uint32_t mask) {
  using S = NttShape<LOGN, LOGR>;
  constexpr int LAST = S::NPASS - 1;
  std::vector<double> lds(S::N);
  double x[S::R];
  for (int t = 0; t < S::T; t++) {
    for (int r = 0; r < S::R; r++) x[r] = X[t][r];
    inv_pass<LOGN, LOGR, LAST>(x, t, itw, q, qinv, mask);
    for (int r = 0; r < S::R; r++) X[t][r] = x[r];
  }
  track<LOGR>(X);
  auto step = [&](auto pass_c) {
    constexpr int P = decltype(pass_c)::value;
    if constexpr (P >= 0 && P < LAST) {
      for (int t = 0; t < S::T; t++) {
        for (int r = 0; r < S::R; r++) x[r] = X[t][r];
        lds_store<LOGN, LOGR, P + 1>(lds.data(), x, t);
      }
      for (int t = 0; t < S::T; t++) {
        lds_load<LOGN, LOGR, P>(lds.data(), x, t);
        inv_pass<LOGN, LOGR, P>(x, t, itw, q, qinv, mask);
        for (int r = 0; r < S::R; r++) X[t][r] = x[r];
      }
      track<LOGR>(X);
    }
  };
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 0>{});
}

// c = a * b in Z_q[X]/(X^N + 1): forward transforms of both, b_hat reduced and scaled by
// N^-1, pointwise product, inverse transform -- the sequence the encryption and decryption
// kernels use.  a_small: a holds small signed values (as v, s do), else canonical residues.
template <int LOGN, int LOGR>
int negacyclic(const int64_t *a, const uint64_t *b, uint64_t *c, uint64_t q, uint64_t psi, int a_small) {
  using S = NttShape<LOGN, LOGR>;
  std::vector<double> twf, twi;
  host::twiddles(q, psi, LOGN, twf, twi);
  const double qd = (double)q, qinv = 1.0 / qd;
  const uint32_t mf_small = host::forward_reduction_mask(LOGN, qd, 1.0);
  const uint32_t mf_big = host::forward_reduction_mask(LOGN, qd, qd);
  const uint32_t mi = host::inverse_reduction_mask(LOGN, qd, 0.75 * qd + 4);
  const double ninv = host::centered(host::inv_mod((uint64_t)S::N % q, q), q);
  std::vector<std::vector<double>> A(S::T, std::vector<double>(S::R)), Bv(S::T, std::vector<double>(S::R));
  for (int t = 0; t < S::T; t++)
    for (int r = 0; r < S::R; r++) {
      A[t][r] = (double)a[t + S::T * r];
      Bv[t][r] = (double)b[t + S::T * r];
    }
  fwd<LOGN, LOGR>(A, twf.data(), qd, qinv, a_small ? mf_small : mf_big);
  fwd<LOGN, LOGR>(Bv, twf.data(), qd, qinv, mf_big);
  for (int t = 0; t < S::T; t++)
    for (int r = 0; r < S::R; r++) {
      const double bh = reduce(mulmod(Bv[t][r], ninv, qd, qinv), qd, qinv);
      A[t][r] = mulmod(A[t][r], bh, qd, qinv);
    }
  track<LOGR>(A);
  inv<LOGN, LOGR>(A, twi.data(), qd, qinv, mi);
  for (int t = 0; t < S::T; t++)
    for (int r = 0; r < S::R; r++) c[t + S::T * r] = (uint64_t)canon(A[t][r], qd, qinv);
  return 0;
}

}  // namespace

extern "C" {

int emu_negacyclic(const int64_t *a, const uint64_t *b, uint64_t *c, int log_n, uint64_t q, uint64_t psi, int a_small) {
  switch (log_n) {
    case 11: return negacyclic<11, 5>(a, b, c, q, psi, a_small);
    case 12: return negacyclic<12, 5>(a, b, c, q, psi, a_small);
    case 13: return negacyclic<13, 5>(a, b, c, q, psi, a_small);
    case 14: return negacyclic<14, 5>(a, b, c, q, psi, a_small);
    default: return -1;
  }
}

double emu_max_abs(void) { return g_max_abs; }
void emu_reset_max(void) { g_max_abs = 0; }

double emu_mulmod(double a, double w, double q) { return mulmod(a, w, q, 1.0 / q); }
double emu_reduce(double x, double q) { return reduce(x, q, 1.0 / q); }
double emu_canon(double x, double q) { return canon(x, q, 1.0 / q); }
double emu_center(double x, double q) { return center(x, q, 1.0 / q); }
uint64_t emu_mul_shoup(uint64_t a, uint64_t w, uint64_t q) { return mul_shoup(a, w, host::shoup_companion(w, q), q); }
uint64_t emu_mod_i64(int64_t x, uint64_t q) { return mod_i64(x, q, 1.0 / (double)q); }
uint64_t emu_residue_of_double(double x, uint64_t q) { return residue_of_double(x, q, 1.0 / (double)q); }
void emu_philox(const uint64_t *ctr, const uint64_t *key, uint64_t *out) {
  Philox4 p = philox4x64_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
  for (int i = 0; i < 4; i++) out[i] = p.w[i];
}
int emu_ternary(uint64_t w) { return ternary_of(w); }
int emu_gauss(uint64_t w, double sigma, int B) {
  std::vector<uint64_t> T = host::cdt_table(sigma, B, kCdtSlots);
  return gauss_of(w, T.data(), B);
}
uint32_t emu_fwd_mask(int log_n, double qmax, double in_bound) { return host::forward_reduction_mask(log_n, qmax, in_bound); }
uint32_t emu_inv_mask(int log_n, double qmax, double in_bound) { return host::inverse_reduction_mask(log_n, qmax, in_bound); }
}
