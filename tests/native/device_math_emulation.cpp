// Host emulation of the library's device arithmetic for CPU tests.
//
// The per-pass NTT functions, the FP64 modular arithmetic and the Philox samplers of
// the HIP library are host-callable; this file runs them for one emulated workgroup,
// thread by thread between the LDS exchanges, so the transforms, their layouts, the LDS
// placement and the compiled lazy-reduction schedules can be checked against the oracle
// without a GPU.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "../../paper_2409_03568_amd/csrc/host_math.hpp"
#include "../../paper_2409_03568_amd/csrc/ntt.hpp"
#include "../../paper_2409_03568_amd/csrc/philox.hpp"

using namespace ckks;

namespace {

double g_max_abs = 0;
bool g_lds_bijective = true;
bool g_lds_conflict_free = true;

// Every access of an exchange (one register, one quarter-wave of 16 lanes) must fall on 16
// different 8-byte banks (slot mod 16).
template <int LOGN, int LOGR, int PASS>
void check_banks() {
  using S = NttShape<LOGN, LOGR>;
  for (int r = 0; r < S::R; r++)
    for (int q0 = 0; q0 < S::T; q0 += 16) {
      unsigned seen = 0;
      for (int t = q0; t < q0 + 16 && t < S::T; t++) seen |= 1u << (lds_pos<LOGR>(elem_index<LOGN, LOGR, PASS>(t, r)) & 15u);
      if (seen != 0xffffu) g_lds_conflict_free = false;
    }
}
bool g_wave_local_ok = true;
int g_wave_local_count = 0;

// An exchange from the layout of pass A to that of pass B that the kernels run without a
// workgroup barrier must have every wave write exactly the LDS slots it then reads.
template <int LOGN, int LOGR, int A, int B>
void check_wave_local() {
  using S = NttShape<LOGN, LOGR>;
  if constexpr (S::same_wave_sets(A, B)) {
    g_wave_local_count++;
    for (int w = 0; w * 64 < S::T; w++) {
      std::vector<unsigned> wr, rd;
      for (int t = w * 64; t < w * 64 + 64 && t < S::T; t++)
        for (int r = 0; r < S::R; r++) {
          wr.push_back(lds_pos<LOGR>(elem_index<LOGN, LOGR, A>(t, r)));
          rd.push_back(lds_pos<LOGR>(elem_index<LOGN, LOGR, B>(t, r)));
        }
      std::sort(wr.begin(), wr.end());
      std::sort(rd.begin(), rd.end());
      if (wr != rd) g_wave_local_ok = false;
    }
  }
}

void track(const std::vector<std::vector<double>> &X) {
  for (auto &v : X)
    for (double d : v) g_max_abs = fmax(g_max_abs, fabs(d));
}

template <int LOGN, int LOGR, uint32_t RED>
void fwd(std::vector<std::vector<double>> &X, const double *tw, double q, double qinv) {
  using S = NttShape<LOGN, LOGR>;
  std::vector<double> lds(LdsSlots<LOGN, LOGR>::value);
  double x[S::R];
  for (int t = 0; t < S::T; t++) {
    for (int r = 0; r < S::R; r++) x[r] = X[t][r];
    PassTw<LOGN, LOGR, 0> w;
    tw_prefetch<LOGN, LOGR, 0>(w, t, tw);
    fwd_pass<LOGN, LOGR, 0, RED>(x, t, tw, w, q, qinv);
    for (int r = 0; r < S::R; r++) X[t][r] = x[r];
  }
  track(X);
  auto step = [&](auto pass_c) {
    constexpr int P = decltype(pass_c)::value;
    if constexpr (P >= 1 && P < S::NPASS) {
      check_wave_local<LOGN, LOGR, P - 1, P>();
      check_banks<LOGN, LOGR, P - 1>();
      check_banks<LOGN, LOGR, P>();
      std::vector<int> hit(LdsSlots<LOGN, LOGR>::value, 0);
      for (int t = 0; t < S::T; t++) {
        for (int r = 0; r < S::R; r++) {
          x[r] = X[t][r];
          const unsigned e = elem_index<LOGN, LOGR, P - 1>(t, r);
          hit[lds_pos<LOGR>(e)]++;
          // the split the kernels use: thread base plus a per-register offset
          const unsigned et = elem_index<LOGN, LOGR, P - 1>(t, 0), er = elem_index<LOGN, LOGR, P - 1>(0, r);
          if ((et & er) != 0 || (et | er) != e ||
              lds_pos<LOGR>(e) != lds_slot(lds_pos<LOGR>(et), lds_pos<LOGR>(er)))
            g_lds_bijective = false;
        }
        lds_store<LOGN, LOGR, P - 1>(lds.data(), x, t);
      }
      for (int h : hit) g_lds_bijective = g_lds_bijective && h <= 1;
      for (int t = 0; t < S::T; t++) {
        lds_load<LOGN, LOGR, P>(lds.data(), x, t);
        PassTw<LOGN, LOGR, P> w;
        tw_prefetch<LOGN, LOGR, P>(w, t, tw);
        fwd_pass<LOGN, LOGR, P, RED>(x, t, tw, w, q, qinv);
        for (int r = 0; r < S::R; r++) X[t][r] = x[r];
      }
      track(X);
    }
  };
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 3>{});
  step(std::integral_constant<int, 4>{});
}

template <int LOGN, int LOGR, uint32_t RED>
void inv(std::vector<std::vector<double>> &X, const double *itw, double q, double qinv) {
  using S = NttShape<LOGN, LOGR>;
  constexpr int LAST = S::NPASS - 1;
  std::vector<double> lds(LdsSlots<LOGN, LOGR>::value);
  double x[S::R];
  for (int t = 0; t < S::T; t++) {
    for (int r = 0; r < S::R; r++) x[r] = X[t][r];
    PassTw<LOGN, LOGR, LAST> w;
    tw_prefetch<LOGN, LOGR, LAST>(w, t, itw);
    inv_pass<LOGN, LOGR, LAST, RED>(x, t, itw, w, q, qinv);
    for (int r = 0; r < S::R; r++) X[t][r] = x[r];
  }
  track(X);
  auto step = [&](auto pass_c) {
    constexpr int P = decltype(pass_c)::value;
    if constexpr (P >= 0 && P < LAST) {
      check_wave_local<LOGN, LOGR, P + 1, P>();
      for (int t = 0; t < S::T; t++) {
        for (int r = 0; r < S::R; r++) x[r] = X[t][r];
        lds_store<LOGN, LOGR, P + 1>(lds.data(), x, t);
      }
      for (int t = 0; t < S::T; t++) {
        lds_load<LOGN, LOGR, P>(lds.data(), x, t);
        PassTw<LOGN, LOGR, P> w;
        tw_prefetch<LOGN, LOGR, P>(w, t, itw);
        inv_pass<LOGN, LOGR, P, RED>(x, t, itw, w, q, qinv);
        for (int r = 0; r < S::R; r++) X[t][r] = x[r];
      }
      track(X);
    }
  };
  step(std::integral_constant<int, 3>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 0>{});
}

// c = a * b in Z_q[X]/(X^N + 1): forward transforms of both, b_hat reduced and scaled by
// N^-1, pointwise product, inverse transform -- the sequence the encryption and decryption
// kernels use.  a_small: a holds small signed values (as v, s do), else canonical residues.
template <int LOGN, int LOGR, int RC>
int negacyclic(const int64_t *a, const uint64_t *b, uint64_t *c, uint64_t q, uint64_t psi, int a_small) {
  using S = NttShape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  if ((double)q > Red::qmax) return -2;
  std::vector<double> twf, twi;
  host::twiddles(q, psi, LOGN, twf, twi);
  const double qd = (double)q, qinv = 1.0 / qd;
  const double ninv = host::centered(host::inv_mod((uint64_t)S::N % q, q), q);
  std::vector<std::vector<double>> A(S::T, std::vector<double>(S::R)), Bv(S::T, std::vector<double>(S::R));
  for (int t = 0; t < S::T; t++)
    for (int r = 0; r < S::R; r++) {
      A[t][r] = (double)a[t + S::T * r];
      Bv[t][r] = (double)b[t + S::T * r];
    }
  if (a_small)
    fwd<LOGN, LOGR, Red::fwd_small>(A, twf.data(), qd, qinv);
  else
    fwd<LOGN, LOGR, Red::fwd_big>(A, twf.data(), qd, qinv);
  fwd<LOGN, LOGR, Red::fwd_big>(Bv, twf.data(), qd, qinv);
  for (int t = 0; t < S::T; t++)
    for (int r = 0; r < S::R; r++) {
      const double bh = reduce(mulmod(Bv[t][r], ninv, qd, qinv), qd, qinv);
      A[t][r] = mulmod(A[t][r], bh, qd, qinv);
    }
  track(A);
  inv<LOGN, LOGR, Red::inv>(A, twi.data(), qd, qinv);
  for (int t = 0; t < S::T; t++)
    for (int r = 0; r < S::R; r++) c[t + S::T * r] = (uint64_t)canon(A[t][r], qd, qinv);
  return 0;
}

template <int LOGN>
int negacyclic_shape(const int64_t *a, const uint64_t *b, uint64_t *c, uint64_t q, uint64_t psi, int a_small, int logr,
                     int rc) {
  if (logr == 3) return rc ? negacyclic<LOGN, 3, 1>(a, b, c, q, psi, a_small) : negacyclic<LOGN, 3, 0>(a, b, c, q, psi, a_small);
  if (logr == 4) return rc ? negacyclic<LOGN, 4, 1>(a, b, c, q, psi, a_small) : negacyclic<LOGN, 4, 0>(a, b, c, q, psi, a_small);
  if (logr == 5) return rc ? negacyclic<LOGN, 5, 1>(a, b, c, q, psi, a_small) : negacyclic<LOGN, 5, 0>(a, b, c, q, psi, a_small);
  return -1;
}

}  // namespace

extern "C" {

int emu_negacyclic(const int64_t *a, const uint64_t *b, uint64_t *c, int log_n, uint64_t q, uint64_t psi, int a_small,
                   int logr, int rc) {
  switch (log_n) {
    case 11: return negacyclic_shape<11>(a, b, c, q, psi, a_small, logr, rc);
    case 12: return negacyclic_shape<12>(a, b, c, q, psi, a_small, logr, rc);
    case 13: return negacyclic_shape<13>(a, b, c, q, psi, a_small, logr, rc);
    case 14: return negacyclic_shape<14>(a, b, c, q, psi, a_small, logr, rc);
    default: return -1;
  }
}

double emu_max_abs(void) { return g_max_abs; }
int emu_lds_bijective(void) { return g_lds_bijective ? 1 : 0; }
int emu_lds_conflict_free(void) { return g_lds_conflict_free ? 1 : 0; }
int emu_wave_local_ok(void) { return g_wave_local_ok ? 1 : 0; }
int emu_wave_local_count(void) { return g_wave_local_count; }
void emu_reset_max(void) {
  g_max_abs = 0;
  g_lds_bijective = true;
  g_lds_conflict_free = true;
  g_wave_local_ok = true;
  g_wave_local_count = 0;
}

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
uint32_t emu_fwd_mask(int log_n, double qmax, double in_bound) { return forward_schedule(log_n, qmax, in_bound).mask; }
uint32_t emu_inv_mask(int log_n, double qmax, double in_bound) { return inverse_schedule(log_n, qmax, in_bound); }
}
