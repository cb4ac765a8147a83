// Negacyclic NTT over Z_q[X]/(X^N+1) for one workgroup, register-blocked.
//
// The product of two ring elements (Sec. 2.2: every ciphertext product v*pk and the
// decryption product c1*s) is a pointwise product after a negacyclic transform.  The
// forward transform is the merged-psi Cooley-Tukey network: stage s (s = 0..logN-1)
// pairs elements e and e + N/2^(s+1) with twiddle psi^brv(2^s + e >> (logN - s)), so the
// output is in bit-reversed order.  The inverse runs the Gentleman-Sande network with
// psi^-1 in the same table positions; its factor N is folded into the operand the
// caller multiplies by.
//
// Work split: the T = N / R threads of the workgroup each hold R = 2^LOGR values in
// registers.  The stages are grouped into passes of LOGR stages (the last pass takes
// the remainder); inside a pass every butterfly is between two registers of the same
// thread, and between passes the values are exchanged through LDS (N doubles).  In the
// first pass thread `tid` holds elements tid + T*r (so global loads and stores of the
// coefficient-domain data are coalesced); in the last pass it holds groups of 2^P
// consecutive elements, which is also where the pointwise product happens.
#pragma once
#include "modarith.hpp"

namespace ckks {

template <int LOGN, int LOGR>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = 1 << LOGR;
  static constexpr int T = N / R;
  static constexpr int NPASS = (LOGN + LOGR - 1) / LOGR;
  static constexpr int start(int p) { return p * LOGR; }
  static constexpr int len(int p) { return p == NPASS - 1 ? LOGN - p * LOGR : LOGR; }
};

// Element index held in register r by thread tid during pass PASS.
template <int LOGN, int LOGR, int PASS>
CKKS_HD int elem_index(int tid, int r) {
  using S = NttShape<LOGN, LOGR>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS);
  constexpr int LTLO = LOGN - S0 - P;  // log2 of the smallest butterfly distance in the pass
  const int u = r >> P, k = r & ((1 << P) - 1);
  const int g = tid + S::T * u;
  const int blk = g >> LTLO, off = g & ((1 << LTLO) - 1);
  return (blk << (LOGN - S0)) + (k << LTLO) + off;
}

// Forward (Cooley-Tukey) stages of one pass.  red_mask bit s: reduce every value after stage s.
template <int LOGN, int LOGR, int PASS>
CKKS_HD void fwd_pass(double (&x)[1 << LOGR], int tid, const double *__restrict__ tw, double q,
                                         double qinv, uint32_t red_mask) {
  using S = NttShape<LOGN, LOGR>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS), G = S::R >> P;
  constexpr int LTLO = LOGN - S0 - P;
#pragma unroll
  for (int u = 0; u < G; u++) {
    const int g = tid + S::T * u;
    const int blk = g >> LTLO;
#pragma unroll
    for (int l = 0; l < P; l++) {
      const int s = S0 + l;
      const int half = 1 << (P - 1 - l);
#pragma unroll
      for (int k = 0; k < (1 << P); k++) {
        if (k & half) continue;
        const double W = tw[(1 << s) + (blk << l) + (k >> (P - l))];
        ct_butterfly(x[u * (1 << P) + k], x[u * (1 << P) + k + half], W, q, qinv);
      }
      if ((red_mask >> s) & 1u) {
#pragma unroll
        for (int k = 0; k < (1 << P); k++) x[u * (1 << P) + k] = reduce(x[u * (1 << P) + k], q, qinv);
      }
    }
  }
}

// Inverse (Gentleman-Sande) stages of one pass, in decreasing stage order.
// red_mask bit s: reduce the sum outputs after stage s.
template <int LOGN, int LOGR, int PASS>
CKKS_HD void inv_pass(double (&x)[1 << LOGR], int tid, const double *__restrict__ itw, double q,
                                         double qinv, uint32_t red_mask) {
  using S = NttShape<LOGN, LOGR>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS), G = S::R >> P;
  constexpr int LTLO = LOGN - S0 - P;
#pragma unroll
  for (int u = 0; u < G; u++) {
    const int g = tid + S::T * u;
    const int blk = g >> LTLO;
#pragma unroll
    for (int l = P - 1; l >= 0; l--) {
      const int s = S0 + l;
      const int half = 1 << (P - 1 - l);
      const bool red = (red_mask >> s) & 1u;
#pragma unroll
      for (int k = 0; k < (1 << P); k++) {
        if (k & half) continue;
        const double W = itw[(1 << s) + (blk << l) + (k >> (P - l))];
        double &X = x[u * (1 << P) + k];
        double &Y = x[u * (1 << P) + k + half];
        gs_butterfly(X, Y, W, q, qinv);
        if (red) X = reduce(X, q, qinv);
      }
    }
  }
}

template <int LOGN, int LOGR, int PASS>
CKKS_HD void lds_store(double *lds, const double (&x)[1 << LOGR], int tid) {
#pragma unroll
  for (int r = 0; r < (1 << LOGR); r++) lds[elem_index<LOGN, LOGR, PASS>(tid, r)] = x[r];
}

template <int LOGN, int LOGR, int PASS>
CKKS_HD void lds_load(const double *lds, double (&x)[1 << LOGR], int tid) {
#pragma unroll
  for (int r = 0; r < (1 << LOGR); r++) x[r] = lds[elem_index<LOGN, LOGR, PASS>(tid, r)];
}

// Passes 1..NPASS-1 of the forward transform (pass 0 is run by the caller on the
// first-pass layout); ends with x in the last-pass layout.  Contains barriers: every
// thread of the workgroup must call it.
template <int LOGN, int LOGR, int PASS = 1>
__device__ __forceinline__ void fwd_rest(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ tw,
                                         double q, double qinv, uint32_t red_mask) {
  if constexpr (PASS < NttShape<LOGN, LOGR>::NPASS) {
    __syncthreads();
    lds_store<LOGN, LOGR, PASS - 1>(lds, x, tid);
    __syncthreads();
    lds_load<LOGN, LOGR, PASS>(lds, x, tid);
    fwd_pass<LOGN, LOGR, PASS>(x, tid, tw, q, qinv, red_mask);
    fwd_rest<LOGN, LOGR, PASS + 1>(x, lds, tid, tw, q, qinv, red_mask);
  }
}

// Whole forward transform from the first-pass layout to the last-pass layout.
template <int LOGN, int LOGR>
__device__ __forceinline__ void ntt_forward(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ tw,
                                            double q, double qinv, uint32_t red_mask) {
  fwd_pass<LOGN, LOGR, 0>(x, tid, tw, q, qinv, red_mask);
  fwd_rest<LOGN, LOGR, 1>(x, lds, tid, tw, q, qinv, red_mask);
}

template <int LOGN, int LOGR, int PASS>
__device__ __forceinline__ void inv_rest(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ itw,
                                         double q, double qinv, uint32_t red_mask) {
  if constexpr (PASS >= 0) {
    __syncthreads();
    lds_store<LOGN, LOGR, PASS + 1>(lds, x, tid);
    __syncthreads();
    lds_load<LOGN, LOGR, PASS>(lds, x, tid);
    inv_pass<LOGN, LOGR, PASS>(x, tid, itw, q, qinv, red_mask);
    inv_rest<LOGN, LOGR, PASS - 1>(x, lds, tid, itw, q, qinv, red_mask);
  }
}

// Whole inverse transform (without the factor 1/N) from the last-pass layout to the
// first-pass layout.
template <int LOGN, int LOGR>
__device__ __forceinline__ void ntt_inverse(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ itw,
                                            double q, double qinv, uint32_t red_mask) {
  constexpr int LAST = NttShape<LOGN, LOGR>::NPASS - 1;
  inv_pass<LOGN, LOGR, LAST>(x, tid, itw, q, qinv, red_mask);
  inv_rest<LOGN, LOGR, LAST - 1>(x, lds, tid, itw, q, qinv, red_mask);
}

}  // namespace ckks
