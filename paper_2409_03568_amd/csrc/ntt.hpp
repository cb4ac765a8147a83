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
//
// Lazy reduction: values are signed and grow through the stages; a reduction after
// stage s is compiled in when bit s of the schedule is set.  The schedules are fixed at
// compile time per reduction class (class 0: primes small enough to need none; class 1:
// primes below 2^50), derived from worst-case magnitude bounds so that forward values
// stay below 2^52 and inverse values below 2^51 (see modarith.hpp for the bounds of the
// primitive operations).
#pragma once
#include "modarith.hpp"

namespace ckks {

// Pass structure of a transform over N = 2^LOGN values, R = 2^LOGR per thread: the
// stages are split into NPASS passes, the first of FIRST (1..LOGR) stages and the others
// of LOGR.  Putting the short pass first keeps the last passes' thread layouts equal on
// the wave-index bits, so their exchanges stay inside a wave (see same_wave_sets).
template <int LOGN, int LOGR>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = 1 << LOGR;
  static constexpr int T = N / R;
  static constexpr int NPASS = (LOGN + LOGR - 1) / LOGR;
  static constexpr int FIRST = LOGN - (NPASS - 1) * LOGR;
  static constexpr int start(int p) { return p == 0 ? 0 : FIRST + (p - 1) * LOGR; }
  static constexpr int len(int p) { return p == 0 ? FIRST : LOGR; }
  // element-index bit that bit b of the thread index occupies in pass p (see elem_index)
  static constexpr int tid_bit_pos(int p, int b) {
    return b < LOGN - start(p) - len(p) ? b : b + len(p);
  }
  // true when every wave holds the same set of elements in passes a and b: the wave-index
  // bits of the thread index (bits 6 and up) sit at the same element bits in both
  static constexpr bool same_wave_sets(int a, int b) {
    for (int t = 6; (1 << t) < T; t++)
      if (tid_bit_pos(a, t) != tid_bit_pos(b, t)) return false;
    return true;
  }
};

// ---------------------------------------------------------------------------
// reduction schedules
// ---------------------------------------------------------------------------
// Bounds on magnitudes (q <= qmax):  mulmod(a, w), |w| <= q/2:  |r| <= q/2 + |a| q 2^-53 + 1;
// reduce(x): |r| <= q/2 + 1.  A stage is followed by a reduction when its outputs could
// exceed 2^51.  The bounds grow with q, so a schedule derived for qmax serves every
// smaller prime.
// Forward (Cooley-Tukey) stages add a product to a value: X +- W*Y.  The product
// precondition |Y W / q| < 2^51 holds for |Y| below 2^52 (|W| <= q/2), so forward values
// may grow to just under 2^52.  Inverse (Gentleman-Sande) stages form X - Y before the
// product, so their values are kept below 2^51 (the difference then stays below 2^52).
constexpr double kFwdLimit = 4222124650659840.0;  // 2^52 - 2^48
constexpr double kInvLimit = 2251799813685248.0;  // 2^51
constexpr double kTwoPowMinus53 = 1.0 / 9007199254740992.0;

// Flag bit of a forward schedule (above every stage bit): the transform's inputs are
// integers in {-1, 0, 1}, so each first-stage product W*Y is an exact double (|W| <= q/2)
// and needs no modular reduction.
constexpr uint32_t kFwdTernaryInput = 1u << 31;

struct FwdPlan {
  uint32_t mask;  // reduce after stage s when bit s is set
  double bound;   // bound on the outputs
};

constexpr FwdPlan forward_schedule(int log_n, double qmax, double input_bound) {
  uint32_t mask = 0;
  double M = input_bound;
  for (int s = 0; s < log_n; s++) {
    M = M + (qmax / 2 + M * qmax * kTwoPowMinus53 + 1);
    if (M > kFwdLimit) {
      mask |= 1u << s;
      M = qmax / 2 + 2;
    }
  }
  return FwdPlan{mask, M};
}

// Inverse: the sum output doubles, the difference output goes through a product; only
// the sum outputs are reduced.
constexpr uint32_t inverse_schedule(int log_n, double qmax, double input_bound) {
  uint32_t mask = 0;
  double M = input_bound;
  for (int s = log_n - 1; s >= 0; s--) {
    const double prod = qmax / 2 + 2 * M * qmax * kTwoPowMinus53 + 1;
    double sum = 2 * M;
    if (sum > kInvLimit) {
      mask |= 1u << s;
      sum = qmax / 2 + 2;
    }
    M = sum > prod ? sum : prod;
  }
  return mask;
}

// Pointwise product of a forward output (bound M) with a reduced key (|w| <= q/2 + 2).
constexpr double pointwise_bound(double qmax, double M) { return qmax / 2 + M * (qmax / 2 + 2) * 2 * kTwoPowMinus53 + 1; }

// Inputs of the transforms: small signed values (ternary, |x| <= 1) or canonical
// residues (< q); the inverse starts from pointwise products of either's output.
constexpr double kClassQmax[2] = {1099511627776.0 /* 2^40 */, 1125899906842624.0 /* 2^50 */};

template <int LOGN, int RC>
struct Schedule {
  static constexpr double qmax = kClassQmax[RC];
  static constexpr FwdPlan small = forward_schedule(LOGN, qmax, 1.0);
  static constexpr FwdPlan big = forward_schedule(LOGN, qmax, qmax);
  static constexpr uint32_t fwd_small = small.mask | kFwdTernaryInput;
  static constexpr uint32_t fwd_big = big.mask;
  static constexpr double inv_input =
      pointwise_bound(qmax, small.bound > big.bound ? small.bound : big.bound);
  static constexpr uint32_t inv = inverse_schedule(LOGN, qmax, inv_input);
  static_assert(small.bound <= kFwdLimit && big.bound <= kFwdLimit, "forward bound");
};

// ---------------------------------------------------------------------------
// layouts
// ---------------------------------------------------------------------------
// Element index held in register r by thread tid during pass PASS.  A pass of P stages
// splits r into the butterfly index k (P bits) and, when P < LOGR, a group index u:
// r = k * G + u with G = R / 2^P, so that in the first pass register r of thread tid
// holds element tid + T * r (the coefficient order the kernels load and store).
// (Indices are unsigned 32-bit so that loads can address a uniform base plus a 32-bit
// per-lane offset instead of building a 64-bit address per load.)
template <int LOGN, int LOGR, int PASS>
CKKS_HD unsigned elem_index(unsigned tid, unsigned r) {
  using S = NttShape<LOGN, LOGR>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS);
  constexpr int LTLO = LOGN - S0 - P;  // log2 of the smallest butterfly distance in the pass
  const unsigned u = r & ((1u << (LOGR - P)) - 1), k = r >> (LOGR - P);
  const unsigned g = tid + (unsigned)S::T * u;
  // in the first pass every g is below 2^LTLO, so blk = 0 (stated, for the compiler)
  const unsigned blk = PASS == 0 ? 0u : g >> LTLO, off = PASS == 0 ? g : g & ((1u << LTLO) - 1);
  return (blk << (LOGN - S0)) + (k << LTLO) + off;
}

// LDS position of element e: an XOR swizzle of the low four index bits with the four bits
// above bit LOGR, e ^ ((e >> LOGR) & 15) -- a permutation, so the exchange needs N slots
// and no padding.  The LDS serves one quarter-wave (16 lanes) of 8-byte accesses per
// cycle from 16 8-byte banks (slot mod 16).  In every pass the 16 lanes of a quarter
// differ in four element bits: bits 0..3 (passes whose smallest butterfly distance is at
// least 16), or bits 0..L-1 together with L+P..3+P (distance 2^L < 16, P stages), or bits
// P..P+3 (distance 1); in each case the swizzle maps those bits one to one onto the four
// bank bits, so no access of an exchange has a bank conflict.
template <int LOGR>
CKKS_HD unsigned lds_pos(unsigned e) { return e ^ ((e >> LOGR) & 15u); }
template <int LOGN, int LOGR>
struct LdsSlots {
  static constexpr int value = 1 << LOGN;
};
// Slot of element t | r (thread part t, register part r on disjoint bits) from tb =
// lds_pos(t) and pr = lds_pos(r): the swizzle is linear over XOR, so the slot is tb ^ pr;
// the bits of pr above bit 3 are those of r, disjoint from tb's, so they can be added as
// a compile-time offset and only pr's low four bits need an XOR with the base.
CKKS_HD unsigned lds_slot(unsigned tb, unsigned pr) { return (tb ^ (pr & 15u)) + (pr & ~15u); }

// ---------------------------------------------------------------------------
// passes
// ---------------------------------------------------------------------------
// Element idx of a table whose base is the same for the whole launch: the byte offset is
// a 32-bit value, so the load can take the base from scalar registers and the offset from
// one vector register instead of building a 64-bit address per load.
CKKS_HD double ld_table(const double *__restrict__ base, unsigned idx) {
  return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + (idx << 3));
}

// The same for one row of 64-bit words (a limb of a ciphertext or of a scratch buffer):
// the row's base is uniform, idx < 2^29.
CKKS_HD const uint64_t *word_at(const uint64_t *base, unsigned idx) {
  return reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(base) + (idx << 3));
}
CKKS_HD uint64_t *word_at(uint64_t *base, unsigned idx) {
  return reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(base) + (idx << 3));
}
CKKS_HD uint64_t ld_word(const uint64_t *base, unsigned idx) { return *word_at(base, idx); }
CKKS_HD void st_word(uint64_t *base, unsigned idx, uint64_t v) { *word_at(base, idx) = v; }

// The thread index as a value the compiler cannot prove loop-invariant: address
// arithmetic derived from it stays next to its use instead of being hoisted out of the
// per-ciphertext loops, where dozens of precomputed pointers would stay live.
CKKS_HD int opaque(int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(v));
#endif
  return v;
}


// Keeps the device scheduler from interleaving consecutive stages: a pass compiles to
// one straight-line block, and hoisting later stages' loads and arithmetic over earlier
// ones raises register pressure past what two waves per SIMD can hold.
CKKS_HD void stage_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// Twiddles of one pass.  Stage l of the pass (global stage s = start + l) uses the 2^l
// factors tw[2^s + (blk << l) + t], t < 2^l, of each of the thread's G groups; slot
// (2^l - 1 + t) of a group holds factor t.  Where a pass needs few of them they are
// loaded into registers before the pass's LDS exchange, so their latency hides behind
// the barriers instead of stalling every stage.
template <int LOGN, int LOGR, int PASS>
struct PassTw {
  using S = NttShape<LOGN, LOGR>;
  static constexpr int P = S::len(PASS), G = S::R >> P, PER = (1 << P) - 1, COUNT = G * PER;
  static constexpr bool kPrefetch = COUNT <= 8;
  static constexpr int SLOTS = kPrefetch ? COUNT : 1;
  double w[SLOTS];  // the prefetched factors (unused without prefetch)
};

template <int LOGN, int LOGR, int PASS>
CKKS_HD void tw_prefetch(PassTw<LOGN, LOGR, PASS> &regs, int tid_in, const double *__restrict__ tw) {
  using S = NttShape<LOGN, LOGR>;
  using PT = PassTw<LOGN, LOGR, PASS>;
  double *w = regs.w;
  if constexpr (PT::kPrefetch) {
    const int tid = opaque(tid_in);
    constexpr int S0 = S::start(PASS), P = PT::P, LTLO = LOGN - S0 - P;
#pragma unroll
    for (int u = 0; u < PT::G; u++) {
      // first pass: blk = 0, so its factors are the same for every thread (scalar loads)
      const unsigned blk = PASS == 0 ? 0u : ((unsigned)tid + (unsigned)S::T * u) >> LTLO;
#pragma unroll
      for (int l = 0; l < P; l++)
#pragma unroll
        for (int t = 0; t < (1 << l); t++)
          w[u * PT::PER + (1 << l) - 1 + t] = ld_table(tw, (1u << (S0 + l)) + (blk << l) + t);
    }
  }
}

// Forward (Cooley-Tukey) stages of one pass; reduce every value after stage s if bit s of
// RED.  Twiddles come from w when the pass prefetches them, else from tw.
template <int LOGN, int LOGR, int PASS, uint32_t RED>
CKKS_HD void fwd_pass(double (&x)[1 << LOGR], int tid_in, const double *__restrict__ tw,
                      const PassTw<LOGN, LOGR, PASS> &regs, double q, double qinv) {
  const int tid = opaque(tid_in);
  using S = NttShape<LOGN, LOGR>;
  using PT = PassTw<LOGN, LOGR, PASS>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS), G = S::R >> P;
  constexpr int LTLO = LOGN - S0 - P;
#pragma unroll
  for (int u = 0; u < G; u++) {
    const unsigned g = (unsigned)tid + (unsigned)S::T * u;
    const unsigned blk = PASS == 0 ? 0u : g >> LTLO;
#pragma unroll
    for (int l = 0; l < P; l++) {
      const int s = S0 + l;
      const int half = 1 << (P - 1 - l);
#pragma unroll
      for (int k = 0; k < (1 << P); k++) {
        if (k & half) continue;
        const unsigned t = (unsigned)(k >> (P - l));
        double W;
        if constexpr (PT::kPrefetch)
          W = regs.w[u * PT::PER + (1 << l) - 1 + t];
        else
          W = ld_table(tw, (1u << s) + (blk << l) + t);
        if (s == 0 && (RED & kFwdTernaryInput)) {
          const double t = x[(k + half) * G + u] * W;  // exact: |Y| <= 1
          x[(k + half) * G + u] = x[k * G + u] - t;
          x[k * G + u] = x[k * G + u] + t;
        } else {
          ct_butterfly(x[k * G + u], x[(k + half) * G + u], W, q, qinv);
        }
      }
      if ((RED >> s) & 1u) {
#pragma unroll
        for (int k = 0; k < (1 << P); k++) x[k * G + u] = reduce(x[k * G + u], q, qinv);
      }
      stage_fence();
    }
  }
}

// Inverse (Gentleman-Sande) stages of one pass, in decreasing stage order; reduce the sum
// outputs after stage s if bit s of RED.
template <int LOGN, int LOGR, int PASS, uint32_t RED>
CKKS_HD void inv_pass(double (&x)[1 << LOGR], int tid_in, const double *__restrict__ itw,
                      const PassTw<LOGN, LOGR, PASS> &regs, double q, double qinv) {
  const int tid = opaque(tid_in);
  using S = NttShape<LOGN, LOGR>;
  using PT = PassTw<LOGN, LOGR, PASS>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS), G = S::R >> P;
  constexpr int LTLO = LOGN - S0 - P;
#pragma unroll
  for (int u = 0; u < G; u++) {
    const unsigned g = (unsigned)tid + (unsigned)S::T * u;
    const unsigned blk = PASS == 0 ? 0u : g >> LTLO;
#pragma unroll
    for (int l = P - 1; l >= 0; l--) {
      const int s = S0 + l;
      const int half = 1 << (P - 1 - l);
#pragma unroll
      for (int k = 0; k < (1 << P); k++) {
        if (k & half) continue;
        const unsigned t = (unsigned)(k >> (P - l));
        double W;
        if constexpr (PT::kPrefetch)
          W = regs.w[u * PT::PER + (1 << l) - 1 + t];
        else
          W = ld_table(itw, (1u << s) + (blk << l) + t);
        double &X = x[k * G + u];
        double &Y = x[(k + half) * G + u];
        gs_butterfly(X, Y, W, q, qinv);
        if ((RED >> s) & 1u) X = reduce(X, q, qinv);
      }
      stage_fence();
    }
  }
}

// The same stages applied to two arrays with the same factors (two independent
// butterfly chains the scheduler can interleave).
template <int LOGN, int LOGR, int PASS, uint32_t RED>
CKKS_HD void inv_pass2(double (&x)[1 << LOGR], double (&x2)[1 << LOGR], int tid_in, const double *__restrict__ itw,
                      const PassTw<LOGN, LOGR, PASS> &regs, double q, double qinv) {
  const int tid = opaque(tid_in);
  using S = NttShape<LOGN, LOGR>;
  using PT = PassTw<LOGN, LOGR, PASS>;
  constexpr int S0 = S::start(PASS), P = S::len(PASS), G = S::R >> P;
  constexpr int LTLO = LOGN - S0 - P;
#pragma unroll
  for (int u = 0; u < G; u++) {
    const unsigned g = (unsigned)tid + (unsigned)S::T * u;
    const unsigned blk = PASS == 0 ? 0u : g >> LTLO;
#pragma unroll
    for (int l = P - 1; l >= 0; l--) {
      const int s = S0 + l;
      const int half = 1 << (P - 1 - l);
#pragma unroll
      for (int k = 0; k < (1 << P); k++) {
        if (k & half) continue;
        const unsigned t = (unsigned)(k >> (P - l));
        double W;
        if constexpr (PT::kPrefetch)
          W = regs.w[u * PT::PER + (1 << l) - 1 + t];
        else
          W = ld_table(itw, (1u << s) + (blk << l) + t);
        gs_butterfly(x[k * G + u], x[(k + half) * G + u], W, q, qinv);
        gs_butterfly(x2[k * G + u], x2[(k + half) * G + u], W, q, qinv);
        if ((RED >> s) & 1u) {
          x[k * G + u] = reduce(x[k * G + u], q, qinv);
          x2[k * G + u] = reduce(x2[k * G + u], q, qinv);
        }
      }
      stage_fence();
    }
  }
}

// The element index is the bitwise OR of a thread part, elem_index(tid, 0), and a
// register part, elem_index(0, r), on disjoint bits (the thread index and the register
// index fill different bit fields of it), so each thread computes one base slot per
// exchange and each register adds a compile-time offset, after an XOR of the base with
// the register part's low swizzled bits where those are not zero (lds_slot).
// (The slot arithmetic is done on byte offsets, so each distinct low part costs one XOR
// and the high part is an instruction's immediate offset.)
template <int LOGN, int LOGR, int PASS>
CKKS_HD void lds_store(double *lds, const double (&x)[1 << LOGR], int tid_in) {
  const int tid = opaque(tid_in);
  const unsigned tb8 = lds_pos<LOGR>(elem_index<LOGN, LOGR, PASS>((unsigned)tid, 0)) << 3;
  char *bytes = reinterpret_cast<char *>(lds);
#pragma unroll
  for (int r = 0; r < (1 << LOGR); r++) {
    const unsigned pr = lds_pos<LOGR>(elem_index<LOGN, LOGR, PASS>(0, r));
    *reinterpret_cast<double *>(bytes + ((tb8 ^ ((pr & 15u) << 3)) + ((pr & ~15u) << 3))) = x[r];
  }
}

template <int LOGN, int LOGR, int PASS>
CKKS_HD void lds_load(const double *lds, double (&x)[1 << LOGR], int tid_in) {
  const int tid = opaque(tid_in);
  const unsigned tb8 = lds_pos<LOGR>(elem_index<LOGN, LOGR, PASS>((unsigned)tid, 0)) << 3;
  const char *bytes = reinterpret_cast<const char *>(lds);
#pragma unroll
  for (int r = 0; r < (1 << LOGR); r++) {
    const unsigned pr = lds_pos<LOGR>(elem_index<LOGN, LOGR, PASS>(0, r));
    x[r] = *reinterpret_cast<const double *>(bytes + ((tb8 ^ ((pr & 15u) << 3)) + ((pr & ~15u) << 3)));
  }
}

// Synchronisation of the LDS exchange between two passes.  Where each wave writes exactly
// the LDS slots it reads back (same_wave_sets), only the wave's own accesses must stay in
// order, and LDS operations of one wave are performed in issue order: a wave-scope fence
// keeps the compiler from reordering them and no workgroup barrier is needed.  The first
// exchange of a transform keeps its leading barrier, since the slots' previous users are
// not known there.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE_LOCAL, bool FIRST_EXCHANGE>
__device__ __forceinline__ void exchange_lead() {
  if constexpr (WAVE_LOCAL && !FIRST_EXCHANGE)
    wave_sync();
  else
    __syncthreads();
}

template <bool WAVE_LOCAL>
__device__ __forceinline__ void exchange_mid() {
  if constexpr (WAVE_LOCAL)
    wave_sync();
  else
    __syncthreads();
}

// Passes 1..NPASS-1 of the forward transform (pass 0 is run by the caller on the
// first-pass layout); ends with x in the last-pass layout.  Contains barriers: every
// thread of the workgroup must call it.
template <int LOGN, int LOGR, uint32_t RED, int PASS = 1>
__device__ __forceinline__ void fwd_rest(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ tw,
                                         double q, double qinv) {
  if constexpr (PASS < NttShape<LOGN, LOGR>::NPASS) {
    constexpr bool kLocal = NttShape<LOGN, LOGR>::same_wave_sets(PASS - 1, PASS);
    PassTw<LOGN, LOGR, PASS> w;
    tw_prefetch<LOGN, LOGR, PASS>(w, tid, tw);
    exchange_lead<kLocal, PASS == 1>();
    lds_store<LOGN, LOGR, PASS - 1>(lds, x, tid);
    exchange_mid<kLocal>();
    lds_load<LOGN, LOGR, PASS>(lds, x, tid);
    fwd_pass<LOGN, LOGR, PASS, RED>(x, tid, tw, w, q, qinv);
    fwd_rest<LOGN, LOGR, RED, PASS + 1>(x, lds, tid, tw, q, qinv);
  }
}

// Whole forward transform from the first-pass layout to the last-pass layout.
template <int LOGN, int LOGR, uint32_t RED>
__device__ __forceinline__ void ntt_forward(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ tw,
                                            double q, double qinv) {
  PassTw<LOGN, LOGR, 0> w;
  tw_prefetch<LOGN, LOGR, 0>(w, tid, tw);
  fwd_pass<LOGN, LOGR, 0, RED>(x, tid, tw, w, q, qinv);
  fwd_rest<LOGN, LOGR, RED, 1>(x, lds, tid, tw, q, qinv);
}

// Passes PASS..0 of the inverse transform; before_last() runs just before the exchange
// that precedes the final pass (a place for the caller's own loads, whose latency then
// hides behind that exchange).
template <int LOGN, int LOGR, uint32_t RED, int PASS, class F>
__device__ __forceinline__ void inv_rest(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ itw,
                                         double q, double qinv, F &&before_last) {
  if constexpr (PASS >= 0) {
    using NS = NttShape<LOGN, LOGR>;
    constexpr bool kLocal = NS::same_wave_sets(PASS + 1, PASS);
    PassTw<LOGN, LOGR, PASS> w;
    tw_prefetch<LOGN, LOGR, PASS>(w, tid, itw);
    if constexpr (PASS == 0) before_last();
    exchange_lead<kLocal, PASS == NS::NPASS - 2>();
    lds_store<LOGN, LOGR, PASS + 1>(lds, x, tid);
    exchange_mid<kLocal>();
    lds_load<LOGN, LOGR, PASS>(lds, x, tid);
    inv_pass<LOGN, LOGR, PASS, RED>(x, tid, itw, w, q, qinv);
    inv_rest<LOGN, LOGR, RED, PASS - 1>(x, lds, tid, itw, q, qinv, before_last);
  }
}

// Whole inverse transform (without the factor 1/N) from the last-pass layout to the
// first-pass layout.  before_last() runs before the final exchange (see inv_rest).
template <int LOGN, int LOGR, uint32_t RED, class F>
__device__ __forceinline__ void ntt_inverse(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ itw,
                                            double q, double qinv, F &&before_last) {
  constexpr int LAST = NttShape<LOGN, LOGR>::NPASS - 1;
  static_assert(LAST >= 1, "the transform has at least two passes");
  PassTw<LOGN, LOGR, LAST> w;
  tw_prefetch<LOGN, LOGR, LAST>(w, tid, itw);
  inv_pass<LOGN, LOGR, LAST, RED>(x, tid, itw, w, q, qinv);
  inv_rest<LOGN, LOGR, RED, LAST - 1>(x, lds, tid, itw, q, qinv, before_last);
}

template <int LOGN, int LOGR, uint32_t RED>
__device__ __forceinline__ void ntt_inverse(double (&x)[1 << LOGR], double *lds, int tid, const double *__restrict__ itw,
                                            double q, double qinv) {
  ntt_inverse<LOGN, LOGR, RED>(x, lds, tid, itw, q, qinv, [] {});
}

// Two inverse transforms with the same prime at once: one set of exchanges (x through
// lds, x2 through lds2, each N slots), shared twiddle loads and barriers.
template <int LOGN, int LOGR, uint32_t RED, int PASS, class F>
__device__ __forceinline__ void inv_rest2(double (&x)[1 << LOGR], double (&x2)[1 << LOGR], double *lds, double *lds2,
                                          int tid, const double *__restrict__ itw, double q, double qinv,
                                          F &&before_last) {
  if constexpr (PASS >= 0) {
    using NS = NttShape<LOGN, LOGR>;
    constexpr bool kLocal = NS::same_wave_sets(PASS + 1, PASS);
    PassTw<LOGN, LOGR, PASS> w;
    tw_prefetch<LOGN, LOGR, PASS>(w, tid, itw);
    if constexpr (PASS == 0) before_last();
    exchange_lead<kLocal, PASS == NS::NPASS - 2>();
    lds_store<LOGN, LOGR, PASS + 1>(lds, x, tid);
    lds_store<LOGN, LOGR, PASS + 1>(lds2, x2, tid);
    exchange_mid<kLocal>();
    lds_load<LOGN, LOGR, PASS>(lds, x, tid);
    lds_load<LOGN, LOGR, PASS>(lds2, x2, tid);
    inv_pass2<LOGN, LOGR, PASS, RED>(x, x2, tid, itw, w, q, qinv);
    inv_rest2<LOGN, LOGR, RED, PASS - 1>(x, x2, lds, lds2, tid, itw, q, qinv, before_last);
  }
}

template <int LOGN, int LOGR, uint32_t RED, class F>
__device__ __forceinline__ void ntt_inverse2(double (&x)[1 << LOGR], double (&x2)[1 << LOGR], double *lds,
                                             double *lds2, int tid, const double *__restrict__ itw, double q,
                                             double qinv, F &&before_last) {
  constexpr int LAST = NttShape<LOGN, LOGR>::NPASS - 1;
  PassTw<LOGN, LOGR, LAST> w;
  tw_prefetch<LOGN, LOGR, LAST>(w, tid, itw);
  inv_pass2<LOGN, LOGR, LAST, RED>(x, x2, tid, itw, w, q, qinv);
  inv_rest2<LOGN, LOGR, RED, LAST - 1>(x, x2, lds, lds2, tid, itw, q, qinv, before_last);
}

}  // namespace ckks
