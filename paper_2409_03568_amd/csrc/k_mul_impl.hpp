// Ciphertext product with relinearization: key-switching keys of s^2, their NTT-domain
// copies, and the fused tensor / key-switch / ModDown kernel.  Included by the NTT
// implementation header, whose shapes, samplers and transforms it uses.
#pragma once

namespace ckks {

// ---------------------------------------------------------------------------
// key-switching keys of s^2 for ciphertext multiplication (Sec. 2.2.3), one workgroup
// per (digit i, prime j); prime j = L is the special prime qP.  Key i in prime j:
//   b = -a * s + e_i + [j == i] (qP mod q_i) s^2,  a uniform mod p_j
// with e_i the Gaussian stream (seed, 0, 48 + i) and a the uniform stream
// (seed, 0, 64 + 32 i + j), both as in the key generation above.
// ---------------------------------------------------------------------------
constexpr uint32_t kTagRkE0 = 48, kTagRkA0 = 64;

template <int LOGN, int LOGR, int RC>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    k_relin_keygen(uint64_t k0, uint64_t k1, const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  uint64_t *cdt = reinterpret_cast<uint64_t *>(lds + S::SLOTS);
  uint16_t *lds16 = reinterpret_cast<uint16_t *>(lds);
  const int tid = threadIdx.x;
  for (int i = tid; i < kCdtSlots; i += T) cdt[i] = dt.cdt[i];
  __syncthreads();
  const int L = lc.L, B = lc.B, i = blockIdx.x, j = blockIdx.y;
  const double q = lc.q[j], qinv = lc.qinv[j];
  const uint64_t qi = lc.qi[j];
  const double *tw = dt.tw_fwd + (size_t)j * N, *itw = dt.tw_inv + (size_t)j * N;
  uint32_t smp[R];
  const uint32_t etag = kTagRkE0 + (uint32_t)i;
  draw_samples<LOGN, LOGR>(smp, lds16, cdt, B, tid, k0, k1, 0, etag, etag, etag);
  const uint64_t limit = 0ULL - ((~0ULL % qi + 1) % qi);
  uint64_t *kb = dt.evk + (((size_t)i * (L + 1) + j) * 2) * N, *ka = kb + N;
  double a[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const uint32_t c = (uint32_t)(tid + T * r);
    uint64_t val = 0;
    bool done = false;
    for (uint64_t att = 0; !done; att++) {
      const Philox4 w = philox4x64_10(0, kTagRkA0 + 32u * (uint32_t)i + (uint32_t)j, att * N + c, 0, k0, k1);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (!done && w.w[k] < limit) {
          val = w.w[k] % qi;
          done = true;
        }
      }
    }
    ka[c] = val;
    a[r] = (double)val;
  }
  // s_hat and s_hat * N^-1 in this prime
  double sh[R], shn[R];
#pragma unroll
  for (int r = 0; r < R; r++) sh[r] = (double)dt.s[tid + T * r];
  ntt_forward<LOGN, LOGR, Red::fwd_small>(sh, lds, tid, tw, q, qinv);
  const double ninv = lc.ninv[j];
#pragma unroll
  for (int r = 0; r < R; r++) {
    sh[r] = reduce(sh[r], q, qinv);
    shn[r] = reduce(mulmod(sh[r], ninv, q, qinv), q, qinv);
  }
  ntt_forward<LOGN, LOGR, Red::fwd_big>(a, lds, tid, tw, q, qinv);
  const bool own = (j == i);
  const double pm = own ? lc.pmod[i] : 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    double v = -mulmod(a[r], shn[r], q, qinv);
    if (own) v += mulmod(mulmod(sh[r], shn[r], q, qinv), pm, q, qinv);
    a[r] = reduce(v, q, qinv);
  }
  ntt_inverse<LOGN, LOGR, Red::inv>(a, lds, tid, itw, q, qinv);
#pragma unroll
  for (int r = 0; r < R; r++) {
    const double e = (double)smp_g(smp[r], kSmpShiftG2, B);
    kb[tid + T * r] = (uint64_t)canon(a[r] + e, q, qinv);
  }
}

// NTT-domain copies of the key-switching keys times N^-1 (grid: digits x primes x 2).
template <int LOGN, int LOGR, int RC>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    k_relin_prepare(const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, i = blockIdx.x, j = blockIdx.y, k = blockIdx.z, L = lc.L;
  const double q = lc.q[j], qinv = lc.qinv[j];
  const size_t off = ((((size_t)i * (L + 1) + j) * 2) + k) * N;
  double x[R];
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = u64_to_f64(dt.evk[off + tid + T * r]);
  ntt_forward<LOGN, LOGR, Red::fwd_big>(x, lds, tid, dt.tw_fwd + (size_t)j * N, q, qinv);
#pragma unroll
  for (int r = 0; r < R; r++)
    dt.evk_hat[off + elem_index<LOGN, LOGR, S::LAST>(tid, r)] = reduce(mulmod(x[r], lc.ninv[j], q, qinv), q, qinv);
}

// ---------------------------------------------------------------------------
// relinearized product of ciphertext pairs (Sec. 2.2.3), one workgroup per pair:
//  1. per limb j, through the NTT: d0 = a0 b0, d1 = a0 b1 + a1 b0 and d2 = a1 b1 (at most
//     three transforms held at once); d0 and d1 stay in the NTT domain (parked in the
//     output limb), d2 goes back to coefficients (the key-switching digit) and its NTT
//     is kept for prime j;
//  2. key switching, prime by prime with the special prime first: every digit i (d2
//     limb i as an integer below q_i) is lifted to the prime, transformed (or taken
//     from step 1 in its own prime) and multiplied by key i;
//  3. ModDown folded into the last transform: out_j = INTT(d_hat + acc_hat * qP^-1)
//     - [acc]_qP * qP^-1, [.]_qP the centered coefficient of the special-prime part.
// Outputs may alias inputs exactly: each residue row (poly, limb) of out is first written
// after the same rows of a and b have been read, and after step 1 only out and scratch
// are read.  All arithmetic is exact FP64 on signed representatives kept inside the
// transform bounds.
// ---------------------------------------------------------------------------
template <int LOGN, int LOGR, int RC>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    k_mul(const uint64_t *A, const uint64_t *Bc, uint64_t *out, uint64_t n, int level,
          uint64_t *__restrict__ scratch, const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  const int L = lc.L;
  const uint64_t S_ct = (uint64_t)2 * level * N;
  // scratch of this workgroup, every element written and read by one thread:
  // [level][N] d2 digits, [level][N] NTT(d2) in its own prime, [2][N] centered
  // special-prime accumulators
  uint64_t *d2s = scratch + (uint64_t)blockIdx.x * (uint64_t)(2 * level + 2) * N;
  uint64_t *own = d2s + (size_t)level * N;
  uint64_t *accw = d2s + (size_t)2 * level * N;  // bit patterns of doubles
  for (uint64_t it = blockIdx.x; it < n; it += gridDim.x) {
    const uint64_t *a = A + it * S_ct, *b = Bc + it * S_ct;
    uint64_t *o = out + it * S_ct;
    // 1. tensor product, limb by limb
    for (int j = 0; j < level; j++) {
      const int tid = opaque(threadIdx.x);
      const double q = lc.q[j], qinv = lc.qinv[j], ninv = lc.ninv[j];
      const double *tw = dt.tw_fwd + (size_t)j * N, *itw = dt.tw_inv + (size_t)j * N;
      // three transforms live at a time: a1 b0 waits in this limb's own-prime scratch row
      // until b1 arrives (not in out, which may be b)
      uint64_t *o0 = o + (size_t)j * N, *o1 = o + ((size_t)level + j) * N;
      const uint64_t *a0 = a + (size_t)j * N, *b0 = b + (size_t)j * N;
      const uint64_t *a1 = a + ((size_t)level + j) * N, *b1 = b + ((size_t)level + j) * N;
      uint64_t *ownj = own + (size_t)j * N, *d2j = d2s + (size_t)j * N;
      double x[R], y[R], z[R];
#pragma unroll
      for (int r = 0; r < R; r++) x[r] = u64_to_f64(ld_word(a0, tid + T * r));
      ntt_forward<LOGN, LOGR, Red::fwd_big>(x, lds, tid, tw, q, qinv);
#pragma unroll
      for (int r = 0; r < R; r++) {
        x[r] = reduce(mulmod(x[r], ninv, q, qinv), q, qinv);  // a0 (the a side carries N^-1)
        y[r] = u64_to_f64(ld_word(b0, tid + T * r));
      }
      ntt_forward<LOGN, LOGR, Red::fwd_big>(y, lds, tid, tw, q, qinv);
#pragma unroll
      for (int r = 0; r < R; r++) {
        y[r] = reduce(y[r], q, qinv);  // b0
        st_word(o0, tid + T * r, __builtin_bit_cast(uint64_t, mulmod(x[r], y[r], q, qinv)));  // d0
        z[r] = u64_to_f64(ld_word(a1, tid + T * r));
      }
      ntt_forward<LOGN, LOGR, Red::fwd_big>(z, lds, tid, tw, q, qinv);
#pragma unroll
      for (int r = 0; r < R; r++) {
        z[r] = reduce(z[r], q, qinv);  // a1 without N^-1
        const double a1n = reduce(mulmod(z[r], ninv, q, qinv), q, qinv);
        st_word(ownj, tid + T * r, __builtin_bit_cast(uint64_t, mulmod(a1n, y[r], q, qinv)));  // a1 b0
        y[r] = u64_to_f64(ld_word(b1, tid + T * r));
      }
      ntt_forward<LOGN, LOGR, Red::fwd_big>(y, lds, tid, tw, q, qinv);
#pragma unroll
      for (int r = 0; r < R; r++) {
        const unsigned c = tid + T * r;
        const double b1h = reduce(y[r], q, qinv);
        st_word(o1, c,
                __builtin_bit_cast(uint64_t, reduce(mulmod(x[r], b1h, q, qinv) +
                                                        __builtin_bit_cast(double, ld_word(ownj, c)),
                                                    q, qinv)));  // d1
        // NTT(d2) for the key product in prime j (keys carry N^-1), and d2 itself
        st_word(ownj, c, __builtin_bit_cast(uint64_t, mulmod(z[r], b1h, q, qinv)));
        y[r] = mulmod(reduce(mulmod(z[r], ninv, q, qinv), q, qinv), b1h, q, qinv);
      }
      ntt_inverse<LOGN, LOGR, Red::inv>(y, lds, tid, itw, q, qinv);
#pragma unroll
      for (int r = 0; r < R; r++) st_word(d2j, tid + T * r, f64_to_u64(canon(y[r], q, qinv)));
    }
    // 2 + 3. key switching, the special prime (index L) first
    for (int jj = 0; jj <= level; jj++) {
      const int tid = opaque(threadIdx.x);
      const int j = jj == 0 ? L : jj - 1;
      const double q = lc.q[j], qinv = lc.qinv[j];
      const double *tw = dt.tw_fwd + (size_t)j * N, *itw = dt.tw_inv + (size_t)j * N;
      double c0[R], c1[R];
#pragma unroll
      for (int r = 0; r < R; r++) c0[r] = c1[r] = 0.0;
      for (int i = 0; i < level; i++) {
        double x[R];
        if (i == j) {
          const uint64_t *owni = own + (size_t)i * N;
#pragma unroll
          for (int r = 0; r < R; r++) x[r] = __builtin_bit_cast(double, ld_word(owni, tid + T * r));
        } else {
          const uint64_t *d2i = d2s + (size_t)i * N;
#pragma unroll
          for (int r = 0; r < R; r++) x[r] = reduce(u64_to_f64(ld_word(d2i, tid + T * r)), q, qinv);
          ntt_forward<LOGN, LOGR, Red::fwd_big>(x, lds, tid, tw, q, qinv);
        }
        const double *kb = dt.evk_hat + (((size_t)i * (L + 1) + j) * 2) * N, *ka = kb + N;
#pragma unroll
        for (int r = 0; r < R; r++) {
          const unsigned e = elem_index<LOGN, LOGR, S::LAST>(tid, r);
          c0[r] = reduce(c0[r] + mulmod(x[r], ld_table(kb, e), q, qinv), q, qinv);
          c1[r] = reduce(c1[r] + mulmod(x[r], ld_table(ka, e), q, qinv), q, qinv);
        }
      }
      if (jj == 0) {
        ntt_inverse<LOGN, LOGR, Red::inv>(c0, lds, tid, itw, q, qinv);
        ntt_inverse<LOGN, LOGR, Red::inv>(c1, lds, tid, itw, q, qinv);
#pragma unroll
        for (int r = 0; r < R; r++) {
          const unsigned c = tid + T * r;
          st_word(accw, c, __builtin_bit_cast(uint64_t, center(c0[r], q, qinv)));
          st_word(accw, N + c, __builtin_bit_cast(uint64_t, center(c1[r], q, qinv)));
        }
        continue;
      }
      const double pinv = lc.pinv[j];
      uint64_t *o0 = o + (size_t)j * N, *o1 = o + ((size_t)level + j) * N;
#pragma unroll
      for (int r = 0; r < R; r++) {
        const unsigned c = tid + T * r;
        c0[r] = reduce(mulmod(c0[r], pinv, q, qinv) + __builtin_bit_cast(double, ld_word(o0, c)), q, qinv);
        c1[r] = reduce(mulmod(c1[r], pinv, q, qinv) + __builtin_bit_cast(double, ld_word(o1, c)), q, qinv);
      }
      ntt_inverse<LOGN, LOGR, Red::inv>(c0, lds, tid, itw, q, qinv);
      ntt_inverse<LOGN, LOGR, Red::inv>(c1, lds, tid, itw, q, qinv);
#pragma unroll
      for (int r = 0; r < R; r++) {
        const unsigned c = tid + T * r;
        const double p0 = __builtin_bit_cast(double, ld_word(accw, c));
        const double p1 = __builtin_bit_cast(double, ld_word(accw, N + c));
        st_word(o0, c, f64_to_u64(canon(c0[r] - mulmod(p0, pinv, q, qinv), q, qinv)));
        st_word(o1, c, f64_to_u64(canon(c1[r] - mulmod(p1, pinv, q, qinv), q, qinv)));
      }
    }
  }
}

}  // namespace ckks
