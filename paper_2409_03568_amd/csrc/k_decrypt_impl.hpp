// Decryption kernels (Sec. 2.2.2): c0 + c1 s through the NTT, the decode of slot 0, and
// the two-limb CRT lift.  Included by the NTT implementation header, whose shapes,
// transforms and tables they use.
#pragma once

namespace ckks {

// ---------------------------------------------------------------------------
// decryption and decoding of slot 0:
//   d_i = c0_i + INTT(NTT(c1_i) * s_hat_i) in limb i;  out = sum_j x_j cos(pi j/N) / scale
// LIMBS = 1: x_j is the centered residue of limb 0, exact while |x_j| < q_0/2.
// LIMBS = 2: x_j is the centered CRT lift of limbs 0 and 1, x = x0 + q_0 k with
//   x0 = [d_0]_{q_0} and k = [(d_1 - x0) q_0^-1]_{q_1}, exact while |x_j| < q_0 q_1 / 2
//   (the sum is formed in FP64, so a lift beyond 2^53 is rounded to 53 bits).
// ---------------------------------------------------------------------------
// Register budget: enough waves per SIMD for as many workgroups as the LDS admits on a
// CU (at most two), so one workgroup's waves compute while another's wait at a barrier.
template <int LOGN, int LOGR>
constexpr int decrypt_waves_per_eu() {
  constexpr int wgs = (int)((160 * 1024) / Shape<LOGN, LOGR>::lds_bytes) >= 2 ? 2 : 1;
  constexpr int w = wgs * (1 << (LOGN - LOGR)) / 256;
  return w < 1 ? 1 : w;
}
// The two-limb form holds limb 0's values across limb 1's transform: half the waves, so
// that they stay in registers (forcing the one-limb occupancy spills them to scratch,
// about 9 GiB of memory traffic per 65,536 ciphertexts, for 2% less time).
template <int LOGN, int LOGR, int LIMBS>
constexpr int decrypt_waves_hint() {
  constexpr int w = decrypt_waves_per_eu<LOGN, LOGR>() / LIMBS;
  return w < 1 ? 1 : w;
}

// d = c0 + c1 * s in limb l of ciphertext (c0, c1), returned in x in the first-pass
// layout as signed values below 2^52 in magnitude (congruent to d mod q_l).
template <int LOGN, int LOGR, int RC>
__device__ __forceinline__ void decrypt_limb(double (&x)[1 << LOGR], const uint64_t *c0, const uint64_t *c1, int l,
                                             double *lds, int tid, const LimbConsts &lc, const DevTables &dt) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const double q = lc.q[l], qinv = lc.qinv[l];
  const uint64_t *c0l = c0 + (size_t)l * N, *c1l = c1 + (size_t)l * N;
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = u64_to_f64(__builtin_nontemporal_load(word_at(c1l, tid + T * r)));
  ntt_forward<LOGN, LOGR, Red::fwd_big>(x, lds, tid, dt.tw_fwd + (size_t)l * N, q, qinv);
  const double *sh = dt.s_hat + (size_t)l * N;
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = mulmod(x[r], ld_table(sh, elem_index<LOGN, LOGR, S::LAST>(tid, r)), q, qinv);
  // c0 is loaded from HBM before the final exchange of the transform
  uint64_t c0w[R];
  ntt_inverse<LOGN, LOGR, Red::inv>(x, lds, tid, dt.tw_inv + (size_t)l * N, q, qinv, [&] {
#pragma unroll
    for (int r = 0; r < R; r++) c0w[r] = __builtin_nontemporal_load(word_at(c0l, tid + T * r));
  });
#pragma unroll
  for (int r = 0; r < R; r++) x[r] += u64_to_f64(c0w[r]);
}

template <int LOGN, int LOGR, int RC, int LIMBS>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    __attribute__((amdgpu_waves_per_eu(decrypt_waves_hint<LOGN, LOGR, LIMBS>())))
    k_decrypt(const uint64_t *__restrict__ cts, uint64_t n, int level, double inv_scale, double *__restrict__ out,
              const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  double *red = lds + S::SLOTS + kCdtSlots;
  const int tid = threadIdx.x;
  const double q = lc.q[0], qinv = lc.qinv[0];
  for (uint64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int tid = opaque(threadIdx.x);
    const uint64_t *c0 = cts + i * (uint64_t)(2 * level) * N;
    const uint64_t *c1 = c0 + (size_t)level * N;
    double x[R];
    decrypt_limb<LOGN, LOGR, RC>(x, c0, c1, 0, lds, tid, lc, dt);
#pragma unroll
    for (int r = 0; r < R; r++) x[r] = center(x[r], q, qinv);
    if constexpr (LIMBS == 2) {
      const double q1 = lc.q[1], q1inv = lc.qinv[1], w = lc.q0inv_q1;
      double y[R];
      decrypt_limb<LOGN, LOGR, RC>(y, c0, c1, 1, lds, tid, lc, dt);
#pragma unroll
      for (int r = 0; r < R; r++) {
        // |y| < 2^52 and |x| <= q_0/2: the difference of the reduced values stays below 2^51
        const double k = center(mulmod(reduce(y[r], q1, q1inv) - x[r], w, q1, q1inv), q1, q1inv);
        x[r] = __builtin_fma(k, q, x[r]);
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < R; r++) acc = __builtin_fma(x[r], ld_table(dt.cosj, tid + T * r), acc);
    // workgroup sum in a fixed order: wave butterflies, then the waves in sequence
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < T / 64; w++) s += red[w];
      out[i] = s * inv_scale;
    }
  }
}

}  // namespace ckks
