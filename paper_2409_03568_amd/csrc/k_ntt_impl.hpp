// NTT-based kernels: key generation, key preparation, fused per-pixel encryption and
// decryption.  One workgroup handles one ciphertext at a time (all limbs), so the
// random polynomials v, e0, e1 are drawn once per ciphertext and reused by every limb.
//
// Template parameters: LOGN (ring degree), LOGR (values per thread, so N / 2^LOGR threads
// per workgroup) and RC (reduction class of the primes, see ntt.hpp).  Each ring degree is
// instantiated in its own translation unit (k_ntt_<LOGN>.hip).
#pragma once
#include <atomic>

#include "internal.hpp"
#include "ntt.hpp"
#include "philox.hpp"

namespace ckks {

template <int LOGN, int LOGR>
struct Shape : NttShape<LOGN, LOGR> {
  static constexpr int LAST = NttShape<LOGN, LOGR>::NPASS - 1;
  // dynamic LDS: the exchange space (N doubles with padding, see lds_pos), the Gaussian
  // table, and a reduction area
  static constexpr int SLOTS = LdsSlots<LOGN, LOGR>::value;
  static constexpr size_t lds_bytes = sizeof(double) * ((size_t)SLOTS + kCdtSlots + 64);
  // Encryption also keeps the packed samples of the current ciphertext (2 bytes per
  // coefficient) in LDS when that fits a CU's 160 KiB, instead of in registers for the
  // whole ciphertext.
  static constexpr size_t smp_bytes = sizeof(uint16_t) * ((size_t)1 << LOGN);
  // When a second exchange space fits as well (N <= 8192), encryption runs the two
  // inverse transforms of a limb as one paired transform; its second space follows the
  // reduction area, and the packed samples follow that when they fit too.
  static constexpr bool kDual = lds_bytes + sizeof(double) * (size_t)SLOTS <= 160 * 1024;
  static constexpr size_t enc_base_bytes = lds_bytes + (kDual ? sizeof(double) * (size_t)SLOTS : 0);
  static constexpr bool kSmpLds = enc_base_bytes + smp_bytes <= 160 * 1024;
  static constexpr size_t enc_lds_bytes = enc_base_bytes + (kSmpLds ? smp_bytes : 0);
};

// Draw the packed samples of one polynomial triple into LDS: word j of dst holds
// coefficient j as (t1 + 1) | (g2 + B) << 2 | (g3 + B) << 9, where t1 is the ternary
// value of stream tag1 and g2, g3 the Gaussian values of streams tag2, tag3 (all at
// Philox index t; 0 <= g + B <= 2B <= 126).  Each thread draws whole Philox blocks; ends
// with a barrier.
constexpr int kSmpShiftG2 = 2, kSmpShiftG3 = 9;

template <int LOGN, int LOGR>
__device__ __forceinline__ void draw_samples(uint16_t *dst, const uint64_t *cdt, int B, int tid, uint64_t k0,
                                             uint64_t k1, uint64_t t, uint32_t tag1, uint32_t tag2, uint32_t tag3) {
  using S = NttShape<LOGN, LOGR>;
  static_assert(S::R >= 4, "each thread draws whole Philox blocks");
#pragma unroll 1
  for (int kk = 0; kk < S::R / 4; kk++) {
    const uint32_t b = (uint32_t)(tid + S::T * kk);
    const Philox4 pv = philox4x64_10(t, tag1, b, 0, k0, k1);
    const Philox4 pa = philox4x64_10(t, tag2, b, 0, k0, k1);
    const Philox4 pb = philox4x64_10(t, tag3, b, 0, k0, k1);
    uint32_t w2[2];
#pragma unroll
    for (int w = 0; w < 4; w++) {
      const uint32_t tv = (uint32_t)(ternary_of(pv.w[w]) + 1);
      const uint32_t ga = (uint32_t)(gauss_of(pa.w[w], cdt, B) + B);
      const uint32_t gb = (uint32_t)(gauss_of(pb.w[w], cdt, B) + B);
      const uint32_t word = tv | (ga << kSmpShiftG2) | (gb << kSmpShiftG3);
      w2[w >> 1] = (w & 1) ? (w2[w >> 1] | (word << 16)) : word;
    }
    reinterpret_cast<uint2 *>(dst)[b] = make_uint2(w2[0], w2[1]);
  }
  __syncthreads();
}

// The same, read back in the first-pass layout: smp[r] holds coefficient tid + T*r.
template <int LOGN, int LOGR>
__device__ __forceinline__ void draw_samples(uint32_t (&smp)[1 << LOGR], uint16_t *lds16, const uint64_t *cdt,
                                             int B, int tid, uint64_t k0, uint64_t k1, uint64_t t, uint32_t tag1,
                                             uint32_t tag2, uint32_t tag3) {
  using S = NttShape<LOGN, LOGR>;
  draw_samples<LOGN, LOGR>(lds16, cdt, B, tid, k0, k1, t, tag1, tag2, tag3);
#pragma unroll
  for (int r = 0; r < S::R; r++) smp[r] = lds16[tid + S::T * r];
}

__device__ __forceinline__ int smp_t(uint32_t s) { return (int)(s & 3u) - 1; }
__device__ __forceinline__ int smp_g(uint32_t s, int shift, int B) { return (int)((s >> shift) & 0x7fu) - B; }

// ---------------------------------------------------------------------------
// fused plain encryption: per ciphertext, per limb
//   x = NTT(v); c0 = INTT(x * pk0^) + e0 + m; c1 = INTT(x * pk1^) + e1
// ---------------------------------------------------------------------------
// Where item i's pixel value and Philox index come from (compiled separately, so each
// variant keeps only the pointers it reads live):
//   kEncPixels:  items 0..n-1, value px[i], index first_index + i;
//   kEncList:    items list[0..*list_count), value px[item], index first_index + item;
//   kEncEntries: items 0..count-1 (count = *list_count if set, else n), value vals[i],
//                index ts[i].
// BRIGHT adds the image's brightness encoding to c0 (EncJob::seg_b).
enum EncMode : int { kEncPixels = 0, kEncList = 1, kEncEntries = 2 };

// One limb of the encryption of the current item, by the whole workgroup (the samples
// are drawn): x = NTT(v); c0 = INTT(x pk0^) + e0 + m (+ the brightness encoding fb);
// c1 = INTT(x pk1^) + e1, stored to out.  With KEEP the canonical values of c0 and c1 are
// also returned in k0 / k1 (first-pass layout: register r holds coefficient tid + T r).
template <int LOGN, int LOGR, int RC, bool BRIGHT, bool KEEP>
__device__ __forceinline__ void encrypt_limb(int l, double *lds, const uint16_t *smpl, const uint32_t (&smp)[1 << LOGR],
                                             int L, int B, double value, double fb, uint64_t *out,
                                             const LimbConsts &lc, const DevTables &dt, double (&k0)[1 << LOGR],
                                             double (&k1)[1 << LOGR]) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const double q = lc.q[l], qinv = lc.qinv[l];
  const int tid = opaque(threadIdx.x);
  auto sample = [&](int r) -> uint32_t {
    if constexpr (S::kSmpLds)
      return (uint32_t)smpl[tid + T * r];
    else
      return smp[r];
  };
  double x[R];
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = (double)smp_t(sample(r));
  ntt_forward<LOGN, LOGR, Red::fwd_small>(x, lds, tid, dt.tw_fwd + (size_t)l * N, q, qinv);
  // both pointwise products at once (one wait for the key loads; x is then dead and
  // the second product takes its registers through the first inverse transform)
  double y[R], y1[R];
  {
    const double *pk0 = dt.pk_hat + (size_t)l * N, *pk1 = dt.pk_hat + ((size_t)L + l) * N;
#pragma unroll
    for (int r = 0; r < R; r++) {
      const unsigned e = elem_index<LOGN, LOGR, S::LAST>(tid, r);
      y[r] = mulmod(x[r], ld_table(pk0, e), q, qinv);
      y1[r] = mulmod(x[r], ld_table(pk1, e), q, qinv);
    }
  }
  if constexpr (S::kDual) {
    // c0 and c1 of this limb through one paired inverse transform; the plaintext and
    // e0 are loaded before its final exchange
    double add[R];
    ntt_inverse2<LOGN, LOGR, Red::inv>(y, y1, lds, lds + S::SLOTS + kCdtSlots + 64, tid, dt.tw_inv + (size_t)l * N,
                                       q, qinv, [&] {
#pragma unroll
      for (int r = 0; r < R; r++) {
        const int j = tid + T * r;
        add[r] = (double)smp_g(sample(r), kSmpShiftG2, B) + __builtin_rint(value * ld_table(dt.enc_T, j));
        if (BRIGHT) add[r] += __builtin_rint(fb * ld_table(dt.cosj, j));
      }
    });
    uint64_t *dst0 = out + (size_t)l * N, *dst1 = out + ((size_t)L + l) * N;
#pragma unroll
    for (int r = 0; r < R; r++) {
      const unsigned c = tid + T * r;
      const double v0 = canon(y[r] + add[r], q, qinv);
      const double v1 = canon(y1[r] + (double)smp_g(sample(r), kSmpShiftG3, B), q, qinv);
      __builtin_nontemporal_store(f64_to_u64(v0), word_at(dst0, c));
      __builtin_nontemporal_store(f64_to_u64(v1), word_at(dst1, c));
      if constexpr (KEEP) {
        k0[r] = v0;
        k1[r] = v1;
      }
    }
    return;
  }
#pragma unroll 1
  for (int poly = 0; poly < 2; poly++) {
    if (poly == 1) {
#pragma unroll
      for (int r = 0; r < R; r++) y[r] = y1[r];
    }
    // the plaintext (poly 0) and the Gaussian term, loaded before the final exchange
    double add[R];
    ntt_inverse<LOGN, LOGR, Red::inv>(y, lds, tid, dt.tw_inv + (size_t)l * N, q, qinv, [&] {
#pragma unroll
      for (int r = 0; r < R; r++) {
        const int j = tid + T * r;
        add[r] = (double)smp_g(sample(r), poly == 0 ? kSmpShiftG2 : kSmpShiftG3, B);
        if (poly == 0) {
          add[r] += __builtin_rint(value * ld_table(dt.enc_T, j));
          if (BRIGHT) add[r] += __builtin_rint(fb * ld_table(dt.cosj, j));
        }
      }
    });
    uint64_t *dst = out + ((size_t)poly * L + l) * N;
#pragma unroll
    for (int r = 0; r < R; r++) {
      const double v = canon(y[r] + add[r], q, qinv);
      __builtin_nontemporal_store(f64_to_u64(v), word_at(dst, tid + T * r));
      if constexpr (KEEP) (poly == 0 ? k0 : k1)[r] = v;
    }
  }
}

template <int LOGN, int LOGR, int RC, int MODE, bool BRIGHT>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    k_encrypt(EncJob job, const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  uint64_t *cdt = reinterpret_cast<uint64_t *>(lds + S::SLOTS);
  uint16_t *lds16 = reinterpret_cast<uint16_t *>(lds);
  uint16_t *smpl = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(lds) + S::enc_base_bytes);
  const int tid = threadIdx.x;
  for (int i = tid; i < kCdtSlots; i += T) cdt[i] = dt.cdt[i];
  const int L = lc.L, B = lc.B;
  uint64_t count = job.n;
  if (MODE == kEncList || (MODE == kEncEntries && job.list_count)) count = *job.list_count;
  for (uint64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const uint64_t item = MODE == kEncList ? (uint64_t)job.list[it] : it;
    const uint64_t t = MODE == kEncEntries ? job.ts[item] : job.first_index + item;
    const double value = MODE == kEncEntries ? (double)job.vals[item] : (double)job.px[item];
    const double fb =
        BRIGHT ? job.seg_b[segment_of(job.seg_end, job.n_seg, job.seg_base + item)] * job.bright_scale : 0.0;
    uint64_t *out = job.out + item * (uint64_t)(2 * L) * N;
    __syncthreads();
    uint32_t smp[R];  // used when the samples stay in registers
    if constexpr (S::kSmpLds)
      draw_samples<LOGN, LOGR>(smpl, cdt, B, opaque(tid), job.seed0, job.seed1, t, kTagV, kTagE0, kTagE1);
    else
      draw_samples<LOGN, LOGR>(smp, lds16, cdt, B, opaque(tid), job.seed0, job.seed1, t, kTagV, kTagE0, kTagE1);
    double unused0[R], unused1[R];
    for (int l = 0; l < L; l++)
      encrypt_limb<LOGN, LOGR, RC, BRIGHT, false>(l, lds, smpl, smp, L, B, value, fb, out, lc, dt, unused0, unused1);
  }
}

// ---------------------------------------------------------------------------
// key generation, one workgroup per limb l: pk0_l = -a_l * s + e, pk1_l = a_l
// ---------------------------------------------------------------------------
template <int LOGN, int LOGR, int RC>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    k_keygen(uint64_t k0, uint64_t k1, const LimbConsts *__restrict__ lcp, DevTables dt) {
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
  const int L = lc.L, B = lc.B, l = blockIdx.x;
  const double q = lc.q[l], qinv = lc.qinv[l];
  const uint64_t qi = lc.qi[l];
  uint32_t smp[R];
  // s from tag 16 (ternary), e from tag 17 (Gaussian); the third stream is unused
  draw_samples<LOGN, LOGR>(smp, lds16, cdt, B, tid, k0, k1, 0, kTagSk, kTagEk, kTagEk);
  // a_l: uniform residues by rejection, coefficient j tries block j, then N + j, ...
  // accept w < q * floor(2^64 / q) = 2^64 - (2^64 mod q)
  const uint64_t limit = 0ULL - ((~0ULL % qi + 1) % qi);
  double a[R];
  uint64_t *pk1 = dt.pk + ((size_t)L + l) * N;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const uint32_t j = (uint32_t)(tid + T * r);
    uint64_t val = 0;
    bool done = false;
    for (uint64_t att = 0; !done; att++) {
      const Philox4 w = philox4x64_10(0, kTagA0 + (uint32_t)l, att * N + j, 0, k0, k1);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (!done && w.w[k] < limit) {
          val = w.w[k] % qi;
          done = true;
        }
      }
    }
    pk1[j] = val;
    a[r] = (double)val;
  }
  if (l == 0) {
#pragma unroll
    for (int r = 0; r < R; r++) dt.s[tid + T * r] = smp_t(smp[r]);
  }
  // s_hat * N^-1 for this limb
  double x[R];
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = (double)smp_t(smp[r]);
  ntt_forward<LOGN, LOGR, Red::fwd_small>(x, lds, tid, dt.tw_fwd + (size_t)l * N, q, qinv);
  const double ninv = lc.ninv[l];
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = reduce(mulmod(x[r], ninv, q, qinv), q, qinv);
  ntt_forward<LOGN, LOGR, Red::fwd_big>(a, lds, tid, dt.tw_fwd + (size_t)l * N, q, qinv);
#pragma unroll
  for (int r = 0; r < R; r++) a[r] = mulmod(a[r], x[r], q, qinv);
  ntt_inverse<LOGN, LOGR, Red::inv>(a, lds, tid, dt.tw_inv + (size_t)l * N, q, qinv);
  uint64_t *pk0 = dt.pk + (size_t)l * N;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const double e = (double)smp_g(smp[r], kSmpShiftG2, B);
    pk0[tid + T * r] = (uint64_t)canon(e - a[r], q, qinv);
  }
}

// ---------------------------------------------------------------------------
// NTT-domain key copies used by encryption and decryption:
//   blockIdx.y = 0: s_hat_l * N^-1;  1: pk0_hat_l * N^-1;  2: pk1_hat_l * N^-1
// ---------------------------------------------------------------------------
template <int LOGN, int LOGR, int RC>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    k_keys_prepare(const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, l = blockIdx.x, which = blockIdx.y, L = lc.L;
  const double q = lc.q[l], qinv = lc.qinv[l];
  double x[R];
  if (which == 0) {
#pragma unroll
    for (int r = 0; r < R; r++) x[r] = (double)dt.s[tid + T * r];
    ntt_forward<LOGN, LOGR, Red::fwd_small>(x, lds, tid, dt.tw_fwd + (size_t)l * N, q, qinv);
  } else {
    const uint64_t *src = dt.pk + ((size_t)(which - 1) * L + l) * N;
#pragma unroll
    for (int r = 0; r < R; r++) x[r] = (double)src[tid + T * r];
    ntt_forward<LOGN, LOGR, Red::fwd_big>(x, lds, tid, dt.tw_fwd + (size_t)l * N, q, qinv);
  }
  double *dst = which == 0 ? dt.s_hat + (size_t)l * N : dt.pk_hat + ((size_t)(which - 1) * L + l) * N;
#pragma unroll
  for (int r = 0; r < R; r++)
    dst[elem_index<LOGN, LOGR, S::LAST>(tid, r)] = reduce(mulmod(x[r], lc.ninv[l], q, qinv), q, qinv);
}

// ---------------------------------------------------------------------------
// launch helpers for one ring degree
// ---------------------------------------------------------------------------
template <int LOGN, int LOGR, auto KERNEL, size_t BYTES = Shape<LOGN, LOGR>::lds_bytes>
static hipError_t set_lds() {
  // once per kernel and device (also keeps the call out of graph captures after the first launch)
  static std::atomic<uint64_t> done{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 63;
  const uint64_t bit = 1ull << dev;
  if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(KERNEL),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)BYTES);
  if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

}  // namespace ckks

#include "k_decrypt_impl.hpp"
#include "k_mul_impl.hpp"
#include "k_fused_impl.hpp"

namespace ckks {

template <int LOGN, int LOGR, int RC>
struct Launch {
  using S = Shape<LOGN, LOGR>;
  template <int MODE, bool BRIGHT>
  static hipError_t encrypt_as(const ckks_ctx *c, const EncJob &job, uint64_t grid, hipStream_t st) {
    hipError_t e = set_lds<LOGN, LOGR, k_encrypt<LOGN, LOGR, RC, MODE, BRIGHT>, S::enc_lds_bytes>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_encrypt<LOGN, LOGR, RC, MODE, BRIGHT>), dim3((uint32_t)grid), dim3(S::T), S::enc_lds_bytes,
                       st, job, c->d_lc, c->dev);
    return hipGetLastError();
  }
  static hipError_t encrypt(const ckks_ctx *c, const EncJob &job, uint64_t grid, hipStream_t st) {
    const bool bright = job.seg_b != nullptr;
    if (job.vals || job.ts) {
      if (!job.vals || !job.ts || bright) return hipErrorInvalidValue;
      return encrypt_as<kEncEntries, false>(c, job, grid, st);
    }
    if (job.list) {
      if (!job.list_count) return hipErrorInvalidValue;
      return bright ? encrypt_as<kEncList, true>(c, job, grid, st) : encrypt_as<kEncList, false>(c, job, grid, st);
    }
    if (job.list_count) return hipErrorInvalidValue;
    return bright ? encrypt_as<kEncPixels, true>(c, job, grid, st) : encrypt_as<kEncPixels, false>(c, job, grid, st);
  }
  template <bool BRIGHT, bool DECRYPT, bool MISSES>
  static hipError_t fused_as(const ckks_ctx *c, const FusedJob &job, hipStream_t st) {
    constexpr auto kernel = k_cached_fused<LOGN, LOGR, RC, BRIGHT, DECRYPT, MISSES>;
    constexpr size_t lds = MISSES ? S::enc_lds_bytes : DECRYPT ? S::lds_bytes : 0;
    hipError_t e = set_lds<LOGN, LOGR, kernel, lds>();
    if (e != hipSuccess) return e;
    // a persistent grid: the workgroups that fit on the device at once
    static std::atomic<int> resident{0};
    int g = resident.load(std::memory_order_relaxed);
    if (g == 0) {
      int per_cu = 0, cus = 0, dev = 0;
      e = hipGetDevice(&dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel), S::T, lds);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      g = (per_cu < 1 ? 1 : per_cu) * (cus < 1 ? 1 : cus);
      resident.store(g, std::memory_order_relaxed);
    }
    uint64_t grid = job.n < (uint64_t)g ? job.n : (uint64_t)g;
    FusedJob jb = job;
    if (jb.ring) {  // each workgroup cycles through slots of its own: at most one per slot
      if (!jb.dec_out) return hipErrorInvalidValue;
      if (grid > jb.ring) grid = jb.ring;
    }
    if (!jb.cursor) return hipErrorInvalidValue;
    e = launch_fill_u32(jb.cursor, kXcds, 0u, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cached_fused<LOGN, LOGR, RC, BRIGHT, DECRYPT, MISSES>), dim3((uint32_t)grid), dim3(S::T), lds,
                       st, jb, c->d_lc, c->dev);
    return hipGetLastError();
  }
  // misses: false when the job's cache holds every value (no pixel is encrypted in full)
  static hipError_t fused(const ckks_ctx *c, const FusedJob &job, bool misses, hipStream_t st) {
    if (job.n == 0) return hipSuccess;
    const bool bright = job.seg_b != nullptr, dec = job.dec_out != nullptr;
    if (!misses) {
      if (!job.counters) return hipErrorInvalidValue;
      if (bright) return dec ? fused_as<true, true, false>(c, job, st) : fused_as<true, false, false>(c, job, st);
      return dec ? fused_as<false, true, false>(c, job, st) : fused_as<false, false, false>(c, job, st);
    }
    if (bright) return dec ? fused_as<true, true, true>(c, job, st) : fused_as<true, false, true>(c, job, st);
    return dec ? fused_as<false, true, true>(c, job, st) : fused_as<false, false, true>(c, job, st);
  }
  static hipError_t keygen(const ckks_ctx *c, uint64_t s0, uint64_t s1, hipStream_t st) {
    hipError_t e = set_lds<LOGN, LOGR, k_keygen<LOGN, LOGR, RC>>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_keygen<LOGN, LOGR, RC>), dim3(c->lc.L), dim3(S::T), S::lds_bytes, st, s0, s1, c->d_lc, c->dev);
    return hipGetLastError();
  }
  static hipError_t prepare(const ckks_ctx *c, hipStream_t st) {
    hipError_t e = set_lds<LOGN, LOGR, k_keys_prepare<LOGN, LOGR, RC>>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_keys_prepare<LOGN, LOGR, RC>), dim3(c->lc.L, 3), dim3(S::T), S::lds_bytes, st, c->d_lc, c->dev);
    return hipGetLastError();
  }
  static hipError_t relin_keygen(const ckks_ctx *c, uint64_t s0, uint64_t s1, hipStream_t st) {
    hipError_t e = set_lds<LOGN, LOGR, k_relin_keygen<LOGN, LOGR, RC>>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_relin_keygen<LOGN, LOGR, RC>), dim3(c->lc.L, c->lc.L + 1), dim3(S::T), S::lds_bytes, st, s0,
                       s1, c->d_lc, c->dev);
    return hipGetLastError();
  }
  static hipError_t relin_prepare(const ckks_ctx *c, hipStream_t st) {
    hipError_t e = set_lds<LOGN, LOGR, k_relin_prepare<LOGN, LOGR, RC>>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_relin_prepare<LOGN, LOGR, RC>), dim3(c->lc.L, c->lc.L + 1, 2), dim3(S::T), S::lds_bytes, st,
                       c->d_lc, c->dev);
    return hipGetLastError();
  }
  static hipError_t mul(const ckks_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n, int level,
                        uint64_t *scratch, hipStream_t st) {
    hipError_t e = set_lds<LOGN, LOGR, k_mul<LOGN, LOGR, RC>>();
    if (e != hipSuccess) return e;
    const uint64_t grid = n < kMulGroups ? n : kMulGroups;
    hipLaunchKernelGGL((k_mul<LOGN, LOGR, RC>), dim3((uint32_t)grid), dim3(S::T), S::lds_bytes, st, a, b, out, n, level,
                       scratch, c->d_lc, c->dev);
    return hipGetLastError();
  }
  template <int LIMBS>
  static hipError_t decrypt_as(const ckks_ctx *c, const uint64_t *cts, uint64_t n, int level, double scale,
                               double *out, hipStream_t st, uint64_t max_grid) {
    hipError_t e = set_lds<LOGN, LOGR, k_decrypt<LOGN, LOGR, RC, LIMBS>>();
    if (e != hipSuccess) return e;
    uint64_t grid = n < (1u << 20) ? n : (1u << 20);
    if (max_grid && grid > max_grid) grid = max_grid;
    hipLaunchKernelGGL((k_decrypt<LOGN, LOGR, RC, LIMBS>), dim3((uint32_t)grid), dim3(S::T), S::lds_bytes, st, cts, n,
                       level, 1.0 / scale, out, c->d_lc, c->dev);
    return hipGetLastError();
  }
  static hipError_t decrypt(const ckks_ctx *c, const uint64_t *cts, uint64_t n, int level, double scale, double *out,
                            int limbs, hipStream_t st, uint64_t max_grid) {
    if (limbs == 2 && level >= 2) return decrypt_as<2>(c, cts, n, level, scale, out, st, max_grid);
    if (limbs != 1) return hipErrorInvalidValue;
    return decrypt_as<1>(c, cts, n, level, scale, out, st, max_grid);
  }
};

// All launchers of one ring degree, selecting the thread shape (c->logr) and the
// reduction class (c->rc) at run time.
template <int LOGN>
struct RingLaunch {
  template <typename F>
  static hipError_t pick(const ckks_ctx *c, int logr, F f) {
    if constexpr (LOGN - 3 <= 10) {  // 8 values per thread: N/8 threads, at most 1024
      if (logr == 3) return c->rc ? f(Launch<LOGN, 3, 1>{}) : f(Launch<LOGN, 3, 0>{});
    }
    if (logr == 4) return c->rc ? f(Launch<LOGN, 4, 1>{}) : f(Launch<LOGN, 4, 0>{});
    if (logr == 5) return c->rc ? f(Launch<LOGN, 5, 1>{}) : f(Launch<LOGN, 5, 0>{});
    return hipErrorInvalidValue;
  }
};

}  // namespace ckks

// Define the per-ring-degree launcher entry points.  Each ring degree's kernels are spread
// over three translation units (k_ntt_<LOGN>_{enc,mul,fused}.hip) so they compile in parallel.
#define CKKS_DEFINE_RING_ENC(LOGN)                                                                                  \
  namespace ckks {                                                                                                  \
  hipError_t launch_encrypt_##LOGN(const ckks_ctx *c, const EncJob &job, uint64_t grid, hipStream_t st) {           \
    return RingLaunch<LOGN>::pick(c, c->logr_enc, [&](auto L) { return decltype(L)::encrypt(c, job, grid, st); });  \
  }                                                                                                                 \
  hipError_t launch_keygen_##LOGN(const ckks_ctx *c, uint64_t s0, uint64_t s1, hipStream_t st) {                    \
    return RingLaunch<LOGN>::pick(c, c->logr_enc, [&](auto L) { return decltype(L)::keygen(c, s0, s1, st); });      \
  }                                                                                                                 \
  hipError_t launch_keys_prepare_##LOGN(const ckks_ctx *c, hipStream_t st) {                                        \
    return RingLaunch<LOGN>::pick(c, c->logr_enc, [&](auto L) { return decltype(L)::prepare(c, st); });             \
  }                                                                                                                 \
  hipError_t launch_decrypt_##LOGN(const ckks_ctx *c, const uint64_t *cts, uint64_t n, int level, double scale,     \
                                   double *out, int limbs, hipStream_t st, uint64_t max_grid) {                     \
    return RingLaunch<LOGN>::pick(c, c->logr_dec, [&](auto L) {                                                     \
      return decltype(L)::decrypt(c, cts, n, level, scale, out, limbs, st, max_grid);                               \
    });                                                                                                             \
  }                                                                                                                 \
  }

#define CKKS_DEFINE_RING_MUL(LOGN)                                                                                  \
  namespace ckks {                                                                                                  \
  hipError_t launch_relin_keygen_##LOGN(const ckks_ctx *c, uint64_t s0, uint64_t s1, hipStream_t st) {              \
    return RingLaunch<LOGN>::pick(c, c->logr_mul, [&](auto L) { return decltype(L)::relin_keygen(c, s0, s1, st); });   \
  }                                                                                                                 \
  hipError_t launch_relin_prepare_##LOGN(const ckks_ctx *c, hipStream_t st) {                                       \
    return RingLaunch<LOGN>::pick(c, c->logr_mul, [&](auto L) { return decltype(L)::relin_prepare(c, st); });          \
  }                                                                                                                 \
  hipError_t launch_mul_##LOGN(const ckks_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n,  \
                               int level, uint64_t *scratch, hipStream_t st) {                                      \
    return RingLaunch<LOGN>::pick(                                                                                  \
        c, c->logr_mul, [&](auto L) { return decltype(L)::mul(c, a, b, out, n, level, scratch, st); });                \
  }                                                                                                                 \
  }

#define CKKS_DEFINE_RING_FUSED(LOGN)                                                                                \
  namespace ckks {                                                                                                  \
  hipError_t launch_cached_fused_##LOGN(const ckks_ctx *c, const FusedJob &job, bool misses, hipStream_t st) {     \
    return RingLaunch<LOGN>::pick(c, misses ? c->logr_enc : c->logr_dec,                                            \
                                  [&](auto L) { return decltype(L)::fused(c, job, misses, st); });                  \
  }                                                                                                                 \
  }
