// Cached encryption in one persistent launch (Sec. 3.2 caching with the randomness of
// Sec. 3.3), optionally with each image's brightness (Sec. 4.4.2) and the decryption of
// every ciphertext (Sec. 2.2.2) fused in.  Included by the NTT implementation header,
// whose shapes, samplers, transforms and encryption body it uses.
//
// The items are the pixels a value cache misses (full encryption: compute-bound) and the
// pixels it holds (entry + pool member: a stream of HBM writes).  Item i of the launch is
// a miss when floor((i+1) M / (M+H)) > floor(i M / (M+H)) for M misses and H hits, so the
// two kinds are spread evenly over the item sequence; each workgroup takes every G-th
// item (G = the resident grid, XCD-contiguous), and at any moment some CUs encrypt while
// others stream, instead of one launch of each kind after the other.  Without a cache
// every pixel is a miss.  The hit list is ordered by pool member and cache slot (see
// k_cache.hip), so consecutive hits, which one XCD processes together, read a few
// entries from its L2.
//
// With decryption, limb 0 of each ciphertext is produced last and its c0, c1 rows stay in
// registers, in the layout the decryption's transform starts from: the ciphertext is still
// written in full (all limbs), and the decryption reads exactly the values written.
#pragma once

namespace ckks {

// One row (polynomial `poly` of limb l) of a cache hit: entry + pool member (+ the brightness
// encoding on c0), written with non-temporal stores.  With KEEP the values are also returned
// in k (register r: coefficient tid + T r, the layout the decryption's transform starts
// from); other rows move as 16-byte pairs (register j: coefficients 2p, 2p + 1 with
// p = tid + T j), half the memory instructions.  One row at a time keeps the registers of
// a kept row and of the loads in flight within the decryption's budget.
template <int LOGN, int LOGR, bool BRIGHT, bool KEEP>
__device__ __forceinline__ void gather_row(int poly, int l, int L, const uint64_t *__restrict__ pe,
                                           const uint64_t *__restrict__ pz, uint64_t *__restrict__ po, double fb,
                                           const LimbConsts &lc, const DevTables &dt, double (&k)[1 << LOGR]) {
  using S = Shape<LOGN, LOGR>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const int tid = opaque(threadIdx.x);
  const uint64_t q = lc.qi[l];
  const size_t row = ((size_t)poly * L + l) * N;
  const uint64_t *e = pe + row, *z = pz + row;
  uint64_t *o = po + row;
  const double qd = lc.q[l], qinv = lc.qinv[l];
  if constexpr (KEEP) {
    uint64_t a[R], b[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const unsigned c = tid + T * r;
      a[r] = ld_word(e, c);
      b[r] = ld_word(z, c);
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const unsigned c = tid + T * r;
      uint64_t v = add_mod(a[r], b[r], q);
      if (BRIGHT && poly == 0)
        v = add_mod(v, f64_to_u64(canon(__builtin_rint(fb * ld_table(dt.cosj, c)), qd, qinv)), q);
      __builtin_nontemporal_store(v, word_at(o, c));
      k[r] = u64_to_f64(v);
    }
  } else {
    const u64x2 *e2 = reinterpret_cast<const u64x2 *>(e), *z2 = reinterpret_cast<const u64x2 *>(z);
    u64x2 *o2 = reinterpret_cast<u64x2 *>(o);
    constexpr int H = R / 4 > 0 ? R / 4 : 1;  // pairs per half row and thread
#pragma unroll
    for (int h = 0; h < R / 2; h += H) {
      u64x2 a[H], b[H];
#pragma unroll
      for (int j = 0; j < H; j++) {
        a[j] = e2[tid + T * (h + j)];
        b[j] = z2[tid + T * (h + j)];
      }
#pragma unroll
      for (int j = 0; j < H; j++) {
        const unsigned p = tid + T * (h + j);
        u64x2 v;
        v.x = add_mod(a[j].x, b[j].x, q);
        v.y = add_mod(a[j].y, b[j].y, q);
        if (BRIGHT && poly == 0) {
          const double2 cs = reinterpret_cast<const double2 *>(dt.cosj)[p];
          v.x = add_mod(v.x, f64_to_u64(canon(__builtin_rint(fb * cs.x), qd, qinv)), q);
          v.y = add_mod(v.y, f64_to_u64(canon(__builtin_rint(fb * cs.y), qd, qinv)), q);
        }
        __builtin_nontemporal_store(v, o2 + p);
      }
    }
  }
}

// Slot 0 of the decryption of the ciphertext whose limb-0 rows are c0 and x (canonical
// values in the first-pass layout; x is consumed): the same operations, in the same order,
// as the one-limb decryption kernel, so the decoded value is identical to it for the same
// thread shape.  Returns the workgroup sum in thread 0.
template <int LOGN, int LOGR, int RC>
__device__ __forceinline__ double decode_regs(const double (&c0)[1 << LOGR], double (&x)[1 << LOGR], double *lds,
                                              double *red, const LimbConsts &lc, const DevTables &dt) {
  using S = Shape<LOGN, LOGR>;
  using Red = Schedule<LOGN, RC>;
  constexpr int R = S::R, T = S::T;
  const int tid = opaque(threadIdx.x);
  const double q = lc.q[0], qinv = lc.qinv[0];
  ntt_forward<LOGN, LOGR, Red::fwd_big>(x, lds, tid, dt.tw_fwd, q, qinv);
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = mulmod(x[r], ld_table(dt.s_hat, elem_index<LOGN, LOGR, S::LAST>(tid, r)), q, qinv);
  ntt_inverse<LOGN, LOGR, Red::inv>(x, lds, tid, dt.tw_inv, q, qinv);
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = center(x[r] + c0[r], q, qinv);
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) acc = __builtin_fma(x[r], ld_table(dt.cosj, tid + T * r), acc);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < T / 64; w++) s += red[w];
  return s;
}

// MISSES = false compiles the kernel for a cache that holds every value (no misses): it
// then needs only the decryption's LDS and registers, so more workgroups share a CU and
// one streams its ciphertext while another runs its transforms.
template <int LOGN, int LOGR, bool MISSES>
constexpr int fused_waves_hint() {
  return MISSES ? 1 : decrypt_waves_per_eu<LOGN, LOGR>();
}

// What one item of the launch is: its position i in the item sequence (total: no item
// left), the pixel index, the meta word of a hit or the pixel value of a miss, and the
// brightness multiplier of its image.
struct ItemDesc {
  uint64_t i, item;
  uint32_t word, miss;
  double fb;
};

// Claims the next item of this workgroup from the XCD regions of xcd_claim, without
// barriers (one thread calls it; `region` keeps its state).
__device__ __forceinline__ uint64_t claim_one(uint32_t *cursor, uint64_t total, uint32_t &region) {
  const uint32_t home = blockIdx.x % kXcds;
  for (; region < kXcds; region++) {
    const uint32_t x = (home + region) % kXcds;
    const uint64_t lo = total * x / kXcds, hi = total * (x + 1) / kXcds;
    const uint64_t i = lo + atomicAdd(&cursor[x], 1u);
    if (i < hi) return i;
  }
  return total;
}

// Item i of M misses and total - M hits: a miss when floor((i+1) M / total) > floor(i M / total).
template <bool BRIGHT, bool MISSES>
__device__ __forceinline__ ItemDesc resolve_item(const FusedJob &job, uint64_t i, uint64_t M, uint64_t total) {
  ItemDesc d{i, 0, 0, 0, 0.0};
  if (i >= total) return d;
  const uint64_t mb = i * M / total, mb1 = (i + 1) * M / total;  // i, M < 2^32: no overflow
  if (MISSES && mb1 > mb) {
    d.miss = 1;
    d.item = job.miss_list ? (uint64_t)job.miss_list[mb] : mb;
    d.word = job.px[d.item];
  } else {
    d.item = job.hits[i - mb];
    d.word = job.meta[d.item];
  }
  if (BRIGHT) d.fb = job.seg_b[segment_of(job.seg_end, job.n_seg, job.seg_base + d.item)] * job.bright_scale;
  return d;
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x), hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (uint64_t)hi << 32 | lo;
}

template <int LOGN, int LOGR, int RC, bool BRIGHT, bool DECRYPT, bool MISSES>
__global__ void __launch_bounds__(1 << (LOGN - LOGR))
    __attribute__((amdgpu_waves_per_eu(fused_waves_hint<LOGN, LOGR, MISSES>())))
    k_cached_fused(FusedJob job, const LimbConsts *__restrict__ lcp, DevTables dt) {
  using S = Shape<LOGN, LOGR>;
  constexpr int N = S::N, R = S::R, T = S::T;
  const LimbConsts &lc = *lcp;
  extern __shared__ double lds[];
  uint64_t *cdt = reinterpret_cast<uint64_t *>(lds + S::SLOTS);
  double *red = lds + S::SLOTS + kCdtSlots;
  uint16_t *lds16 = reinterpret_cast<uint16_t *>(lds);
  uint16_t *smpl = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(lds) + S::enc_base_bytes);
  const int tid = threadIdx.x;
  if constexpr (MISSES)
    for (int i = tid; i < kCdtSlots; i += T) cdt[i] = dt.cdt[i];
  const int L = lc.L, B = lc.B;
  const uint64_t S_ct = (uint64_t)2 * L * N;
  const uint64_t M = !MISSES ? 0 : job.counters ? job.counters[0] : job.n;  // misses (all pixels without a cache)
  const uint64_t H = job.counters ? job.counters[1] : 0;      // hits
  const uint64_t total = M + H;
  // ring: workgroup b owns slots [b K, (b+1) K), K = ring / grid, and cycles through them
  const uint64_t K = job.ring / gridDim.x;
  // Thread 0 claims and resolves the next item (dependent loads: hit list, meta word, image
  // of the pixel) while the other waves work on the current one; the descriptors alternate
  // between two LDS slots, and the barrier that ends an item publishes the next.
  __shared__ ItemDesc s_desc[2];
  __shared__ uint32_t s_region;  // claim state of thread 0 (kept in LDS: no register across the item)
  if (tid == 0) {
    uint32_t region = 0;
    s_desc[0] = resolve_item<BRIGHT, MISSES>(job, claim_one(job.cursor, total, region), M, total);
    s_region = region;
  }
  __syncthreads();
  for (uint64_t done = 0;; done++) {
    const ItemDesc &cd = s_desc[done & 1];
    if (uniform_u64(cd.i) >= total) break;
    const uint64_t item = uniform_u64(cd.item);
    const uint32_t word = __builtin_amdgcn_readfirstlane(cd.word);
    const bool miss = MISSES && __builtin_amdgcn_readfirstlane(cd.miss) != 0;
    const double fb = BRIGHT ? __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, cd.fb))) : 0.0;
    if (tid == 0) {
      uint32_t region = s_region;
      s_desc[(done + 1) & 1] = resolve_item<BRIGHT, MISSES>(job, claim_one(job.cursor, total, region), M, total);
      s_region = region;
    }
    const uint64_t ring_slot = job.ring ? blockIdx.x * K + done % K : 0;
    uint64_t *po = job.out + (job.ring ? ring_slot : item) * S_ct;
    double k0[R], k1[R];
    if (miss) {
      if constexpr (MISSES) {  // compiled only where misses can occur
        const double value = (double)word;
        uint32_t smp[R];
        if constexpr (S::kSmpLds)
          draw_samples<LOGN, LOGR>(smpl, cdt, B, opaque(tid), job.seed0, job.seed1, job.first_index + item, kTagV,
                                   kTagE0, kTagE1);
        else
          draw_samples<LOGN, LOGR>(smp, lds16, cdt, B, opaque(tid), job.seed0, job.seed1, job.first_index + item,
                                   kTagV, kTagE0, kTagE1);
        double u0[R], u1[R];
        for (int l = 1; l < L; l++)
          encrypt_limb<LOGN, LOGR, RC, BRIGHT, false>(l, lds, smpl, smp, L, B, value, fb, po, lc, dt, u0, u1);
        encrypt_limb<LOGN, LOGR, RC, BRIGHT, DECRYPT>(0, lds, smpl, smp, L, B, value, fb, po, lc, dt, k0, k1);
      }
    } else {
      const uint64_t *pe = job.entries + (uint64_t)((word & 0xffffu) - 1) * S_ct;
      const uint64_t *pz = job.pool + (uint64_t)(word >> 16) * S_ct;
      double u[R];
      for (int l = 1; l < L; l++) {
        gather_row<LOGN, LOGR, BRIGHT, false>(0, l, L, pe, pz, po, fb, lc, dt, u);
        gather_row<LOGN, LOGR, BRIGHT, false>(1, l, L, pe, pz, po, fb, lc, dt, u);
      }
      gather_row<LOGN, LOGR, BRIGHT, DECRYPT>(1, 0, L, pe, pz, po, fb, lc, dt, k1);
      gather_row<LOGN, LOGR, BRIGHT, DECRYPT>(0, 0, L, pe, pz, po, fb, lc, dt, k0);
    }
    if constexpr (DECRYPT) {
      const double s = decode_regs<LOGN, LOGR, RC>(k0, k1, lds, red, lc, dt);
      if (tid == 0) job.dec_out[item] = s * job.inv_scale;
    }
    __syncthreads();
  }
}

}  // namespace ckks
