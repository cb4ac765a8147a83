// Cached encryption (Sec. 3.2) with the randomness of Sec. 3.3.
//
// A small metadata pass decides, per pixel, how its ciphertext is assembled (which
// cache entry, which pool member, which signed radix multiples); the gather kernels
// then stream the ciphertext rows, reading cache entries that stay resident in the
// L2 / Infinity Cache and writing each output residue once.  Pixels a value cache
// does not hold go to a compacted list that the plain encryption kernel consumes.
#include <algorithm>

#include "internal.hpp"
#include "modarith.hpp"
#include "philox.hpp"

namespace ckks {

constexpr int kThreads = 256;

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// 256-bin histogram of a pixel array (LDS counters per workgroup, then global).
__global__ void __launch_bounds__(kThreads) k_histogram(const uint8_t *__restrict__ px, uint64_t n, uint32_t *hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
    atomicAdd(&h[px[i]], 1u);
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Rank of every value by (count descending, value ascending); the first k values that
// occur become cache slots 0..count-1 with Philox index 256 + value.
__global__ void __launch_bounds__(256)
    k_topk(const uint32_t *__restrict__ hist, uint32_t k, int16_t *slot_of, uint32_t *vals, uint64_t *ts,
           uint32_t *count) {
  __shared__ uint32_t h[256];
  const int v = threadIdx.x;
  h[v] = hist[v];
  __syncthreads();
  const uint32_t hv = h[v];
  uint32_t rank = 0, nz = 0;
  for (int w = 0; w < 256; w++) {
    const uint32_t hw = h[w];
    rank += (hw > hv || (hw == hv && w < v)) ? 1u : 0u;
    nz += hw > 0 ? 1u : 0u;
  }
  if (hv > 0 && rank < k) {
    slot_of[v] = (int16_t)rank;
    vals[rank] = (uint32_t)v;
    ts[rank] = 256 + (uint64_t)v;
  } else {
    slot_of[v] = -1;
  }
  if (v == 0) *count = nz < k ? nz : k;
}

// Bucket of a hit with pool member u and cache slot: pool members are taken in groups of
// kPoolGroup, and within a group the order is slot-major, so a stretch of the hit list
// touches a few pool entries and few value entries at a time (both stay in L2).  With
// nslots = 1 the bucket is the pool member.
constexpr uint32_t kPoolGroup = 2;
__device__ __forceinline__ uint32_t hit_bucket(uint32_t u, uint32_t slot, uint32_t nslots, uint32_t npool) {
  if (nslots == 1) return u;
  const uint32_t g0 = u - u % kPoolGroup, gsz = min(kPoolGroup, npool - g0);
  return g0 * nslots + slot * gsz + (u - g0);
}

// Per pixel t: meta = (slot + 1) | u << 16 for a cached value, with pool member
// u = floor(npool * w / 2^64) from auxiliary word 0; 0 for a value that is not cached,
// whose index is appended to the miss list.  Hits are counted per bucket (hit_bucket).
__global__ void __launch_bounds__(kThreads)
    k_value_meta(const uint8_t *__restrict__ px, uint64_t n, uint64_t first_index, uint64_t s0, uint64_t s1,
                 const int16_t *__restrict__ slot_of, uint32_t npool, uint32_t nslots, uint32_t *__restrict__ meta,
                 uint32_t *__restrict__ miss_list, uint32_t *miss_count, uint32_t *__restrict__ ucount) {
  for (uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kThreads) {
    const int slot = slot_of[px[t]];
    if (slot >= 0) {
      const uint64_t w = philox4x64_10(first_index + t, kTagAux, 0, 0, s0, s1).w[0];
      const uint32_t u = (uint32_t)mulhi64(w, npool);
      meta[t] = (uint32_t)(slot + 1) | (u << 16);
      atomicAdd(&ucount[hit_bucket(u, (uint32_t)slot, nslots, npool)], 1u);
    } else {
      meta[t] = 0;
      miss_list[atomicAdd(miss_count, 1u)] = (uint32_t)t;
    }
  }
}

// Exclusive prefix sum of the per-bucket hit counts in two levels: each workgroup of
// kScanThreads threads scans its block of buckets in place (they become the bucket cursors
// within the block) and writes the block's total; then one small workgroup turns the block
// totals into block offsets and the total hit count.  The scatter adds a bucket's block
// offset to the cursor it takes.
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(uint32_t *__restrict__ ucount, uint32_t nb,
                                                              uint32_t *__restrict__ block_tot) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const uint32_t i = blockIdx.x * kScanThreads + threadIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t v = i < nb ? ucount[i] : 0u;
  uint32_t x = v;  // inclusive scan within the wave
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t k = 0; k < w; k++) before += wsum[k];
  if (i < nb) ucount[i] = before + x - v;
  if (threadIdx.x == kScanThreads - 1) block_tot[blockIdx.x] = before + x;
}

// Block totals -> exclusive block offsets (in place) and the total hit count.
__global__ void __launch_bounds__(64) k_scan_tops(uint32_t *__restrict__ block_tot, uint32_t nblk,
                                                  uint32_t *__restrict__ total) {
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t b = 0; b < nblk; b++) {
      const uint32_t t = block_tot[b];
      block_tot[b] = run;
      run += t;
    }
    *total = run;
  }
}

// Hit pixels grouped by bucket (order inside a bucket is arbitrary; every output row is
// written independently, so the result does not depend on it).
__global__ void __launch_bounds__(kThreads)
    k_value_scatter(const uint32_t *__restrict__ meta, uint64_t n, uint32_t nslots, uint32_t npool,
                    uint32_t *__restrict__ cursor, const uint32_t *__restrict__ block_off, uint32_t *__restrict__ hits) {
  for (uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t m = meta[t];
    if (m != 0) {
      const uint32_t b = hit_bucket(m >> 16, (m & 0xffffu) - 1u, nslots, npool);
      hits[block_off[b / kScanThreads] + atomicAdd(&cursor[b], 1u)] = (uint32_t)t;
    }
  }
}

// out = entry[slot] + pool[u] for cached pixels (missed pixels are written by the plain
// encryption kernel), plus the optional fused brightness encode(b_image) on c0 (see
// EncJob).  A persistent grid whose workgroups claim hit-list positions per XCD
// (xcd_claim) and stream all 2L rows of each: the hit list is grouped by pool member and
// cache slot, so each XCD works through a few (entry, pool member) pairs at a time and
// they stay in its L2, while the output streams past with non-temporal stores.
struct Bright {
  const uint64_t *seg_end;
  const double *seg_b;
  uint32_t n_seg;
  uint64_t seg_base;
  double scale;  // scale * 2^(1 - log N)
  const double *cosj;
};

__device__ __forceinline__ uint64_t add_encoded(uint64_t z, double fb, double cj, double q, double qinv, uint64_t qi) {
  return add_mod(z, f64_to_u64(canon(__builtin_rint(fb * cj), q, qinv)), qi);
}

__global__ void __launch_bounds__(kThreads)
    k_value_gather(const uint64_t *__restrict__ entries, const uint64_t *__restrict__ pool,
                   const uint32_t *__restrict__ meta, const uint32_t *__restrict__ hits,
                   uint32_t *__restrict__ counters, int L, int log_n, const LimbConsts *__restrict__ lcp,
                   Bright br, uint64_t *__restrict__ out) {
  const LimbConsts &lc = *lcp;
  const int N = 1 << log_n;
  const uint64_t S = (uint64_t)2 * L * N;
  const uint64_t nh = counters[1];
  __shared__ uint64_t s_item;
  uint32_t region = 0;
  for (uint64_t idx = xcd_claim(counters + 2, nh, region, &s_item); idx < nh;
       idx = xcd_claim(counters + 2, nh, region, &s_item)) {
    const uint64_t ct = hits[idx];
    const uint32_t m = meta[ct];
    const u64x2 *pe = reinterpret_cast<const u64x2 *>(entries + (uint64_t)((m & 0xffffu) - 1) * S);
    const u64x2 *pz = reinterpret_cast<const u64x2 *>(pool + (uint64_t)(m >> 16) * S);
    u64x2 *po = reinterpret_cast<u64x2 *>(out + ct * S);
    const double fb = br.seg_b ? br.seg_b[segment_of(br.seg_end, br.n_seg, br.seg_base + ct)] * br.scale : 0.0;
    for (int pl = 0; pl < 2 * L; pl++) {
      const int l = pl % L;
      const uint64_t q = lc.qi[l];
      const int base = pl * (N / 2);
      if (pl < L && fb != 0.0) {
        const double qd = lc.q[l], qinv = lc.qinv[l];
        const double2 *cs = reinterpret_cast<const double2 *>(br.cosj);
        for (int i = threadIdx.x; i < N / 2; i += kThreads) {
          const u64x2 a = pe[base + i], b = pz[base + i];
          const double2 c = cs[i];
          u64x2 z;
          z.x = add_encoded(add_mod(a.x, b.x, q), fb, c.x, qd, qinv, q);
          z.y = add_encoded(add_mod(a.y, b.y, q), fb, c.y, qd, qinv, q);
          __builtin_nontemporal_store(z, po + base + i);
        }
        continue;
      }
      for (int i = threadIdx.x; i < N / 2; i += 2 * kThreads) {
        const u64x2 a0 = pe[base + i], b0 = pz[base + i];
        const u64x2 a1 = pe[base + i + kThreads], b1 = pz[base + i + kThreads];
        u64x2 z0, z1;
        z0.x = add_mod(a0.x, b0.x, q);
        z0.y = add_mod(a0.y, b0.y, q);
        z1.x = add_mod(a1.x, b1.x, q);
        z1.y = add_mod(a1.y, b1.y, q);
        __builtin_nontemporal_store(z0, po + base + i);
        __builtin_nontemporal_store(z1, po + base + i + kThreads);
      }
    }
  }
}

// Per pixel: signed multiples k_i of the radix entries Enc(r^i) so that
//   c = Enc(0) + sum_i k_i Enc(r^i),  k_i = d_i + b_i - r * b_{i+1},
// where d_i are the base-r digits and b_i (i = 1..D-1) bit i-1 of auxiliary word 1:
// each set bit adds Enc(r^i) and subtracts r copies of Enc(r^(i-1)) (Sec. 3.3).
__global__ void __launch_bounds__(kThreads)
    k_radix_meta(const uint8_t *__restrict__ px, uint64_t n, uint64_t first_index, uint64_t s0, uint64_t s1,
                 uint32_t r, uint32_t D, int16_t *__restrict__ meta, uint32_t *bad) {
  for (uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kThreads) {
    uint32_t p = px[t];
    const uint64_t aux = philox4x64_10(first_index + t, kTagAux, 0, 0, s0, s1).w[1];
    int k[kMaxDigits];
#pragma unroll
    for (int i = 0; i < kMaxDigits; i++) {
      k[i] = 0;
      if ((uint32_t)i < D) {
        k[i] = (int)(p % r);
        p /= r;
      }
    }
    if (p != 0) atomicOr(bad, 1u);
#pragma unroll
    for (int i = 1; i < kMaxDigits; i++) {
      if ((uint32_t)i < D && ((aux >> (i - 1)) & 1)) {
        k[i] += 1;
        k[i - 1] -= (int)r;
      }
    }
    int16_t *o = meta + t * kMaxDigits;
#pragma unroll
    for (int i = 0; i < kMaxDigits; i++) o[i] = (int16_t)k[i];
  }
}

// out row = entry0 row + sum_i k_i entry(1+i) row, in exact FP64 arithmetic: each
// product k_i e is a modular product with a small multiplier (|k_i| <= 256), the sum of
// at most 1 + 8 reduced terms stays below 2^53, and one final reduction makes it
// canonical.  The D + 1 table rows (D + 1 rows of N residues per limb and polynomial)
// stay L2-resident; the output is written with non-temporal stores.
__global__ void __launch_bounds__(kThreads)
    k_radix_gather(const uint64_t *__restrict__ entries, const int16_t *__restrict__ meta, uint64_t rows, int L,
                   int log_n, uint32_t D, const LimbConsts *__restrict__ lcp, uint64_t *__restrict__ out) {
  const LimbConsts &lc = *lcp;
  const int N = 1 << log_n;
  const uint64_t S = (uint64_t)2 * L * N;
  for (uint64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const uint64_t ct = row / (uint64_t)(2 * L);
    const int pl = (int)(row % (uint64_t)(2 * L));
    const int l = pl % L;
    const double q = lc.q[l], qinv = lc.qinv[l];
    double k[kMaxDigits];
#pragma unroll
    for (int i = 0; i < kMaxDigits; i++) k[i] = (double)meta[ct * kMaxDigits + i];
    const u64x2 *e0 = reinterpret_cast<const u64x2 *>(entries + (uint64_t)pl * N);
    u64x2 *po = reinterpret_cast<u64x2 *>(out + row * N);
    for (int j = threadIdx.x; j < N / 2; j += kThreads) {
      const u64x2 a = e0[j];
      double x0 = u64_to_f64(a.x), x1 = u64_to_f64(a.y);
#pragma unroll
      for (int i = 0; i < kMaxDigits; i++) {
        if ((uint32_t)i < D) {
          const u64x2 b = e0[(uint64_t)(1 + i) * (S / 2) + j];
          x0 += mulmod(u64_to_f64(b.x), k[i], q, qinv);
          x1 += mulmod(u64_to_f64(b.y), k[i], q, qinv);
        }
      }
      u64x2 z;
      z.x = f64_to_u64(canon(x0, q, qinv));
      z.y = f64_to_u64(canon(x1, q, qinv));
      __builtin_nontemporal_store(z, po + j);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static uint32_t grid_for(uint64_t items, uint64_t per_block) {
  const uint64_t g = (items + per_block - 1) / per_block;
  return (uint32_t)(g == 0 ? 1 : (g < (1u << 20) ? g : (1u << 20)));
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t n, uint32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_histogram_topk(const ckks_ctx *c, const uint8_t *px, uint64_t n, uint32_t topk, uint32_t *hist,
                                 ckks_cache *cache, hipStream_t st) {
  (void)c;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, hist, 256u, 0u);
  if (n) hipLaunchKernelGGL(k_histogram, dim3(grid_for(n, 16 * kThreads)), dim3(kThreads), 0, st, px, n, hist);
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(256), 0, st, hist, topk, cache->slot_of, cache->vals, cache->ts,
                     cache->count);
  return hipGetLastError();
}

hipError_t launch_value_meta(const ckks_ctx *c, const ckks_cache *cache, const uint8_t *px, uint64_t n,
                             uint64_t first_index, uint64_t seed0, uint64_t seed1, uint32_t *meta,
                             uint32_t *miss_list, uint32_t *counters, uint32_t *hits, hipStream_t st) {
  (void)c;
  uint32_t *miss_count = counters, *hit_count = counters + 1, *ucount = counters + kCountersHead;
  const uint32_t nb = value_buckets(cache), nblk = value_scan_blocks(cache);
  uint32_t *block_tot = ucount + nb;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(kCountersHead + nb, kThreads)), dim3(kThreads), 0, st, counters,
                     kCountersHead + nb, 0u);
  hipLaunchKernelGGL(k_value_meta, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, st, px, n, first_index, seed0,
                     seed1, cache->slot_of, cache->pool, value_slot_buckets(cache), meta, miss_list, miss_count,
                     ucount);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nblk), dim3(kScanThreads), 0, st, ucount, nb, block_tot);
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(64), 0, st, block_tot, nblk, hit_count);
  hipLaunchKernelGGL(k_value_scatter, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, st, meta, n,
                     value_slot_buckets(cache), cache->pool, ucount, block_tot, hits);
  return hipGetLastError();
}

hipError_t launch_value_gather(const ckks_ctx *c, const ckks_cache *cache, const uint32_t *meta,
                               uint32_t *counters, const uint32_t *hits, uint64_t n, uint64_t *out,
                               const EncJob *bright, hipStream_t st, uint64_t max_grid) {
  Bright br{nullptr, nullptr, 0, 0, 0.0, c->dev.cosj};
  if (bright && bright->seg_b) {
    br.seg_end = bright->seg_end;
    br.seg_b = bright->seg_b;
    br.n_seg = bright->n_seg;
    br.seg_base = bright->seg_base;
    br.scale = bright->bright_scale;
  }
  // n is an upper bound of the hit count, which the kernel reads; a persistent grid claims
  // the hits per XCD (the cursors were zeroed with the counters by the metadata pass), at
  // most max_grid workgroups when another kernel is to run beside it
  uint64_t grid = std::min<uint64_t>(n, (uint64_t)c->gather_wgs * c->num_cus);
  if (max_grid && grid > max_grid) grid = max_grid;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_value_gather, dim3((uint32_t)grid), dim3(kThreads), 0, st, cache->entries, cache->pool_cts,
                     meta, hits, counters, c->prm.L, c->prm.log_n, c->d_lc, br, out);
  return hipGetLastError();
}

hipError_t launch_radix_meta(const ckks_ctx *c, const ckks_cache *cache, const uint8_t *px, uint64_t n,
                             uint64_t first_index, uint64_t seed0, uint64_t seed1, int16_t *meta, uint32_t *bad,
                             hipStream_t st) {
  (void)c;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, bad, 1u, 0u);
  hipLaunchKernelGGL(k_radix_meta, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, st, px, n, first_index, seed0,
                     seed1, cache->base, cache->digits, meta, bad);
  return hipGetLastError();
}

hipError_t launch_radix_gather(const ckks_ctx *c, const ckks_cache *cache, const int16_t *meta, uint64_t n,
                               uint64_t *out, hipStream_t st) {
  const int L = c->prm.L;
  const uint64_t rows = n * 2 * (uint64_t)L;
  hipLaunchKernelGGL(k_radix_gather, dim3(row_grid(c, rows)), dim3(kThreads), 0, st, cache->entries, meta, rows, L,
                     c->prm.log_n, cache->digits, c->d_lc, out);
  return hipGetLastError();
}

}  // namespace ckks
