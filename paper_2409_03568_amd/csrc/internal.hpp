// Internal declarations shared by the C-ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/ckks_mi355x.h"
#include <rocprofiler-sdk-roctx/roctx.h>
#include "host_math.hpp"

#define CKKS_SEG_HD __host__ __device__

namespace ckks {

constexpr int kMaxL = 16;
constexpr int kMaxDigits = 8;
// Streams whose per-call scratch buffer a context keeps at once (least recently used
// released first).
constexpr size_t kMaxStreamWs = 16;

// Per-limb constants; kernels read the device copy held by the context.  Index L holds
// the special prime of key switching (when the context has one).
struct LimbConsts {
  int L;                 // limbs of the context
  int B;                 // Gaussian bound (0 = no noise)
  double q[kMaxL + 1];
  double qinv[kMaxL + 1];
  double ninv[kMaxL + 1];    // N^-1 mod q_i, centered
  uint64_t qi[kMaxL + 1];
  double pinv[kMaxL];        // qP^-1 mod q_i, centered (ModDown)
  double pmod[kMaxL];        // qP mod q_i, centered (the s^2 term of key-switching key i)
  double q0inv_q1;           // q_0^-1 mod q_1, centered (two-limb CRT of decryption)
};

// Device tables owned by a context.
struct DevTables {
  double *tw_fwd = nullptr;  // [L+1][N] (row L: the special prime)
  double *tw_inv = nullptr;  // [L+1][N]
  double *enc_T = nullptr;   // [N] encoding table at scale Delta
  double *cosj = nullptr;    // [N] cos(pi j / N)
  uint64_t *cdt = nullptr;   // [kCdtSlots]
  int64_t *s = nullptr;      // [N] secret key
  uint64_t *pk = nullptr;    // [2][L][N] public key, coefficient domain
  double *pk_hat = nullptr;  // [2][L][N] NTT domain times N^-1, centered
  double *s_hat = nullptr;   // [L][N] NTT domain times N^-1, centered
  uint64_t *evk = nullptr;   // [L][L+1][2][N] key-switching keys of s^2, coefficient domain
  double *evk_hat = nullptr; // [L][L+1][2][N] the same in the NTT domain times N^-1, centered
};

// What to encrypt, in one of three forms (the launcher picks the kernel variant):
//   pixels:  items 0..n-1 with value px[i] and Philox index first_index + i;
//   list:    items list[0..*list_count) with value px[item], index first_index + item;
//   entries: items 0..count-1 (count = *list_count if set, else n) with value vals[i],
//            index ts[i].
struct EncJob {
  const uint8_t *px = nullptr;
  const uint32_t *vals = nullptr;
  const uint64_t *ts = nullptr;
  const uint32_t *list = nullptr;
  const uint32_t *list_count = nullptr;
  uint64_t n = 0;
  uint64_t first_index = 0;
  uint64_t seed0 = 0, seed1 = 0;
  uint64_t *out = nullptr;  // [n][2][L][N]
  // Optional brightness (Sec. 4.4.2) fused into c0: item i belongs to image
  // upper_bound(seg_end, seg_base + i) and gets encode(seg_b[image]) added in slot 0,
  // i.e. rint(seg_b[image] * bright_scale * cos(pi j / N)) with bright_scale = scale * 2^(1 - log N).
  const uint64_t *seg_end = nullptr;
  const double *seg_b = nullptr;
  uint32_t n_seg = 0;
  uint64_t seg_base = 0;
  double bright_scale = 0.0;
};

// Cached encryption in one persistent launch (k_cached_fused): misses miss_list[0..counters[0])
// are encrypted in full, hits hits[0..counters[1]) are entry + pool member as meta[pixel]
// says; without a cache (counters == NULL) every pixel 0..n-1 is encrypted in full.
// Optional fused brightness (seg_* as in EncJob) and decryption of limb 0 into dec_out.
struct FusedJob {
  const uint8_t *px = nullptr;
  uint64_t n = 0;
  uint64_t first_index = 0;
  uint64_t seed0 = 0, seed1 = 0;
  uint64_t *out = nullptr;               // [n][2][L][N]
  const uint32_t *counters = nullptr;    // [miss count, hit count], or NULL: every pixel a miss
  const uint32_t *miss_list = nullptr;
  const uint32_t *hits = nullptr;
  const uint32_t *meta = nullptr;
  const uint64_t *entries = nullptr;
  const uint64_t *pool = nullptr;
  const uint64_t *seg_end = nullptr;
  const double *seg_b = nullptr;
  uint32_t n_seg = 0;
  uint64_t seg_base = 0;
  double bright_scale = 0.0;
  uint32_t *cursor = nullptr;            // [kXcds] work cursors, zeroed by the launcher
  double *dec_out = nullptr;             // [n] decrypted slot 0 (limb 0), or NULL
  double inv_scale = 0.0;
  // ring = 0: the ciphertext of pixel t goes to out + t S.  Otherwise out holds `ring`
  // ciphertexts: workgroup b owns slots [b K, (b+1) K), K = ring / grid, and writes its
  // successive items to them in turn (only with dec_out: the ciphertexts are written in
  // full but not kept).
  uint64_t ring = 0;
};

// Image of flat pixel index g: the first i with g < seg_end[i] (seg_end ascending, last = total).
CKKS_SEG_HD inline uint32_t segment_of(const uint64_t *seg_end, uint32_t n_seg, uint64_t g) {
  uint32_t lo = 0, hi = n_seg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if (g < seg_end[mid])
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

}  // namespace ckks

// The per-call scratch buffer of one stream (see ckks::WsLease).
struct StreamWorkspace {
  hipStream_t stream = nullptr;
  void *ptr = nullptr;
  uint64_t bytes = 0;
  hipEvent_t last = nullptr;  // recorded after the last call that used ptr
  uint64_t used = 0;          // the context's lease count at the last use (for eviction)
};

struct ckks_ctx {
  int device = 0;
  ckks::host::Resolved prm;
  int N = 0;
  double scale = 0;
  int logr_enc = 4;  // 2^logr values per thread in the encryption / key kernels (4 or 5)
  int logr_dec = 4;  // the same for decryption
  int logr_mul = 4;  // the same for the ciphertext product and its keys
  // Launch shapes of the HBM-bound kernels, in workgroups per compute unit: the row-wise
  // kernels (add, sub, constants, rescale, radix gather; 0 = one workgroup per row) and
  // the value-cache gather.  Results never depend on them.
  int row_wgs = 0;
  int gather_wgs = 8;
  int rc = 1;    // reduction class of the primes: 0 if all q < 2^40, else 1 (q < 2^50)
  ckks::LimbConsts lc{};
  ckks::LimbConsts *d_lc = nullptr;  // device copy of lc (kernels read it with scalar loads)
  ckks::DevTables dev{};
  std::vector<uint64_t> ninv;  // N^-1 mod q_i
  bool has_keys = false;
  bool has_relin = false;      // key-switching keys of s^2 generated
  // Incremented whenever the keys are replaced (keygen, import): caches, batch plans and
  // servers remember the epoch they were made under and refuse to run after a change.
  uint64_t key_epoch = 0;
  hipStream_t pipe[3] = {nullptr, nullptr, nullptr};  // image pipeline stages, created on first use
  hipMemPool_t pool = nullptr;  // stream-ordered scratch that keeps its memory between calls
  int num_cus = 1;              // compute units of the device (bounded, co-resident grids)
  hipStream_t aux = nullptr;    // second stream of cached encryption (misses beside the hit gather)
  void *noalloc_scratch = nullptr;  // this device's fixed scratch array (ckks_encrypt_cached_noalloc)
  std::mutex ws_mu;                 // guards ws for the whole of a call that uses it
  std::vector<StreamWorkspace> ws;  // per-call scratch, one buffer per stream (at most kMaxStreamWs)
  uint64_t ws_leases = 0;           // leases taken so far (orders the buffers by last use)
};


struct ckks_cache {
  ckks_ctx *ctx = nullptr;
  uint64_t key_epoch = 0;         // keys the entries were encrypted under
  int device = 0;
  int kind = 0;
  uint32_t base = 0, digits = 0, topk = 0, pool = 0;
  uint32_t n_slots = 0;           // value entries allocated
  uint64_t *entries = nullptr;    // [n_slots][2][L][N]
  uint64_t *pool_cts = nullptr;   // [pool][2][L][N]
  int16_t *slot_of = nullptr;     // [256] value -> entry slot or -1 (value caches)
  uint32_t *vals = nullptr;       // [n_slots] value of each entry
  uint64_t *ts = nullptr;         // [n_slots] Philox index of each entry
  uint32_t *count = nullptr;      // device: number of valid entries
};

// Hit buckets of value-cached encryption: one per (pool member, cache slot) pair while
// there are at most 65,536 of them (a scan of at most 64 blocks), else one per pool
// member.
inline uint32_t value_slot_buckets(const ckks_cache *cache) {
  return (uint64_t)cache->pool * cache->n_slots <= 65536 ? cache->n_slots : 1u;
}
inline uint32_t value_buckets(const ckks_cache *cache) { return cache->pool * value_slot_buckets(cache); }
// Blocks of 1024 buckets of the two-level hit-count scan.
inline uint32_t value_scan_blocks(const ckks_cache *cache) { return (value_buckets(cache) + 1023) / 1024; }
// Value-cache counters: [0] miss count, [1] hit count, [2..10) the per-XCD work cursors
// of the gather (see xcd_claim), then the bucket cursors and the scan's block offsets.
constexpr uint32_t kCountersHead = 10;
inline uint64_t value_counter_words(const ckks_cache *cache) {
  return kCountersHead + (uint64_t)value_buckets(cache) + value_scan_blocks(cache);
}

// Grid of a row-wise kernel (grid-stride loop over `rows` rows): one workgroup per row,
// or ctx->row_wgs workgroups per compute unit when that is set.
inline uint32_t row_grid(const ckks_ctx *c, uint64_t rows) {
  uint64_t g = rows < (1u << 24) ? rows : (1u << 24);
  if (c->row_wgs > 0 && g > (uint64_t)c->row_wgs * c->num_cus) g = (uint64_t)c->row_wgs * c->num_cus;
  return (uint32_t)(g ? g : 1);
}

namespace ckks {

// A named range around each C-ABI call and each server job, for profilers that record
// markers (rocprofv3 --marker-trace); without one attached a range costs two calls.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// Records a message for ckks_last_error() (thread-local) and returns `code`.
int api_fail(int code, const char *fmt, ...);

// Per-call device scratch (cache metadata, product scratch, tile buffers): the context
// keeps one buffer per stream, grown when a call needs more, and calls on a stream reuse
// it in stream order.  The lease holds the context's workspace lock for the call (the
// enqueue only) and records the buffer's event when the call returns, which orders the
// buffer's next use after this call's work even if a different stream gets the same
// handle later.  Growth waits for the old buffer's last use before freeing it.  (Scratch
// from a stream-ordered pool, freed after each call, made the next call on the same
// stream wait on the host until the device had reached that free.)
class WsLease {
 public:
  WsLease(ckks_ctx *c, hipStream_t st) : c_(c), st_(st), lk_(c->ws_mu) {}
  ~WsLease() {
    if (w_) (void)hipEventRecord(w_->last, st_);
  }
  hipError_t get(uint64_t bytes, void **out);
  WsLease(const WsLease &) = delete;
  WsLease &operator=(const WsLease &) = delete;

 private:
  ckks_ctx *c_;
  hipStream_t st_;
  std::unique_lock<std::mutex> lk_;
  StreamWorkspace *w_ = nullptr;
};
// Frees every stream's scratch buffer (the device must be idle).
void ws_free_all(ckks_ctx *c);

// Mean-filter multiplier: 1/k^2 as rint(q_{level-1} / k^2) per limb, and the scale after it.
int filter_multiplier(const ckks_ctx *c, uint32_t level, double scale, uint32_t k, std::vector<uint64_t> &K,
                      double *new_scale);

// Cached encryption of n pixels with caller-provided scratch (cached_ws_bytes(cache, n)
// bytes of device memory, 256-byte aligned): value caches gather hits and plain-encrypt
// misses, radix caches combine their entries.
uint64_t cached_ws_bytes(const ckks_cache *cache, uint64_t n);
// With `concurrent`, a value cache's misses run on the context's auxiliary stream beside the
// hit gather (forked from and joined back into `stream` by events).
hipError_t encrypt_cached_ws(const ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *px, uint64_t n,
                             uint64_t seed0, uint64_t seed1, uint64_t first_index, uint64_t *out, void *ws,
                             hipStream_t stream, bool concurrent);

// Number of fresh-encryption error terms a ciphertext of this cache kind carries (1 for
// plain encryption, cache == NULL).
double encryption_terms(const ckks_cache *cache);
// True when limb 0 alone decodes exactly every ciphertext that encrypts a slot-0 value of
// magnitude at most value_bound at the context's scale with `terms` fresh error terms,
// optionally after one k x k mean filter: a worst-case bound on the decrypted
// coefficients (message, errors bounded by the Gaussian tail cut, rescale rounding) stays
// below q_0/2.  Internal pipelines whose inputs are pixels use it to decode one limb.
bool limb0_decode_exact(const ckks_ctx *c, double value_bound, double terms, bool filtered);

// Row tiles of an image job (pipeline.cpp): bytes of one tile's buffers (encrypted rows with
// k/2 halo rows, filtered rows, cache metadata), the largest tile height within a byte
// budget (0 = the whole image), and encrypt -> k x k filter (k = 0: none) -> decrypt of
// the image tile by tile on one stream with those buffers at `mem`.
uint64_t tile_ws_bytes(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t k,
                       uint32_t tile_rows);
uint32_t tile_rows_for(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t k,
                       uint64_t budget);
hipError_t run_tiles(const ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint32_t H, uint32_t W,
                     uint64_t seed0, uint64_t seed1, uint64_t first_index, uint32_t k, uint32_t tile_rows,
                     const uint64_t *K, double out_scale, int dec_limbs, double *d_out, void *mem, hipStream_t st);

// Launchers (return a hipError_t; enqueue on `stream`).
// misses = false: the cache holds every value (VALUE_FULL), so only hits occur; the kernel
// is then compiled without the encryption path (decryption-sized LDS and registers) and
// uses the decryption's NTT width.
hipError_t launch_cached_fused(const ckks_ctx *c, const FusedJob &job, bool misses, hipStream_t stream);
hipError_t launch_keygen(const ckks_ctx *c, uint64_t seed0, uint64_t seed1, hipStream_t stream);
hipError_t launch_keys_prepare(const ckks_ctx *c, hipStream_t stream);
hipError_t launch_encrypt(const ckks_ctx *c, const EncJob &job, uint64_t grid, hipStream_t stream);
// limbs = 1: decode the centered residue of limb 0; limbs = 2 (level >= 2): decode the
// centered CRT lift of limbs 0 and 1.  max_grid (0 = no bound): at most this many
// workgroups, each taking every max_grid-th ciphertext.
hipError_t launch_decrypt(const ckks_ctx *c, const uint64_t *cts, uint64_t n, int level, double scale, double *out,
                          int limbs, hipStream_t stream, uint64_t max_grid = 0);
// Key-switching keys of s^2 (grid: digits x primes), then their NTT-domain copies.
hipError_t launch_relin_keygen(const ckks_ctx *c, uint64_t seed0, uint64_t seed1, hipStream_t stream);
hipError_t launch_relin_prepare(const ckks_ctx *c, hipStream_t stream);
// Relinearized products out = a * b of n ciphertext pairs at `level`; the kernel runs
// min(n, kMulGroups) workgroups and scratch holds (2 level + 2) * N words for each.
constexpr uint64_t kMulGroups = 2048;
inline uint64_t mul_scratch_words(uint64_t n, int level, int N) {
  return (n < kMulGroups ? n : kMulGroups) * (uint64_t)(2 * level + 2) * (uint64_t)N;
}
hipError_t launch_mul(const ckks_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n, int level,
                      uint64_t *scratch, hipStream_t stream);

hipError_t launch_add_sub(const ckks_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n,
                          int level, bool sub, hipStream_t stream);
hipError_t launch_mul_const(const ckks_ctx *c, const uint64_t *a, uint64_t *out, uint64_t n, int level,
                            const uint64_t *K, hipStream_t stream);
hipError_t launch_add_const(const ckks_ctx *c, uint64_t *a, uint64_t n, int level, double scale, const double *d_b,
                            double b, hipStream_t stream);
hipError_t launch_rescale(const ckks_ctx *c, const uint64_t *a, uint64_t *out, uint64_t n, int level,
                          hipStream_t stream);
// k x k mean filter of an H x W image of ciphertexts, output rows [y0, y1) (out holds
// y1 - y0 rows); K = the per-limb multiplier rint(q_last / k^2) mod q_i.  Image row y is
// read from row y mod ring_rows of `in` (0: ring_rows = H, `in` holds the whole image).
hipError_t launch_mean_filter(const ckks_ctx *c, const uint64_t *in, uint64_t *out, uint32_t H, uint32_t W,
                              uint32_t y0, uint32_t y1, uint32_t k, int level, const uint64_t *K, hipStream_t stream,
                              uint32_t ring_rows = 0);

// Fills n words with v (a kernel, so it can be captured in a graph).
hipError_t launch_fill_u32(uint32_t *p, uint32_t n, uint32_t v, hipStream_t stream);
hipError_t launch_histogram_topk(const ckks_ctx *c, const uint8_t *px, uint64_t n, uint32_t topk, uint32_t *hist,
                                 ckks_cache *cache, hipStream_t stream);
// Value-cache metadata for n pixels: meta[t], the miss list, and the hit list grouped by
// pool member.  counters = [miss count, hit count, per-member counts (pool entries)].
hipError_t launch_value_meta(const ckks_ctx *c, const ckks_cache *cache, const uint8_t *px, uint64_t n,
                             uint64_t first_index, uint64_t seed0, uint64_t seed1, uint32_t *meta,
                             uint32_t *miss_list, uint32_t *counters, uint32_t *hits, hipStream_t stream);
// max_grid (0 = no bound): at most this many workgroups, walking the hit list persistently.
hipError_t launch_value_gather(const ckks_ctx *c, const ckks_cache *cache, const uint32_t *meta,
                               uint32_t *counters, const uint32_t *hits, uint64_t n, uint64_t *out,
                               const EncJob *bright, hipStream_t stream, uint64_t max_grid = 0);
hipError_t launch_radix_meta(const ckks_ctx *c, const ckks_cache *cache, const uint8_t *px, uint64_t n,
                             uint64_t first_index, uint64_t seed0, uint64_t seed1, int16_t *meta, uint32_t *bad,
                             hipStream_t stream);
hipError_t launch_radix_gather(const ckks_ctx *c, const ckks_cache *cache, const int16_t *meta, uint64_t n,
                               uint64_t *out, hipStream_t stream);

// Largest grid the persistent (list-driven) encryption uses.
constexpr uint64_t kListGrid = 8192;

// The dispatcher hands workgroup b to XCD b mod 8.  This maps the hardware index to a
// logical one so that each XCD receives a contiguous range of logical workgroups (a
// bijection on [0, nb) for any nb): neighbouring logical workgroups, which read
// neighbouring data, then share one XCD's L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_logical_block(uint32_t b, uint32_t nb) {
  const uint32_t x = b % kXcds, i = b / kXcds;
  const uint32_t per = nb / kXcds, rem = nb % kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

// Dynamic work claiming for persistent kernels whose items are ordered for cache locality
// (the bucketed hit list): the item range [0, total) is cut into one contiguous region per
// XCD; the workgroups of XCD x take items of region x in order from an atomic cursor, then
// help with the other regions in turn.  All workgroups of an XCD thus work on neighbouring
// items at any time, whatever their speeds, and share that XCD's L2; a static stride
// would let them drift apart over the list.  cursor[kXcds] must start at zero.  Returns
// the next item of this workgroup, or `total` when there is none left; `region` keeps its
// state (start at 0).  Contains barriers: every thread of the workgroup must call it.
__device__ __forceinline__ uint64_t xcd_claim(uint32_t *cursor, uint64_t total, uint32_t &region, uint64_t *slot) {
  const uint32_t home = blockIdx.x % kXcds;
  for (; region < kXcds; region++) {
    const uint32_t x = (home + region) % kXcds;
    const uint64_t lo = total * x / kXcds, hi = total * (x + 1) / kXcds;
    __syncthreads();
    if (threadIdx.x == 0) *slot = lo + atomicAdd(&cursor[x], 1u);
    __syncthreads();
    const uint64_t i = *slot;
    if (i < hi) return i;
  }
  return total;
}

// 16-byte vector of two residues, for non-temporal stores of ciphertext rows that are not
// read again by the same kernel (they would otherwise evict cache tables from L2/MALL).
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

}  // namespace ckks
