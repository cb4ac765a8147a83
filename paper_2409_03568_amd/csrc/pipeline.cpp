// Streamed image pipeline: encrypt -> k x k mean filter -> decrypt over row tiles.
//
// One stream (the default, also the server's job runner): the encrypted rows live in a
// ring of T + 2R rows (tile rows T, filter radius R = k/2); image row y sits in ring row
// y mod (T + 2R).  Tile t encrypts only the rows it adds to the ring -- rows
// [r1 - T + R, r1 + R) of the image for output rows [r0, r1), the first tile also its
// upper halo -- so every pixel is encrypted once, and filters its output rows straight
// from the ring; the rows it overwrites are those no later tile reads.  The ciphertexts
// equal the whole-image ones because every ciphertext depends only on its pixel and its
// global Philox index (Sec. 3.3 and the counter-based sampling of the encryption).
//
// Three streams: the stages on their own streams, so that tile t+1 can be encrypted while
// tile t is filtered and tile t-1 decrypted.  Tile t's input buffer holds the encrypted
// rows [r0 - R, r1 + R) clipped to the image: the halo rows are encrypted again for each
// tile instead of being exchanged.  The filter computes only the tile's own output rows,
// whose windows lie inside the buffer (at the image border the buffer ends where the
// image does, so the clamp-edge rule applies unchanged).  Two buffers per stage alternate
// between tiles; events order each buffer's reuse after its readers.  Every launch of the
// three stages fills the device by itself, so the overlap gains nothing measurable and the
// recomputed halos cost their share: one stream is the faster mode.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.hpp"

using namespace ckks;

namespace {

struct Events {
  std::vector<hipEvent_t> ev;
  ~Events() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipError_t make(size_t n) {
    ev.assign(n, nullptr);
    for (auto &e : ev) {
      const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
};

struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

uint64_t al(uint64_t x) { return (x + 255) / 256 * 256; }

// Byte sizes of one tile's buffers: encrypted rows (with halos), filtered rows, cache metadata.
struct TileSizes {
  uint32_t rows = 0, cap_rows = 0;
  uint64_t enc = 0, flt = 0, ws = 0;
};

TileSizes tile_sizes(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t k,
                     uint32_t tile_rows) {
  const uint32_t L = (uint32_t)ctx->prm.L, R = k / 2;
  TileSizes t;
  t.rows = tile_rows < H ? tile_rows : H;
  t.cap_rows = t.rows + 2 * R < H ? t.rows + 2 * R : H;
  t.enc = al((uint64_t)t.cap_rows * W * ckks_ct_bytes(ctx, L));
  t.flt = k ? al((uint64_t)t.rows * W * ckks_ct_bytes(ctx, L - 1)) : 0;
  t.ws = cache ? al(cached_ws_bytes(cache, (uint64_t)t.cap_rows * W)) : 0;
  return t;
}

}  // namespace

namespace ckks {

uint64_t tile_ws_bytes(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t k,
                       uint32_t tile_rows) {
  const TileSizes t = tile_sizes(ctx, cache, H, W, k, tile_rows);
  return t.enc + t.flt + t.ws;
}

uint32_t tile_rows_for(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t k,
                       uint64_t budget) {
  if (!budget) return H;
  uint32_t lo = 1, hi = H;  // the largest row count whose buffers fit the budget (at least one row)
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo + 1) / 2;
    if (tile_ws_bytes(ctx, cache, H, W, k, mid) <= budget)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

hipError_t run_tiles(const ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint32_t H, uint32_t W,
                     uint64_t seed0, uint64_t seed1, uint64_t first_index, uint32_t k, uint32_t tile_rows,
                     const uint64_t *K, double out_scale, int dec_limbs, double *d_out, void *mem, hipStream_t st) {
  const uint32_t L = (uint32_t)ctx->prm.L, R = k / 2;
  const TileSizes ts = tile_sizes(ctx, cache, H, W, k, tile_rows);
  const uint32_t ring = ts.cap_rows;  // T + 2R rows, or the whole image
  const uint64_t row_words = (uint64_t)W * 2 * L * ctx->N;
  uint8_t *m = static_cast<uint8_t *>(mem);
  uint64_t *enc = reinterpret_cast<uint64_t *>(m), *flt = reinterpret_cast<uint64_t *>(m + ts.enc);
  void *ws = m + ts.enc + ts.flt;
  // image rows [a, b) into their ring rows (at most two contiguous runs)
  auto encrypt_rows = [&](uint32_t a, uint32_t b) {
    hipError_t e = hipSuccess;
    while (a < b && e == hipSuccess) {
      const uint32_t slot = a % ring, cnt = b - a < ring - slot ? b - a : ring - slot;
      const uint64_t n = (uint64_t)cnt * W, px0 = (uint64_t)a * W;
      uint64_t *out = enc + (uint64_t)slot * row_words;
      if (cache) {
        e = encrypt_cached_ws(ctx, cache, d_px + px0, n, seed0, seed1, first_index + px0, out, ws, st, true);
      } else {
        EncJob job;
        job.px = d_px + px0;
        job.n = n;
        job.first_index = first_index + px0;
        job.seed0 = seed0;
        job.seed1 = seed1;
        job.out = out;
        e = launch_encrypt(ctx, job, n < (1u << 24) ? n : (1u << 24), st);
      }
      a += cnt;
    }
    return e;
  };
  hipError_t e = hipSuccess;
  uint32_t ready = 0;  // image rows [0, ready) have been encrypted
  for (uint32_t r0 = 0; r0 < H && e == hipSuccess; r0 += ts.rows) {
    const uint32_t r1 = r0 + ts.rows < H ? r0 + ts.rows : H;
    const uint32_t need = r1 + R < H ? r1 + R : H;
    e = encrypt_rows(ready, need);
    ready = need;
    if (e != hipSuccess) break;
    if (k) {
      e = launch_mean_filter(ctx, enc, flt, H, W, r0, r1, k, (int)L, K, st, ring);
      if (e == hipSuccess)
        e = launch_decrypt(ctx, flt, (uint64_t)(r1 - r0) * W, (int)L - 1, out_scale, d_out + (uint64_t)r0 * W,
                           L - 1 >= 2 ? dec_limbs : 1, st);
    } else {  // R = 0: the tile's rows start a ring of T rows
      e = launch_decrypt(ctx, enc + (uint64_t)(r0 % ring) * row_words, (uint64_t)(r1 - r0) * W, (int)L, out_scale,
                         d_out + (uint64_t)r0 * W, L >= 2 ? dec_limbs : 1, st);
    }
  }
  return e;
}

}  // namespace ckks

extern "C" int ckks_image_pipeline(ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint32_t H,
                                   uint32_t W, const uint64_t seed[2], uint64_t first_index,
                                   const ckks_pipeline_config *cfg, double *d_out, void *stream) {
  TraceRange trace_range_("ckks_image_pipeline");
  if (!ctx || !cfg || !seed) return api_fail(CKKS_EINVAL, "ctx/cfg/seed is NULL");
  if (!ctx->has_keys) return api_fail(CKKS_ESTATE, "no keys on the context");
  if (cache && cache->ctx != ctx) return api_fail(CKKS_ECACHE, "cache belongs to another context");
  if (cache && cache->key_epoch != ctx->key_epoch)
    return api_fail(CKKS_ESTATE, "the cache was built under keys that have since been replaced");
  const uint32_t k = cfg->filter_k;
  if (k != 1 && k != 3 && k != 5 && k != 7) return api_fail(CKKS_EUNSUPPORTED, "filter_k must be 1, 3, 5 or 7");
  const uint32_t L = (uint32_t)ctx->prm.L;
  if (L < 2 || L > 8) return api_fail(CKKS_ELEVEL, "the mean filter needs 2..8 limbs");
  if (cfg->streams != 1 && cfg->streams != 3) return api_fail(CKKS_EINVAL, "streams must be 1 or 3");
  if (cfg->tile_rows < 1) return api_fail(CKKS_EINVAL, "tile_rows must be >= 1");
  if ((uint64_t)H * W == 0) return CKKS_OK;
  if (!d_px || !d_out) return api_fail(CKKS_EINVAL, "NULL buffer");
  if ((uint64_t)H * W > 0xFFFFFFFFull) return api_fail(CKKS_EINVAL, "at most 2^32-1 pixels");
  std::vector<uint64_t> K;
  double s1 = 0;
  int rc = filter_multiplier(ctx, L, ctx->scale, k, K, &s1);
  if (rc) return rc;
  const double out_scale = s1 / (double)ctx->prm.q[L - 1];
  // filtered pixels: limb 0 decodes exactly unless the parameters leave no room
  const int dec_limbs = limb0_decode_exact(ctx, 255.0, encryption_terms(cache), true) || L < 3 ? 1 : 2;
  DeviceScope g(ctx->device);
  hipStream_t user = reinterpret_cast<hipStream_t>(stream);
  const uint32_t R = k / 2, T = cfg->tile_rows < H ? cfg->tile_rows : H;
  const uint32_t ntiles = (H + T - 1) / T;
  const uint32_t cap_rows = T + 2 * R < H ? T + 2 * R : H;
  const int nbuf = cfg->streams == 3 ? 2 : 1;
  const uint64_t S_in = ckks_ct_bytes(ctx, L), S_out = ckks_ct_bytes(ctx, L - 1);
  const uint64_t enc_bytes = al((uint64_t)cap_rows * W * S_in), flt_bytes = al((uint64_t)T * W * S_out);
  const uint64_t ws_bytes = cache ? al(cached_ws_bytes(cache, (uint64_t)cap_rows * W)) : 0;
  hipStream_t E = user, F = user, D = user;
  if (nbuf == 2) {
    for (hipStream_t &st : ctx->pipe)
      if (!st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return api_fail(CKKS_EDEVICE, "pipeline stream creation failed");
    E = ctx->pipe[0];
    F = ctx->pipe[1];
    D = ctx->pipe[2];
  }
  uint8_t *mem = nullptr;
  if (nbuf == 1) {  // one stream: the tiles one after another
    const uint64_t total = tile_ws_bytes(ctx, cache, H, W, k, T);
    if (hipMallocFromPoolAsync(reinterpret_cast<void **>(&mem), total, ctx->pool, user) != hipSuccess)
      return api_fail(CKKS_ENOMEM, "pipeline buffers (%llu bytes)", (unsigned long long)total);
    const hipError_t e1 = run_tiles(ctx, cache, d_px, H, W, seed[0], seed[1], first_index, k, T, K.data(), out_scale,
                                    dec_limbs, d_out, mem, user);
    (void)hipFreeAsync(mem, user);
    if (e1 != hipSuccess) return api_fail(CKKS_EDEVICE, "image pipeline: %s", hipGetErrorString(e1));
    return CKKS_OK;
  }
  const uint64_t total = nbuf * (enc_bytes + flt_bytes) + ws_bytes;
  if (hipMallocFromPoolAsync(reinterpret_cast<void **>(&mem), total, ctx->pool, user) != hipSuccess)
    return api_fail(CKKS_ENOMEM, "pipeline buffers (%llu bytes)", (unsigned long long)total);
  uint64_t *enc[2], *flt[2];
  for (int b = 0; b < nbuf; b++) {
    enc[b] = reinterpret_cast<uint64_t *>(mem + b * (enc_bytes + flt_bytes));
    flt[b] = reinterpret_cast<uint64_t *>(mem + b * (enc_bytes + flt_bytes) + enc_bytes);
  }
  void *ws = mem + nbuf * (enc_bytes + flt_bytes);
  // events: 0 start, then per buffer: encrypted, filtered, decrypted; 7..9 stage ends
  Events evs;
  hipError_t e = evs.make(10);
  auto ev_enc = [&](int b) { return evs.ev[1 + 3 * b]; };
  auto ev_flt = [&](int b) { return evs.ev[2 + 3 * b]; };
  auto ev_dec = [&](int b) { return evs.ev[3 + 3 * b]; };
  if (e == hipSuccess && nbuf == 2) {
    e = hipEventRecord(evs.ev[0], user);
    for (hipStream_t st : {E, F, D})
      if (e == hipSuccess) e = hipStreamWaitEvent(st, evs.ev[0], 0);
  }
  for (uint32_t t = 0; t < ntiles && e == hipSuccess; t++) {
    const int b = (int)(t % nbuf);
    const uint32_t r0 = t * T, r1 = r0 + T < H ? r0 + T : H;
    const uint32_t s0 = r0 >= R ? r0 - R : 0, s1r = r1 + R < H ? r1 + R : H;
    const uint64_t n_in = (uint64_t)(s1r - s0) * W, px0 = (uint64_t)s0 * W;
    if (nbuf == 2 && t >= 2) e = hipStreamWaitEvent(E, ev_flt(b), 0);  // filter of tile t-2 has read enc[b]
    if (e != hipSuccess) break;
    if (cache) {
      e = encrypt_cached_ws(ctx, cache, d_px + px0, n_in, seed[0], seed[1], first_index + px0, enc[b], ws, E, true);
    } else {
      EncJob job;
      job.px = d_px + px0;
      job.n = n_in;
      job.first_index = first_index + px0;
      job.seed0 = seed[0];
      job.seed1 = seed[1];
      job.out = enc[b];
      e = launch_encrypt(ctx, job, n_in < (1u << 24) ? n_in : (1u << 24), E);
    }
    if (e == hipSuccess && nbuf == 2) e = hipEventRecord(ev_enc(b), E);
    if (e == hipSuccess && nbuf == 2) e = hipStreamWaitEvent(F, ev_enc(b), 0);
    if (e == hipSuccess && nbuf == 2 && t >= 2) e = hipStreamWaitEvent(F, ev_dec(b), 0);  // flt[b] was decrypted
    if (e == hipSuccess)
      e = launch_mean_filter(ctx, enc[b], flt[b], s1r - s0, W, r0 - s0, r1 - s0, k, (int)L, K.data(), F);
    if (e == hipSuccess && nbuf == 2) e = hipEventRecord(ev_flt(b), F);
    if (e == hipSuccess && nbuf == 2) e = hipStreamWaitEvent(D, ev_flt(b), 0);
    if (e == hipSuccess)
      e = launch_decrypt(ctx, flt[b], (uint64_t)(r1 - r0) * W, (int)L - 1, out_scale, d_out + (uint64_t)r0 * W,
                         dec_limbs, D);
    if (e == hipSuccess && nbuf == 2) e = hipEventRecord(ev_dec(b), D);
  }
  if (nbuf == 2) {
    // the caller's stream continues after all three stages (also on error, before the buffers go)
    const hipStream_t stages[3] = {E, F, D};
    for (int i = 0; i < 3; i++) {
      (void)hipEventRecord(evs.ev[7 + i], stages[i]);
      (void)hipStreamWaitEvent(user, evs.ev[7 + i], 0);
    }
  }
  (void)hipFreeAsync(mem, user);
  if (e != hipSuccess) return api_fail(CKKS_EDEVICE, "image pipeline: %s", hipGetErrorString(e));
  return CKKS_OK;
}
