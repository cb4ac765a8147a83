// Batched images (flat pixel index space, ring buffer of ciphertext chunks, HIP graph
// replay) and the per-context autotuner of the NTT kernels' register blocking.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"
#include "tune_file.hpp"

using namespace ckks;

namespace {

#define BATCH_TRY(expr, what)                                                               \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return api_fail(CKKS_EDEVICE, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

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

struct RunKey {
  const uint8_t *px = nullptr;
  uint64_t n = 0;
  std::vector<uint64_t> seg_end;
  std::vector<double> seg_b;
  uint64_t seed[2] = {0, 0};
  uint64_t first_index = 0;
  double *out = nullptr;
  uint64_t *cts = nullptr;  // caller's ciphertext buffer, or NULL for the ring
  int dec_limbs = 1;
  bool operator==(const RunKey &o) const {
    return px == o.px && n == o.n && seg_end == o.seg_end && seg_b == o.seg_b && seed[0] == o.seed[0] &&
           seed[1] == o.seed[1] && first_index == o.first_index && out == o.out && cts == o.cts &&
           dec_limbs == o.dec_limbs;
  }
};

}  // namespace

struct ckks_batch_plan {
  ckks_ctx *ctx = nullptr;
  uint64_t key_epoch = 0;        // keys the plan was made under
  const ckks_cache *cache = nullptr;
  ckks_batch_config cfg{};
  uint64_t *ring = nullptr;      // [chunk][2][L][N]
  uint32_t *meta = nullptr;      // [px_cap] per-pixel cache metadata
  uint32_t *miss = nullptr;      // [px_cap]
  uint32_t *hits = nullptr;      // [px_cap]
  uint64_t px_cap = 0;
  uint32_t *counters = nullptr;  // value_counter_words(cache), or kCountersHead without a cache
  uint64_t *seg_end = nullptr;   // [seg_cap]
  double *seg_b = nullptr;       // [seg_cap]
  uint32_t seg_cap = 0;
  hipStream_t cap = nullptr;     // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool have_key = false;
  RunKey key;
};

namespace {

void drop_graph(ckks_batch_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->have_key = false;
}

void free_plan(ckks_batch_plan *p) {
  drop_graph(p);
  void *ptrs[] = {p->ring, p->meta, p->miss, p->hits, p->counters, p->seg_end, p->seg_b};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

// Enqueues one run on stream st (which may be capturing).
//
// When limb 0 decodes exactly (the usual case), the whole batch is one pass: with a cache,
// the metadata of every pixel is computed first, so that the hit list is ordered by pool
// member and cache slot over the whole batch and each (entry, pool member) pair is read
// from L2 for all its pixels at once; then one persistent launch assembles every
// ciphertext -- cache hit, or full encryption of a miss or of every pixel without a cache
// -- with the brightness fused in, writes it in full to a slot of the ring (of chunk_cts
// ciphertexts, or of cts_out) and decrypts it from the registers holding its limb-0 rows.
// With a cache that holds every value the launch has no encryption path: its workgroups
// need only the decryption's LDS and registers, so several share a CU and one streams
// while another transforms.  Otherwise the batch goes chunk by chunk through the ring,
// each chunk decrypted from it with the two-limb lift.
hipError_t enqueue_run(ckks_batch_plan *p, const RunKey &k, uint32_t n_seg, hipStream_t st) {
  const ckks_ctx *c = p->ctx;
  const uint64_t S = 2 * (uint64_t)c->prm.L * (uint64_t)c->N;
  const bool misses = !p->cache || p->cache->kind != CKKS_CACHE_VALUE_FULL;
  const bool whole = k.dec_limbs == 1;
  const uint64_t chunk = whole ? k.n : p->cfg.chunk_cts;
  for (uint64_t first = 0; first < k.n; first += chunk) {
    const uint64_t cnt = k.n - first < chunk ? k.n - first : chunk;
    FusedJob job;
    job.px = k.px + first;
    job.n = cnt;
    job.first_index = k.first_index + first;
    job.seed0 = k.seed[0];
    job.seed1 = k.seed[1];
    job.out = k.cts ? k.cts + first * S : p->ring;
    job.seg_end = p->seg_end;
    job.seg_b = p->seg_b;
    job.n_seg = n_seg;
    job.seg_base = first;
    job.bright_scale = ldexp(c->scale, 1 - c->prm.log_n);
    job.cursor = p->counters + 2;
    if (whole) {
      job.dec_out = k.out;
      job.inv_scale = 1.0 / c->scale;
      job.ring = k.cts ? 0 : p->cfg.chunk_cts;
    }
    hipError_t e = hipSuccess;
    if (p->cache) {
      e = launch_value_meta(c, p->cache, job.px, cnt, job.first_index, job.seed0, job.seed1, p->meta, p->miss,
                            p->counters, p->hits, st);
      job.counters = p->counters;
      job.miss_list = p->miss;
      job.hits = p->hits;
      job.meta = p->meta;
      job.entries = p->cache->entries;
      job.pool = p->cache->pool_cts;
    }
    if (e == hipSuccess) e = launch_cached_fused(c, job, misses, st);
    if (e == hipSuccess && !whole)
      e = launch_decrypt(c, job.out, cnt, c->prm.L, c->scale, k.out + first, k.dec_limbs, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int ckks_batch_plan_create(ckks_ctx *ctx, const ckks_cache *cache, const ckks_batch_config *cfg,
                           ckks_batch_plan **out) {
  if (!ctx || !cfg || !out) return api_fail(CKKS_EINVAL, "ctx/cfg/out is NULL");
  *out = nullptr;
  if (!ctx->has_keys) return api_fail(CKKS_ESTATE, "no keys on the context");
  if (cfg->chunk_cts < 1 || cfg->chunk_cts > 0xFFFFFFFFull) return api_fail(CKKS_EINVAL, "chunk_cts must be 1..2^32-1");
  if (cache && cache->ctx != ctx) return api_fail(CKKS_ECACHE, "cache belongs to another context");
  if (cache && cache->key_epoch != ctx->key_epoch)
    return api_fail(CKKS_ESTATE, "the cache was built under keys that have since been replaced");
  if (cache && cache->kind == CKKS_CACHE_RADIX) return api_fail(CKKS_EUNSUPPORTED, "batches take a value cache or none");
  DeviceScope g(ctx->device);
  ckks_batch_plan *p = new ckks_batch_plan;
  p->ctx = ctx;
  p->key_epoch = ctx->key_epoch;
  p->cache = cache;
  p->cfg = *cfg;
  const uint64_t chunk = cfg->chunk_cts;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->ring), chunk * ckks_ct_bytes(ctx, (uint32_t)ctx->prm.L));
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void **>(&p->counters),
                  (cache ? value_counter_words(cache) : kCountersHead) * sizeof(uint32_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_plan(p);
    return api_fail(CKKS_ENOMEM, "batch plan allocation: %s", hipGetErrorString(e));
  }
  *out = p;
  return CKKS_OK;
}

int ckks_batch_run(ckks_batch_plan *p, const uint8_t *d_px, uint64_t n, const uint64_t *host_seg_end,
                   const double *host_seg_b, uint32_t n_seg, const uint64_t seed[2], uint64_t first_index,
                   double *d_out, ckks_ct_batch *cts_out, void *stream) {
  TraceRange trace_range_("ckks_batch_run");
  if (!p || !seed) return api_fail(CKKS_EINVAL, "plan/seed is NULL");
  ckks_ctx *c = p->ctx;
  if (p->key_epoch != c->key_epoch) return api_fail(CKKS_ESTATE, "the keys were replaced after the plan was made");
  const uint32_t L = (uint32_t)c->prm.L;
  if (cts_out) {
    if (n && !cts_out->data) return api_fail(CKKS_EINVAL, "cts_out data is NULL");
    if (cts_out->count && (cts_out->level ? cts_out->level : L) != L)
      return api_fail(CKKS_ELEVEL, "cts_out must hold ciphertexts of level %u", L);
    if (cts_out->count && cts_out->count < n)
      return api_fail(CKKS_EINVAL, "cts_out holds %llu ciphertexts, the batch has %llu",
                      (unsigned long long)cts_out->count, (unsigned long long)n);
  }
  if (n == 0) return CKKS_OK;
  if (!d_px || !d_out || !host_seg_end || !host_seg_b) return api_fail(CKKS_EINVAL, "NULL buffer");
  if (n_seg < 1) return api_fail(CKKS_EINVAL, "need at least one image");
  const double bscale = ldexp(c->scale, 1 - c->prm.log_n);
  double bmax = 0.0;
  for (uint32_t i = 0; i < n_seg; i++) {
    if (i && host_seg_end[i] < host_seg_end[i - 1]) return api_fail(CKKS_EINVAL, "seg_end must be ascending");
    if (!(fabs(host_seg_b[i] * bscale) < 1125899906842624.0))  // 2^50
      return api_fail(CKKS_EINVAL, "brightness %g too large for the fused encoding", host_seg_b[i]);
    bmax = fmax(bmax, fabs(host_seg_b[i]));
  }
  if (host_seg_end[n_seg - 1] != n) return api_fail(CKKS_EINVAL, "last seg_end must equal n");
  if (cts_out) {
    cts_out->count = n;
    cts_out->level = L;
    cts_out->scale = c->scale;
  }
  DeviceScope g(c->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RunKey k;
  k.px = d_px;
  k.n = n;
  k.seg_end.assign(host_seg_end, host_seg_end + n_seg);
  k.seg_b.assign(host_seg_b, host_seg_b + n_seg);
  k.seed[0] = seed[0];
  k.seed[1] = seed[1];
  k.first_index = first_index;
  k.out = d_out;
  k.cts = cts_out ? cts_out->data : nullptr;
  // pixels plus brightness, one or two fresh error terms: limb 0 decodes exactly unless the
  // parameters leave no room (then the two-limb lift)
  k.dec_limbs = limb0_decode_exact(c, 255.0 + bmax, encryption_terms(p->cache), false) || L < 2 ? 1 : 2;
  const bool same = p->have_key && p->key == k;
  if (!same) {
    // the segment tables may still be read by work enqueued for an earlier run: let it
    // finish before they are replaced
    BATCH_TRY(hipStreamSynchronize(st), "stream synchronize");
    drop_graph(p);
    if (n_seg > p->seg_cap) {
      if (p->seg_end) (void)hipFree(p->seg_end);
      if (p->seg_b) (void)hipFree(p->seg_b);
      p->seg_end = nullptr;
      p->seg_b = nullptr;
      p->seg_cap = 0;
      BATCH_TRY(hipMalloc(reinterpret_cast<void **>(&p->seg_end), n_seg * sizeof(uint64_t)), "segment alloc");
      BATCH_TRY(hipMalloc(reinterpret_cast<void **>(&p->seg_b), n_seg * sizeof(double)), "segment alloc");
      p->seg_cap = n_seg;
    }
    BATCH_TRY(hipMemcpy(p->seg_end, host_seg_end, n_seg * sizeof(uint64_t), hipMemcpyHostToDevice), "segment upload");
    BATCH_TRY(hipMemcpy(p->seg_b, host_seg_b, n_seg * sizeof(double), hipMemcpyHostToDevice), "segment upload");
    // per-pixel cache metadata for the whole batch (or one chunk on the two-limb path)
    const uint64_t need = p->cache ? (k.dec_limbs == 1 ? n : std::min<uint64_t>(n, p->cfg.chunk_cts)) : 0;
    if (need > p->px_cap) {
      for (uint32_t **q : {&p->meta, &p->miss, &p->hits}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
      }
      p->px_cap = 0;
      for (uint32_t **q : {&p->meta, &p->miss, &p->hits})
        BATCH_TRY(hipMalloc(reinterpret_cast<void **>(q), need * sizeof(uint32_t)), "metadata alloc");
      p->px_cap = need;
    }
  }
  if (!p->cfg.use_graph || !same) {
    // eager launch: the first run with new arguments (and every run without graphs)
    BATCH_TRY(enqueue_run(p, k, n_seg, st), "batch launch");
    p->key = k;
    p->have_key = true;
    if (!p->cfg.use_graph) return CKKS_OK;
    // record the same sequence for the next runs with these arguments (capture does not execute it)
    BATCH_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    const hipError_t e = enqueue_run(p, k, n_seg, p->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(p->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      p->have_key = false;
      return api_fail(CKKS_EDEVICE, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    p->graph = graph;
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
      drop_graph(p);
      return api_fail(CKKS_EDEVICE, "graph instantiate failed");
    }
    return CKKS_OK;
  }
  BATCH_TRY(hipGraphLaunch(p->exec, st), "graph launch");
  return CKKS_OK;
}

void ckks_batch_plan_destroy(ckks_batch_plan *p) {
  if (!p) return;
  DeviceScope g(p->ctx->device);
  (void)hipDeviceSynchronize();
  free_plan(p);
}

int ckks_autotune(ckks_ctx *ctx, uint32_t trial_cts, ckks_tune_report *out) {
  TraceRange trace_range_("ckks_autotune");
  if (!ctx || !out) return api_fail(CKKS_EINVAL, "ctx/out is NULL");
  if (!ctx->has_keys) return api_fail(CKKS_ESTATE, "no keys on the context");
  if (trial_cts < 1 || trial_cts > (1u << 20)) return api_fail(CKKS_EINVAL, "trial_cts must be 1..2^20");
  DeviceScope g(ctx->device);
  const uint32_t L = (uint32_t)ctx->prm.L;
  uint8_t *px = nullptr;
  uint64_t *cts = nullptr, *gout = nullptr;
  double *dec = nullptr;
  uint64_t *prod = nullptr, *scratch = nullptr;
  uint32_t *meta = nullptr, *hits = nullptr, *counters = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&px), trial_cts);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&cts), (uint64_t)trial_cts * ckks_ct_bytes(ctx, L));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&gout), (uint64_t)trial_cts * ckks_ct_bytes(ctx, L));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&dec), (uint64_t)trial_cts * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&meta), (uint64_t)trial_cts * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&hits), (uint64_t)trial_cts * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&counters), kCountersHead * sizeof(uint32_t));
  if (e == hipSuccess && ctx->has_relin)
    e = hipMalloc(reinterpret_cast<void **>(&prod), (uint64_t)trial_cts * ckks_ct_bytes(ctx, L));
  if (e == hipSuccess && ctx->has_relin)
    e = hipMalloc(reinterpret_cast<void **>(&scratch), mul_scratch_words(trial_cts, (int)L, ctx->N) * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemset(px, 0x5a, trial_cts);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // Best of three timed runs after one warm-up; `before` runs untimed ahead of each.
  auto best_ms = [&](auto &&launch, auto &&before) {
    double best = INFINITY;
    for (int rep = 0; rep < 4 && e == hipSuccess; rep++) {
      float ms = 0.f;
      e = before();
      if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
      if (e == hipSuccess) e = launch();
      if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && rep) best = fmin(best, ms);
    }
    return best;
  };
  auto nothing = [] { return hipSuccess; };
  const int keep_enc = ctx->logr_enc, keep_dec = ctx->logr_dec, keep_mul = ctx->logr_mul;
  const int keep_row = ctx->row_wgs, keep_gather = ctx->gather_wgs;
  double enc_ms[3] = {INFINITY, INFINITY, INFINITY}, dec_ms[3] = {INFINITY, INFINITY, INFINITY};
  double mul_ms[3] = {INFINITY, INFINITY, INFINITY};
  for (int w = 0; w < 3 && e == hipSuccess; w++) {
    if ((ctx->N >> (3 + w)) > 1024) continue;  // more threads than a workgroup holds
    ctx->logr_enc = ctx->logr_dec = ctx->logr_mul = 3 + w;
    EncJob job;
    job.px = px;
    job.n = trial_cts;
    job.seed0 = 0x7u;
    job.seed1 = 0x70u;
    job.out = cts;
    enc_ms[w] = best_ms([&] { return launch_encrypt(ctx, job, trial_cts, nullptr); }, nothing);
    dec_ms[w] = best_ms([&] { return launch_decrypt(ctx, cts, trial_cts, (int)L, ctx->scale, dec, 1, nullptr); },
                        nothing);
    if (prod)
      mul_ms[w] = best_ms([&] { return launch_mul(ctx, cts, cts, prod, trial_cts, (int)L, scratch, nullptr); },
                          nothing);
  }
  int be = 0, bd = 0, bm = 0;
  for (int w = 1; w < 3; w++) {
    if (enc_ms[w] < enc_ms[be]) be = w;
    if (dec_ms[w] < dec_ms[bd]) bd = w;
    if (mul_ms[w] < mul_ms[bm]) bm = w;
  }
  ctx->logr_enc = 3 + be;
  ctx->logr_dec = 3 + bd;
  ctx->logr_mul = prod ? 3 + bm : keep_mul;
  // Launch shapes.  The row-wise kernels are timed on the addition of the trial
  // ciphertexts; the gather on a synthetic all-hit job: 16 entries and 2 pool members
  // taken from the trial ciphertexts (canonical residues), every ciphertext a hit.
  static const int kRow[5] = {0, 2, 4, 8, 16}, kGather[5] = {2, 4, 8, 16, 32};
  double row_ms[5], gather_ms[5];
  for (int i = 0; i < 5; i++) {
    ctx->row_wgs = kRow[i];
    row_ms[i] = best_ms([&] { return launch_add_sub(ctx, cts, cts, gout, trial_cts, (int)L, false, nullptr); }, nothing);
  }
  const uint32_t n_ent = std::min<uint32_t>(16, trial_cts), n_pool = std::min<uint32_t>(2, trial_cts);
  std::vector<uint32_t> h_meta(trial_cts), h_hits(trial_cts), h_counters(kCountersHead, 0);
  for (uint32_t i = 0; i < trial_cts; i++) {
    h_meta[i] = ((i % n_pool) << 16) | (1 + (i * 7) % n_ent);
    h_hits[i] = i;
  }
  h_counters[1] = trial_cts;
  if (e == hipSuccess) e = hipMemcpy(meta, h_meta.data(), trial_cts * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(hits, h_hits.data(), trial_cts * sizeof(uint32_t), hipMemcpyHostToDevice);
  ckks_cache fake;
  fake.ctx = ctx;
  fake.entries = cts;
  fake.pool_cts = cts;
  for (int i = 0; i < 5; i++) {
    ctx->gather_wgs = kGather[i];
    gather_ms[i] = best_ms(
        [&] {
          return launch_value_gather(ctx, &fake, meta, counters, hits, trial_cts, gout, nullptr, nullptr, 0);
        },
        [&] { return hipMemcpy(counters, h_counters.data(), kCountersHead * sizeof(uint32_t), hipMemcpyHostToDevice); });
  }
  int br = 0, bg = 0;
  for (int i = 1; i < 5; i++) {
    if (row_ms[i] < row_ms[br]) br = i;
    if (gather_ms[i] < gather_ms[bg]) bg = i;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void *ptr : {(void *)px, (void *)cts, (void *)gout, (void *)dec, (void *)prod, (void *)scratch, (void *)meta,
                    (void *)hits, (void *)counters})
    if (ptr) (void)hipFree(ptr);
  if (e != hipSuccess) {
    ctx->logr_enc = keep_enc;
    ctx->logr_dec = keep_dec;
    ctx->logr_mul = keep_mul;
    ctx->row_wgs = keep_row;
    ctx->gather_wgs = keep_gather;
    return api_fail(CKKS_EDEVICE, "autotune: %s", hipGetErrorString(e));
  }
  ctx->row_wgs = kRow[br];
  ctx->gather_wgs = kGather[bg];
  out->encrypt_width = 1u << ctx->logr_enc;
  out->decrypt_width = 1u << ctx->logr_dec;
  out->trial_cts = trial_cts;
  out->mul_width = prod ? 1u << ctx->logr_mul : 0;
  for (int w = 0; w < 3; w++) {
    out->encrypt_ms[w] = enc_ms[w];
    out->decrypt_ms[w] = dec_ms[w];
    out->mul_ms[w] = mul_ms[w];
  }
  out->row_wgs_per_cu = (uint32_t)ctx->row_wgs;
  out->gather_wgs_per_cu = (uint32_t)ctx->gather_wgs;
  for (int i = 0; i < 5; i++) {
    out->row_ms[i] = row_ms[i];
    out->gather_ms[i] = gather_ms[i];
  }
  return CKKS_OK;
}

static int tune_key(const ckks_ctx *ctx, tune::Key *k) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return api_fail(CKKS_EDEVICE, "device properties");
  k->arch = prop.gcnArchName;
  for (char &c : k->arch)
    if (c == ' ' || c == '\t') c = '_';
  if (k->arch.empty()) k->arch = "unknown";
  k->cus = ctx->num_cus;
  k->log_n = ctx->prm.log_n;
  k->L = ctx->prm.L;
  return CKKS_OK;
}

int ckks_tune_save(const ckks_ctx *ctx, const char *path) {
  if (!ctx || !path) return api_fail(CKKS_EINVAL, "ctx/path is NULL");
  tune::Key k;
  if (int rc = tune_key(ctx, &k)) return rc;
  tune::Values v;
  v.enc = 1 << ctx->logr_enc;
  v.dec = 1 << ctx->logr_dec;
  v.mul = 1 << ctx->logr_mul;
  v.row = ctx->row_wgs;
  v.gather = ctx->gather_wgs;
  if (int err = tune::store(path, k, v)) return api_fail(CKKS_EIO, "tune file %s: %s", path, strerror(err));
  return CKKS_OK;
}

int ckks_tune_load(ckks_ctx *ctx, const char *path, int *found) {
  if (!ctx || !path || !found) return api_fail(CKKS_EINVAL, "ctx/path/found is NULL");
  *found = 0;
  tune::Key k;
  if (int rc = tune_key(ctx, &k)) return rc;
  tune::Values v;
  bool hit = false;
  if (int err = tune::lookup(path, k, &v, &hit)) return api_fail(CKKS_EIO, "tune file %s: %s", path, strerror(err));
  if (!hit) return CKKS_OK;
  if (!tune::valid(v, ctx->prm.log_n)) return api_fail(CKKS_EINVAL, "tune file %s: unsupported settings", path);
  auto logr = [](int w) { return w == 8 ? 3 : w == 16 ? 4 : 5; };
  ctx->logr_enc = logr(v.enc);
  ctx->logr_dec = logr(v.dec);
  ctx->logr_mul = logr(v.mul);
  ctx->row_wgs = v.row;
  ctx->gather_wgs = v.gather;
  *found = 1;
  return CKKS_OK;
}

}  // extern "C"
