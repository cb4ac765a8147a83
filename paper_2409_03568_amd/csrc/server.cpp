// Serving runtime: image jobs (encrypt -> mean filter -> decrypt) admitted in arrival
// order into an arena of device memory and run concurrently, one HIP stream per slot.
//
// A dispatcher thread owns all device work of the server.  Under the server mutex it
//   1. retires slots whose last event has completed (copies the decrypted values to the
//      caller's buffer, returns the job's arena range and slot),
//   2. starts queued jobs while the oldest one fits, then younger ones that fit within the
//      waiting jobs' bypass budgets (Admission in arena.hpp), and
//   3. sleeps until a submission arrives or, while jobs run, for a short poll interval.
// Submissions only queue a copy of the pixels, so callers never wait for the GPU.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "arena.hpp"
#include "internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint64_t kAlign = 256;
constexpr auto kPollInterval = std::chrono::microseconds(50);

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Job {
  uint64_t id = 0;
  int forced_status = 0;  // failure injected by ckks_server_inject_failure (0 = none)
  uint32_t H = 0, W = 0;
  uint64_t n = 0;
  uint64_t seed[2] = {0, 0};
  uint64_t first_index = 0;
  std::vector<uint8_t> px;
  double *host_out = nullptr;
  uint64_t bytes = 0;
  double t_submit = 0, t_admit = 0;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint8_t *pin_px = nullptr;
  double *pin_out = nullptr;
  uint64_t pin_cap = 0;
  bool busy = false;
  Job job;
  uint64_t offset = 0;
  int status = CKKS_OK;
};

}  // namespace

struct ckks_server {
  ckks_ctx *ctx = nullptr;
  uint64_t key_epoch = 0;  // keys the server was created under
  int dec_limbs = 1;       // limbs decoded by decryption (see limb0_decode_exact)
  std::vector<uint64_t> K;  // the filter's multiplier rint(q_{L-1} / k^2) per limb
  double out_scale = 0.0;   // scale of the decrypted values
  ckks_server_config cfg{};
  uint8_t *arena = nullptr;
  ckks::rt::Admission adm;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<uint64_t, Job> queued;
  std::deque<ckks_job_result> results;
  std::thread th;
  bool stop = false;
  uint64_t next_id = 1;
  Clock::time_point t0;
  ckks_server_stats st{};

  ckks_server(uint64_t budget, uint32_t nslots, uint32_t max_bypass)
      : adm(budget, nslots, kAlign, max_bypass), slots(nslots) {}
  double now_us() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
  uint32_t busy_slots() const {
    uint32_t b = 0;
    for (const Slot &s : slots) b += s.busy ? 1u : 0u;
    return b;
  }
};

namespace {

// Arena bytes of a job: its pixels and decrypted values, and the buffers of one row tile
// (tile_bytes caps those; 0 = the whole image in one tile).
uint64_t job_bytes_of(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t k,
                      uint64_t tile_bytes) {
  const uint64_t n = (uint64_t)H * W;
  const uint32_t rows = ckks::tile_rows_for(ctx, cache, H, W, k, tile_bytes);
  return align_up(n) + align_up(8 * n) + ckks::tile_ws_bytes(ctx, cache, H, W, k, rows);
}

uint64_t job_bytes(const ckks_server *s, uint32_t H, uint32_t W) {
  return job_bytes_of(s->ctx, s->cfg.cache, H, W, s->cfg.filter_k, s->cfg.tile_bytes);
}

hipError_t ensure_pinned(Slot &sl, uint64_t n) {
  if (n <= sl.pin_cap) return hipSuccess;
  if (sl.pin_px) (void)hipHostFree(sl.pin_px);
  if (sl.pin_out) (void)hipHostFree(sl.pin_out);
  sl.pin_px = nullptr;
  sl.pin_out = nullptr;
  sl.pin_cap = 0;
  hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&sl.pin_px), n, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.pin_out), n * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) sl.pin_cap = n;
  return e;
}

// Enqueues the whole job on the slot's stream -- pixels in, then encrypt -> filter -> decrypt
// tile by tile in the job's arena range, decrypted values out; returns the status of the
// first failing step (or the injected failure, before any device work).
int launch_job(ckks_server *s, Slot &sl) {
  ckks::TraceRange trace_range_("server job");
  const Job &j = sl.job;
  if (j.forced_status) return j.forced_status;
  ckks_ctx *ctx = s->ctx;
  if (ensure_pinned(sl, j.n) != hipSuccess) return CKKS_ENOMEM;
  memcpy(sl.pin_px, j.px.data(), j.n);
  uint8_t *base = s->arena + sl.offset;
  uint8_t *d_px = base;
  double *d_out = reinterpret_cast<double *>(base + align_up(j.n));
  void *tiles = base + align_up(j.n) + align_up(8 * j.n);
  const uint32_t rows = ckks::tile_rows_for(ctx, s->cfg.cache, j.H, j.W, s->cfg.filter_k, s->cfg.tile_bytes);
  if (hipEventRecord(sl.ev0, sl.st) != hipSuccess) return CKKS_EDEVICE;
  if (hipMemcpyAsync(d_px, sl.pin_px, j.n, hipMemcpyHostToDevice, sl.st) != hipSuccess) return CKKS_EDEVICE;
  if (ckks::run_tiles(ctx, s->cfg.cache, d_px, j.H, j.W, j.seed[0], j.seed[1], j.first_index, s->cfg.filter_k, rows,
                      s->K.data(), s->out_scale, s->dec_limbs, d_out, tiles, sl.st) != hipSuccess)
    return CKKS_EDEVICE;
  if (hipMemcpyAsync(sl.pin_out, d_out, j.n * sizeof(double), hipMemcpyDeviceToHost, sl.st) != hipSuccess)
    return CKKS_EDEVICE;
  return CKKS_OK;
}

void retire(ckks_server *s, Slot &sl, int status) {
  ckks_job_result r{};
  r.job_id = sl.job.id;
  r.height = sl.job.H;
  r.width = sl.job.W;
  r.t_submit_us = sl.job.t_submit;
  r.t_admit_us = sl.job.t_admit;
  r.status = status;
  if (status == CKKS_OK) {
    memcpy(sl.job.host_out, sl.pin_out, sl.job.n * sizeof(double));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sl.ev0, sl.ev1) == hipSuccess) r.gpu_ms = ms;
    s->st.completed++;
  } else {
    s->st.failed++;
  }
  r.t_done_us = s->now_us();
  s->results.push_back(r);
  s->adm.finish(sl.offset);
  sl.busy = false;
  sl.job = Job{};
}

void dispatcher(ckks_server *s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool retired = false;
    for (Slot &sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.ev1);
      if (q == hipErrorNotReady) continue;
      retire(s, sl, q == hipSuccess ? sl.status : CKKS_EDEVICE);
      retired = true;
    }
    std::vector<ckks::rt::Admitted> started;
    if (!s->stop) s->adm.admit(started);
    for (const auto &a : started) {
      Slot *sl = nullptr;
      for (Slot &c : s->slots)
        if (!c.busy) {
          sl = &c;
          break;
        }
      auto it = s->queued.find(a.id);
      sl->job = std::move(it->second);
      s->queued.erase(it);
      sl->offset = a.offset;
      sl->busy = true;
      sl->job.t_admit = s->now_us();
      sl->status = launch_job(s, *sl);
      if (hipEventRecord(sl->ev1, sl->st) != hipSuccess) {
        // nothing will signal this slot: wait for what was enqueued, then retire it
        (void)hipStreamSynchronize(sl->st);
        retire(s, *sl, sl->status ? sl->status : CKKS_EDEVICE);
        retired = true;
      }
    }
    const uint32_t busy = s->busy_slots();
    const uint64_t used = s->adm.arena().used();
    if (used > s->st.peak_inflight_bytes) s->st.peak_inflight_bytes = used;
    if (busy > s->st.peak_inflight_jobs) s->st.peak_inflight_jobs = busy;
    if (retired) s->cv_done.notify_all();
    if (s->stop && busy == 0) break;
    if (busy)
      s->cv_work.wait_for(lk, kPollInterval);
    else
      s->cv_work.wait(lk, [s] { return s->stop || s->adm.queued() > 0; });
  }
  s->cv_done.notify_all();
}

void free_server(ckks_server *s) {
  for (Slot &sl : s->slots) {
    if (sl.ev0) (void)hipEventDestroy(sl.ev0);
    if (sl.ev1) (void)hipEventDestroy(sl.ev1);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.pin_px) (void)hipHostFree(sl.pin_px);
    if (sl.pin_out) (void)hipHostFree(sl.pin_out);
  }
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

}  // namespace

extern "C" {

int ckks_server_create(ckks_ctx *ctx, const ckks_server_config *cfg, ckks_server **out) {
  if (!ctx || !cfg || !out) return ckks::api_fail(CKKS_EINVAL, "ctx/cfg/out is NULL");
  *out = nullptr;
  if (!ctx->has_keys) return ckks::api_fail(CKKS_ESTATE, "no keys on the context");
  if (cfg->max_inflight < 1 || cfg->max_inflight > 64) return ckks::api_fail(CKKS_EINVAL, "max_inflight must be 1..64");
  const uint32_t k = cfg->filter_k;
  if (k != 0 && k != 1 && k != 3 && k != 5 && k != 7) return ckks::api_fail(CKKS_EUNSUPPORTED, "filter_k must be 0, 1, 3, 5 or 7");
  if (k && (ctx->prm.L < 2 || ctx->prm.L > 8)) return ckks::api_fail(CKKS_ELEVEL, "the mean filter needs 2..8 limbs");
  if (cfg->cache && cfg->cache->ctx != ctx) return ckks::api_fail(CKKS_ECACHE, "cache belongs to another context");
  if (cfg->cache && cfg->cache->key_epoch != ctx->key_epoch)
    return ckks::api_fail(CKKS_ESTATE, "the cache was built under keys that have since been replaced");
  if (cfg->hbm_budget_bytes < kAlign) return ckks::api_fail(CKKS_EINVAL, "hbm_budget_bytes too small");
  if (cfg->max_bypass > 1024) return ckks::api_fail(CKKS_EINVAL, "max_bypass must be 0..1024");
  ckks_server *s = new ckks_server(cfg->hbm_budget_bytes, cfg->max_inflight, cfg->max_bypass);
  s->ctx = ctx;
  s->key_epoch = ctx->key_epoch;
  s->dec_limbs = ckks::limb0_decode_exact(ctx, 255.0, ckks::encryption_terms(cfg->cache), cfg->filter_k != 0) ? 1 : 2;
  s->cfg = *cfg;
  s->out_scale = ctx->scale;
  if (k) {
    double s1 = 0;
    const int rc = ckks::filter_multiplier(ctx, (uint32_t)ctx->prm.L, ctx->scale, k, s->K, &s1);
    if (rc) {
      delete s;
      return rc;
    }
    s->out_scale = s1 / (double)ctx->prm.q[ctx->prm.L - 1];
  }
  s->t0 = Clock::now();
  int dev_prev = -1;
  (void)hipGetDevice(&dev_prev);
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&s->arena), s->adm.arena().capacity());
  for (Slot &sl : s->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sl.ev0);
    if (e == hipSuccess) e = hipEventCreate(&sl.ev1);
    if (e == hipSuccess && cfg->max_job_pixels) e = ensure_pinned(sl, cfg->max_job_pixels);
  }
  if (dev_prev >= 0) (void)hipSetDevice(dev_prev);
  if (e != hipSuccess) {
    free_server(s);
    return ckks::api_fail(CKKS_ENOMEM, "server allocation: %s", hipGetErrorString(e));
  }
  s->st.arena_bytes = s->adm.arena().capacity();
  s->th = std::thread(dispatcher, s);
  *out = s;
  return CKKS_OK;
}

int ckks_server_submit(ckks_server *s, const uint8_t *host_px, uint32_t H, uint32_t W, const uint64_t job_seed[2],
                       uint64_t first_index, double *host_out, uint64_t *job_id) {
  if (!s || !host_px || !host_out || !job_seed) return ckks::api_fail(CKKS_EINVAL, "NULL argument");
  if (s->key_epoch != s->ctx->key_epoch)
    return ckks::api_fail(CKKS_ESTATE, "the keys were replaced after the server was created");
  const uint64_t n = (uint64_t)H * W;
  if (n == 0 || n > 0xFFFFFFFFull) return ckks::api_fail(CKKS_EINVAL, "H*W must be in 1..2^32-1");
  const uint64_t bytes = job_bytes(s, H, W);
  if (!s->adm.fits_ever(bytes))
    return ckks::api_fail(CKKS_ENOMEM_BUDGET, "job needs %llu bytes, budget is %llu", (unsigned long long)bytes,
                          (unsigned long long)s->adm.arena().capacity());
  Job j;
  j.H = H;
  j.W = W;
  j.n = n;
  j.seed[0] = job_seed[0];
  j.seed[1] = job_seed[1];
  j.first_index = first_index;
  j.px.assign(host_px, host_px + n);
  j.host_out = host_out;
  j.bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return ckks::api_fail(CKKS_ESTATE, "server is stopping");
    j.id = s->next_id++;
    j.t_submit = s->now_us();
    if (job_id) *job_id = j.id;
    s->adm.push(j.id, bytes);
    s->queued.emplace(j.id, std::move(j));
    s->st.submitted++;
  }
  s->cv_work.notify_one();
  return CKKS_OK;
}

int ckks_server_poll(ckks_server *s, ckks_job_result *out, uint32_t max, uint32_t *n_out, int32_t wait_ms) {
  if (!s || !n_out || (max && !out)) return ckks::api_fail(CKKS_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [s] { return !s->results.empty() || (s->adm.queued() == 0 && s->busy_slots() == 0) || s->stop; };
  if (wait_ms < 0)
    s->cv_done.wait(lk, ready);
  else if (wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
  uint32_t k = 0;
  while (k < max && !s->results.empty()) {
    out[k++] = s->results.front();
    s->results.pop_front();
  }
  *n_out = k;
  return CKKS_OK;
}

int ckks_server_cancel(ckks_server *s, uint64_t job_id) {
  if (!s) return ckks::api_fail(CKKS_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queued.find(job_id);
    if (it == s->queued.end() || !s->adm.cancel(job_id)) {
      if (job_id == 0 || job_id >= s->next_id) return ckks::api_fail(CKKS_EINVAL, "no job %llu", (unsigned long long)job_id);
      return ckks::api_fail(CKKS_ESTATE, "job %llu has already been admitted", (unsigned long long)job_id);
    }
    ckks_job_result r{};
    r.job_id = job_id;
    r.status = CKKS_ECANCELED;
    r.height = it->second.H;
    r.width = it->second.W;
    r.t_submit_us = it->second.t_submit;
    r.t_done_us = s->now_us();
    s->results.push_back(r);
    s->queued.erase(it);
    s->st.canceled++;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_one();
  return CKKS_OK;
}

int ckks_server_inject_failure(ckks_server *s, uint64_t job_id, int32_t status) {
  if (!s) return ckks::api_fail(CKKS_EINVAL, "server is NULL");
  if (status >= 0) return ckks::api_fail(CKKS_EINVAL, "an injected status must be a CKKS_E* code");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->queued.find(job_id);
  if (it == s->queued.end()) return ckks::api_fail(CKKS_ESTATE, "job %llu is not queued", (unsigned long long)job_id);
  it->second.forced_status = status;
  return CKKS_OK;
}

uint64_t ckks_job_bytes(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t filter_k,
                        uint64_t tile_bytes) {
  if (!ctx || (uint64_t)H * W == 0) return 0;
  return job_bytes_of(ctx, cache, H, W, filter_k, tile_bytes);
}

int ckks_server_drain(ckks_server *s) {
  if (!s) return ckks::api_fail(CKKS_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return (s->adm.queued() == 0 && s->busy_slots() == 0) || s->stop; });
  return CKKS_OK;
}

int ckks_server_stats_get(ckks_server *s, ckks_server_stats *out) {
  if (!s || !out) return ckks::api_fail(CKKS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = s->adm.queued();
  out->backfilled = s->adm.backfilled();
  out->inflight = s->busy_slots();
  out->inflight_bytes = s->adm.arena().used();
  return CKKS_OK;
}

void ckks_server_destroy(ckks_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    std::vector<uint64_t> dropped;
    s->adm.cancel_queued(dropped);
    for (uint64_t id : dropped) s->queued.erase(id);
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  int dev_prev = -1;
  (void)hipGetDevice(&dev_prev);
  (void)hipSetDevice(s->ctx->device);
  free_server(s);
  if (dev_prev >= 0) (void)hipSetDevice(dev_prev);
}

}  // extern "C"
