// C ABI: argument validation, context and cache management, and kernel dispatch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "modarith.hpp"
#include "philox.hpp"

using namespace ckks;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(CKKS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Keeps the caller's current device and restores it on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

template <typename T>
hipError_t upload(T *dst, const std::vector<T> &src) {
  return hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

int resolve_params(const ckks_params *p, host::Resolved *r) {
  if (!p) return fail(CKKS_EINVAL, "params is NULL");
  int code = CKKS_OK;
  std::string why = host::resolve(p->log_n, p->num_primes, p->prime_bits, p->log_scale, p->sigma, p->gauss_bound,
                                  p->primes, r, &code);
  if (code != CKKS_OK) return fail(code, "%s", why.c_str());
  return CKKS_OK;
}

void free_tables(ckks_ctx *c) {
  DevTables &d = c->dev;
  void *ptrs[] = {d.tw_fwd, d.tw_inv, d.enc_T, d.cosj, d.cdt, d.s, d.pk, d.pk_hat, d.s_hat, d.evk, d.evk_hat, c->d_lc};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  d = DevTables{};
  c->d_lc = nullptr;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Fixed device scratch of ckks_encrypt_cached_noalloc: one copy per GPU the library runs
// on, held until the process ends.  In host code `scratch` names a host-side stand-in, not
// the device array: its device address comes from hipGetSymbolAddress, resolved once per
// device (with that device current) when a context is created there.
constexpr uint64_t kNoAllocScratchBytes = 32ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, or NULL if it cannot be resolved.
void *noalloc_scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

uint64_t ct_words(const ckks_ctx *c, uint32_t level) { return (uint64_t)2 * level * (uint64_t)c->N; }

int check_ctx(const ckks_ctx *c) {
  if (!c) return fail(CKKS_EINVAL, "context is NULL");
  return CKKS_OK;
}

int check_keys(const ckks_ctx *c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->has_keys) return fail(CKKS_ESTATE, "no keys: call ckks_keygen or ckks_keys_import first");
  return CKKS_OK;
}

int check_batch(const ckks_ctx *c, const ckks_ct_batch *b, const char *name) {
  if (!b) return fail(CKKS_EINVAL, "%s is NULL", name);
  if (b->level < 1 || b->level > (uint32_t)c->prm.L) return fail(CKKS_ELEVEL, "%s: level %u outside [1, %d]", name, b->level, c->prm.L);
  if (b->count && !b->data) return fail(CKKS_EINVAL, "%s: data is NULL", name);
  if (!(b->scale > 0.0) || !isfinite(b->scale)) return fail(CKKS_ESCALE, "%s: scale must be positive and finite", name);
  return CKKS_OK;
}

// An output descriptor's incoming count and level describe its buffer: count = 0 means
// the caller vouches for the size; otherwise the buffer holds count ciphertexts of level
// `level` (0: the result's level), and must have room for n ciphertexts at result_level.
int check_out(const ckks_ctx *c, const ckks_ct_batch *out, uint64_t n, uint32_t result_level) {
  if (!out) return fail(CKKS_EINVAL, "out is NULL");
  if (n && !out->data) return fail(CKKS_EINVAL, "out data is NULL");
  if (!out->count) return CKKS_OK;
  const uint32_t lv = out->level ? out->level : result_level;
  if (lv < 1 || lv > (uint32_t)c->prm.L) return fail(CKKS_ELEVEL, "out: level %u outside [1, %d]", lv, c->prm.L);
  const unsigned __int128 have = (unsigned __int128)out->count * ct_words(c, lv);
  const unsigned __int128 need = (unsigned __int128)n * ct_words(c, result_level);
  if (have < need)
    return fail(CKKS_EINVAL, "out holds %llu ciphertexts of level %u, the result needs %llu of level %u",
                (unsigned long long)out->count, lv, (unsigned long long)n, result_level);
  return CKKS_OK;
}

int check_cache(const ckks_ctx *c, const ckks_cache *cache) {
  if (!cache || cache->ctx != c) return fail(CKKS_ECACHE, "cache is NULL or belongs to another context");
  if (cache->key_epoch != c->key_epoch)
    return fail(CKKS_ESTATE, "the cache was built under keys that have since been replaced");
  return CKKS_OK;
}

// Constant c as a per-limb multiplier (integer c keeps the scale unless `scaled`; any
// other c becomes K = rint(c * q_{level-1}) at scale * q_{level-1}).
int const_multiplier(const ckks_ctx *c, uint32_t level, double scale, double cst, std::vector<uint64_t> &K,
                     double *new_scale, bool scaled = false) {
  if (!isfinite(cst)) return fail(CKKS_EINVAL, "constant is not finite");
  double Kd = cst;
  double ns = scale;
  if (scaled || cst != rint(cst)) {
    const double ql = (double)c->prm.q[level - 1];
    Kd = rint(cst * ql);
    ns = scale * ql;
  }
  if (!isfinite(Kd) || !isfinite(ns)) return fail(CKKS_ESCALE, "scaled constant overflows");
  K.resize(level);
  for (uint32_t i = 0; i < level; i++) {
    const uint64_t q = c->prm.q[i];
    K[i] = residue_of_double(Kd, q, 1.0 / (double)q);
  }
  *new_scale = ns;
  return CKKS_OK;
}

}  // namespace

namespace ckks {

static uint64_t ws_align(uint64_t x) { return (x + 255) / 256 * 256; }

uint64_t cached_ws_bytes(const ckks_cache *cache, uint64_t n) {
  if (cache->kind == CKKS_CACHE_RADIX) return ws_align(n * kMaxDigits * sizeof(int16_t)) + 256;
  return 3 * ws_align(n * sizeof(uint32_t)) + ws_align(value_counter_words(cache) * sizeof(uint32_t));
}

hipError_t encrypt_cached_ws(const ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *px, uint64_t n,
                             uint64_t seed0, uint64_t seed1, uint64_t first_index, uint64_t *out, void *ws,
                             hipStream_t st, bool concurrent) {
  uint8_t *w = static_cast<uint8_t *>(ws);
  if (cache->kind == CKKS_CACHE_RADIX) {
    int16_t *meta = reinterpret_cast<int16_t *>(w);
    uint32_t *bad = reinterpret_cast<uint32_t *>(w + ws_align(n * kMaxDigits * sizeof(int16_t)));
    hipError_t e = launch_radix_meta(ctx, cache, px, n, first_index, seed0, seed1, meta, bad, st);
    return e == hipSuccess ? launch_radix_gather(ctx, cache, meta, n, out, st) : e;
  }
  const uint64_t a = ws_align(n * sizeof(uint32_t));
  uint32_t *meta = reinterpret_cast<uint32_t *>(w);
  uint32_t *miss = reinterpret_cast<uint32_t *>(w + a);
  uint32_t *hits = reinterpret_cast<uint32_t *>(w + 2 * a);
  uint32_t *counters = reinterpret_cast<uint32_t *>(w + 3 * a);
  hipError_t e = launch_value_meta(ctx, cache, px, n, first_index, seed0, seed1, meta, miss, counters, hits, st);
  if (e != hipSuccess) return e;
  EncJob job;
  job.px = px;
  job.list = miss;
  job.list_count = counters;
  job.n = n;
  job.first_index = first_index;
  job.seed0 = seed0;
  job.seed1 = seed1;
  job.out = out;
  if (cache->kind == CKKS_CACHE_VALUE_FULL)  // every value is cached: no misses
    return launch_value_gather(ctx, cache, meta, counters, hits, n, out, nullptr, st);
  if (!concurrent || !ctx->aux) {
    e = launch_value_gather(ctx, cache, meta, counters, hits, n, out, nullptr, st);
    return e == hipSuccess ? launch_encrypt(ctx, job, std::min<uint64_t>(n, kListGrid), st) : e;
  }
  // The misses (compute-bound full encryptions) run on the auxiliary stream beside the hit
  // gather (bound by HBM writes); both grids are bounded so that every CU holds one
  // encryption workgroup and one gather workgroup at once (of 1/2, 3/4, 1, 2 or 3 gather
  // workgroups per CU, one balanced the two streams best).
  hipEvent_t fork = nullptr, join = nullptr;
  e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(ctx->aux, fork, 0);
  if (e == hipSuccess) e = launch_encrypt(ctx, job, std::min<uint64_t>(n, (uint64_t)ctx->num_cus), ctx->aux);
  if (e == hipSuccess) e = hipEventRecord(join, ctx->aux);
  if (e == hipSuccess)
    e = launch_value_gather(ctx, cache, meta, counters, hits, n, out, nullptr, st, (uint64_t)ctx->num_cus);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
  // events may be destroyed while their work is pending; the runtime releases them after
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  return e;
}

int filter_multiplier(const ckks_ctx *c, uint32_t level, double scale, uint32_t k, std::vector<uint64_t> &K,
                      double *new_scale) {
  return const_multiplier(c, level, scale, 1.0 / (double)(k * k), K, new_scale, true);
}

double encryption_terms(const ckks_cache *cache) {
  if (!cache) return 1.0;
  if (cache->kind != CKKS_CACHE_RADIX) return 2.0;  // entry + pool member
  // radix: Enc(0) plus k_i Enc(r^i) with |k_i| = |d_i + b_i - r b_{i+1}| <= 2r
  return 1.0 + 2.0 * cache->base * cache->digits;
}

bool limb0_decode_exact(const ckks_ctx *c, double value_bound, double terms, bool filtered) {
  const double N = (double)c->N, B = (double)c->prm.B;
  // message: |rint(p T_j)| <= |p| Delta 2^(1 - log N) + 1/2 for each encoded term
  double x = value_bound * ldexp(c->scale, 1 - c->prm.log_n) + 2.0;
  // noise of one encryption: v e + e0 + e1 s with v, s ternary and |e| <= B in every coefficient
  x += terms * (2.0 * N + 1.0) * B;
  // a filter output is (K sum)/q_last plus the rescale rounding r0 + r1 s over q_last, with
  // K <= q_last / k^2 + 1/2: at most the input bound (1 + k^2 / (2 q_last)) plus (N + 1) / 2
  if (filtered) x = x * (1.0 + 1.0 / 1048576.0) + N;
  return x < 0.49 * (double)c->prm.q[0];
}

hipError_t WsLease::get(uint64_t bytes, void **out) {
  size_t i = 0;
  while (i < c_->ws.size() && c_->ws[i].stream != st_) i++;
  if (i == c_->ws.size() && c_->ws.size() >= kMaxStreamWs) {
    // release the least recently used stream's buffer once its last use is done, and
    // give its entry (and event) to this stream
    i = 0;
    for (size_t j = 1; j < c_->ws.size(); j++)
      if (c_->ws[j].used < c_->ws[i].used) i = j;
    StreamWorkspace &old = c_->ws[i];
    hipError_t e = hipEventSynchronize(old.last);
    if (e == hipSuccess && old.ptr) e = hipFree(old.ptr);
    old.ptr = nullptr;
    old.bytes = 0;
    if (e != hipSuccess) return e;
    old.stream = st_;
  } else if (i == c_->ws.size()) {
    StreamWorkspace w;
    w.stream = st_;
    const hipError_t e = hipEventCreateWithFlags(&w.last, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    c_->ws.push_back(w);
  }
  StreamWorkspace &w = c_->ws[i];
  w.used = ++c_->ws_leases;
  if (w.bytes < bytes) {
    if (w.ptr) {
      hipError_t e = hipEventSynchronize(w.last);
      if (e == hipSuccess) e = hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
      if (e != hipSuccess) return e;
    }
    const uint64_t want = (bytes + bytes / 2 + (2ull << 20) - 1) / (2ull << 20) * (2ull << 20);
    const hipError_t e = hipMalloc(&w.ptr, want);
    if (e != hipSuccess) {
      w.ptr = nullptr;
      return e;
    }
    w.bytes = want;
  }
  const hipError_t e = hipStreamWaitEvent(st_, w.last, 0);
  if (e != hipSuccess) return e;
  w_ = &w;
  *out = w.ptr;
  return hipSuccess;
}

void ws_free_all(ckks_ctx *c) {
  std::lock_guard<std::mutex> lk(c->ws_mu);
  for (StreamWorkspace &w : c->ws) {
    if (w.ptr) (void)hipFree(w.ptr);
    if (w.last) (void)hipEventDestroy(w.last);
  }
  c->ws.clear();
}

int api_fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace ckks

extern "C" {

const char *ckks_last_error(void) { return g_err.c_str(); }

int ckks_params_resolve(const ckks_params *params, uint64_t *host_primes, uint32_t *gauss_bound) {
  host::Resolved r;
  int rc = resolve_params(params, &r);
  if (rc) return rc;
  if (host_primes)
    for (int i = 0; i < r.L; i++) host_primes[i] = r.q[(size_t)i];
  if (gauss_bound) *gauss_bound = (uint32_t)r.B;
  return CKKS_OK;
}

int ckks_host_cdt_table(const ckks_params *params, uint64_t *host_out, uint32_t capacity) {
  host::Resolved r;
  int rc = resolve_params(params, &r);
  if (rc) return rc;
  if ((uint32_t)(2 * r.B) > capacity || (!host_out && r.B)) return fail(CKKS_EINVAL, "need room for %d entries", 2 * r.B);
  std::vector<uint64_t> T = host::cdt_table(r.sigma, r.B, kCdtSlots);
  for (int k = 0; k < 2 * r.B; k++) host_out[k] = T[(size_t)k];
  return CKKS_OK;
}

int ckks_host_encode_table(const ckks_params *params, double *host_out, uint64_t capacity) {
  host::Resolved r;
  int rc = resolve_params(params, &r);
  if (rc) return rc;
  const uint64_t N = 1ULL << r.log_n;
  if (!host_out || capacity < N) return fail(CKKS_EINVAL, "need room for %llu entries", (unsigned long long)N);
  std::vector<double> T = host::encode_table(r.log_n, r.log_scale);
  memcpy(host_out, T.data(), N * sizeof(double));
  return CKKS_OK;
}

int ckks_context_create(const ckks_params *params, int device, ckks_ctx **out) {
  if (!out) return fail(CKKS_EINVAL, "out is NULL");
  *out = nullptr;
  host::Resolved r;
  int rc = resolve_params(params, &r);
  if (rc) return rc;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(CKKS_EINVAL, "device %d outside [0, %d)", device, ndev);
  DeviceGuard g(device);
  ckks_ctx *c = new ckks_ctx();
  c->device = device;
  c->prm = r;
  c->N = 1 << r.log_n;
  c->scale = ldexp(1.0, r.log_scale);
  const int N = c->N, L = r.L;
  LimbConsts &lc = c->lc;
  memset(&lc, 0, sizeof(lc));
  lc.L = L;
  lc.B = r.B;
  double qmax = 0;
  // rows 0..L-1: the ciphertext primes; row L: the special prime of key switching (if any)
  const int rows = L + (r.qP ? 1 : 0);
  std::vector<double> twf((size_t)rows * N), twi((size_t)rows * N);
  for (int i = 0; i < rows; i++) {
    const uint64_t q = i < L ? r.q[(size_t)i] : r.qP;
    lc.q[i] = (double)q;
    lc.qinv[i] = 1.0 / (double)q;
    lc.qi[i] = q;
    const uint64_t ni = host::inv_mod((uint64_t)N % q, q);
    if (i < L) c->ninv.push_back(ni);
    lc.ninv[i] = host::centered(ni, q);
    qmax = std::max(qmax, (double)q);
    std::vector<double> f, iv;
    host::twiddles(q, i < L ? r.psi[(size_t)i] : r.psiP, r.log_n, f, iv);
    std::copy(f.begin(), f.end(), twf.begin() + (size_t)i * N);
    std::copy(iv.begin(), iv.end(), twi.begin() + (size_t)i * N);
    if (i < L && r.qP) {
      lc.pinv[i] = host::centered(host::inv_mod(r.qP % q, q), q);
      lc.pmod[i] = host::centered(r.qP % q, q);
    }
  }
  if (L >= 2) lc.q0inv_q1 = host::centered(host::inv_mod(r.q[0] % r.q[1], r.q[1]), r.q[1]);
  // the transforms' lazy-reduction schedule is compiled per class of prime sizes
  c->rc = qmax < 1099511627776.0 ? 0 : 1;
  // values per NTT thread (measured on MI355X at N = 8192): encryption, decryption and
  // the product are fastest with 8 (16 waves per ciphertext, 4 waves per SIMD); 8 needs
  // N / 8 <= 1024 threads
  c->logr_enc = N / 8 <= 1024 ? 3 : 4;
  c->logr_dec = c->logr_enc;
  c->logr_mul = c->logr_enc;
  hipError_t e = hipSuccess;
  DevTables &d = c->dev;
  if (e == hipSuccess) e = dev_alloc(&d.tw_fwd, (size_t)rows * N);
  if (e == hipSuccess) e = dev_alloc(&d.tw_inv, (size_t)rows * N);
  if (e == hipSuccess) e = dev_alloc(&d.enc_T, (size_t)N);
  if (e == hipSuccess) e = dev_alloc(&d.cosj, (size_t)N);
  if (e == hipSuccess) e = dev_alloc(&d.cdt, (size_t)kCdtSlots);
  if (e == hipSuccess) e = dev_alloc(&d.s, (size_t)N);
  if (e == hipSuccess) e = dev_alloc(&d.pk, (size_t)2 * L * N);
  if (e == hipSuccess) e = dev_alloc(&d.pk_hat, (size_t)2 * L * N);
  if (e == hipSuccess) e = dev_alloc(&d.s_hat, (size_t)L * N);
  if (e != hipSuccess) {
    free_tables(c);
    delete c;
    return fail(CKKS_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  if (e == hipSuccess) e = upload(d.tw_fwd, twf);
  if (e == hipSuccess) e = upload(d.tw_inv, twi);
  if (e == hipSuccess) e = upload(d.enc_T, host::encode_table(r.log_n, r.log_scale));
  if (e == hipSuccess) e = upload(d.cosj, host::cos_table(r.log_n));
  if (e == hipSuccess) e = upload(d.cdt, host::cdt_table(r.sigma, r.B, kCdtSlots));
  if (e == hipSuccess) e = dev_alloc(&c->d_lc, 1);
  if (e == hipSuccess) e = hipMemcpy(c->d_lc, &c->lc, sizeof(LimbConsts), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    // scratch pool of the context: per-call workspaces come from it on the call's
    // stream; memory freed into it is kept for the next call instead of being unmapped
    // at every synchronization (the default pool's behaviour)
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    e = hipMemPoolCreate(&c->pool, &props);
    uint64_t keep = ~0ull;
    if (e == hipSuccess) e = hipMemPoolSetAttribute(c->pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  if (e != hipSuccess) {
    free_tables(c);
    delete c;
    return hip_fail(e, "uploading tables");
  }
  c->noalloc_scratch = noalloc_scratch_address(device);  // with `device` current (DeviceGuard)
  if (hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->num_cus < 1)
    c->num_cus = 1;
  if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) c->aux = nullptr;
  *out = c;
  return CKKS_OK;
}

void ckks_context_destroy(ckks_ctx *ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  for (hipStream_t &st : ctx->pipe)
    if (st) (void)hipStreamDestroy(st);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  ws_free_all(ctx);
  free_tables(ctx);
  if (ctx->pool) (void)hipMemPoolDestroy(ctx->pool);
  delete ctx;
}

int ckks_context_set_ntt_width(ckks_ctx *ctx, uint32_t values_per_thread) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (values_per_thread != 8 && values_per_thread != 16 && values_per_thread != 32)
    return fail(CKKS_EINVAL, "values_per_thread must be 8, 16 or 32");
  if (ctx->N / values_per_thread > 1024) return fail(CKKS_EINVAL, "N / values_per_thread exceeds 1024 threads");
  ctx->logr_enc = ctx->logr_dec = ctx->logr_mul = values_per_thread == 8 ? 3 : (values_per_thread == 16 ? 4 : 5);
  return CKKS_OK;
}

int ckks_context_get_ntt_width(const ckks_ctx *ctx, uint32_t *values_per_thread) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!values_per_thread) return fail(CKKS_EINVAL, "values_per_thread is NULL");
  *values_per_thread = 1u << ctx->logr_enc;
  return CKKS_OK;
}

int ckks_context_set_launch_shapes(ckks_ctx *ctx, uint32_t row_wgs, uint32_t gather_wgs) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (row_wgs > 64) return fail(CKKS_EINVAL, "row_wgs must be 0..64");
  if (gather_wgs < 1 || gather_wgs > 64) return fail(CKKS_EINVAL, "gather_wgs must be 1..64");
  ctx->row_wgs = (int)row_wgs;
  ctx->gather_wgs = (int)gather_wgs;
  return CKKS_OK;
}

int ckks_context_get_launch_shapes(const ckks_ctx *ctx, uint32_t *row_wgs, uint32_t *gather_wgs) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!row_wgs || !gather_wgs) return fail(CKKS_EINVAL, "row_wgs/gather_wgs is NULL");
  *row_wgs = (uint32_t)ctx->row_wgs;
  *gather_wgs = (uint32_t)ctx->gather_wgs;
  return CKKS_OK;
}

uint64_t ckks_ct_bytes(const ckks_ctx *ctx, uint32_t level) {
  if (!ctx || level < 1 || level > (uint32_t)ctx->prm.L) return 0;
  return ct_words(ctx, level) * sizeof(uint64_t);
}

int ckks_context_info(const ckks_ctx *ctx, uint32_t *log_n, uint32_t *num_primes, double *scale,
                      uint64_t *host_primes) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (log_n) *log_n = (uint32_t)ctx->prm.log_n;
  if (num_primes) *num_primes = (uint32_t)ctx->prm.L;
  if (scale) *scale = ctx->scale;
  if (host_primes)
    for (int i = 0; i < ctx->prm.L; i++) host_primes[i] = ctx->prm.q[(size_t)i];
  return CKKS_OK;
}

int ckks_keygen(ckks_ctx *ctx, const uint64_t seed[2]) {
  TraceRange trace_range_("ckks_keygen");
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!seed) return fail(CKKS_EINVAL, "seed is NULL");
  DeviceGuard g(ctx->device);
  // the old keys are gone from here on: key-switching keys of the old s and every cache,
  // plan or server built under them become invalid
  ctx->has_keys = false;
  ctx->has_relin = false;
  ctx->key_epoch++;
  HIP_TRY(launch_keygen(ctx, seed[0], seed[1], nullptr), "keygen launch");
  HIP_TRY(launch_keys_prepare(ctx, nullptr), "key preparation launch");
  HIP_TRY(hipDeviceSynchronize(), "keygen");
  ctx->has_keys = true;
  return CKKS_OK;
}

int ckks_keys_export(ckks_ctx *ctx, int64_t *host_s, uint64_t *host_pk) {
  int rc = check_keys(ctx);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  const size_t N = (size_t)ctx->N, L = (size_t)ctx->prm.L;
  if (host_s) HIP_TRY(hipMemcpy(host_s, ctx->dev.s, N * sizeof(int64_t), hipMemcpyDeviceToHost), "export s");
  if (host_pk) HIP_TRY(hipMemcpy(host_pk, ctx->dev.pk, 2 * L * N * sizeof(uint64_t), hipMemcpyDeviceToHost), "export pk");
  return CKKS_OK;
}

int ckks_relin_keygen(ckks_ctx *ctx, const uint64_t seed[2]) {
  TraceRange trace_range_("ckks_relin_keygen");
  int rc = check_keys(ctx);
  if (rc) return rc;
  if (!seed) return fail(CKKS_EINVAL, "seed is NULL");
  if (!ctx->prm.qP) return fail(CKKS_EUNSUPPORTED, "no special prime of the NTT form exists for these parameters");
  DeviceGuard g(ctx->device);
  const size_t words = (size_t)ctx->prm.L * (ctx->prm.L + 1) * 2 * ctx->N;
  if (!ctx->dev.evk) {
    if (dev_alloc(&ctx->dev.evk, words) != hipSuccess) return fail(CKKS_ENOMEM, "key-switching key allocation");
    if (dev_alloc(&ctx->dev.evk_hat, words) != hipSuccess) return fail(CKKS_ENOMEM, "key-switching key allocation");
  }
  ctx->has_relin = false;
  HIP_TRY(launch_relin_keygen(ctx, seed[0], seed[1], nullptr), "key-switching keygen launch");
  HIP_TRY(launch_relin_prepare(ctx, nullptr), "key-switching key preparation launch");
  HIP_TRY(hipDeviceSynchronize(), "key-switching keygen");
  ctx->has_relin = true;
  return CKKS_OK;
}

int ckks_relin_keys_export(ckks_ctx *ctx, uint64_t *host_evk, uint64_t *host_special_prime) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!ctx->has_relin) return fail(CKKS_ESTATE, "no key-switching keys: call ckks_relin_keygen first");
  if (host_special_prime) *host_special_prime = ctx->prm.qP;
  if (!host_evk) return CKKS_OK;
  DeviceGuard g(ctx->device);
  const size_t words = (size_t)ctx->prm.L * (ctx->prm.L + 1) * 2 * ctx->N;
  HIP_TRY(hipMemcpy(host_evk, ctx->dev.evk, words * sizeof(uint64_t), hipMemcpyDeviceToHost), "export evk");
  return CKKS_OK;
}

int ckks_keys_import(ckks_ctx *ctx, const int64_t *host_s, const uint64_t *host_pk) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!host_s || !host_pk) return fail(CKKS_EINVAL, "keys are NULL");
  const size_t N = (size_t)ctx->N, L = (size_t)ctx->prm.L;
  for (size_t j = 0; j < N; j++)
    if (host_s[j] < -1 || host_s[j] > 1) return fail(CKKS_EINVAL, "secret key coefficient %zu not in {-1,0,1}", j);
  for (size_t p = 0; p < 2; p++)
    for (size_t i = 0; i < L; i++)
      for (size_t j = 0; j < N; j++)
        if (host_pk[(p * L + i) * N + j] >= ctx->prm.q[i]) return fail(CKKS_EINVAL, "public key residue not canonical");
  DeviceGuard g(ctx->device);
  ctx->has_keys = false;
  ctx->has_relin = false;
  ctx->key_epoch++;
  HIP_TRY(hipMemcpy(ctx->dev.s, host_s, N * sizeof(int64_t), hipMemcpyHostToDevice), "import s");
  HIP_TRY(hipMemcpy(ctx->dev.pk, host_pk, 2 * L * N * sizeof(uint64_t), hipMemcpyHostToDevice), "import pk");
  HIP_TRY(launch_keys_prepare(ctx, nullptr), "key preparation launch");
  HIP_TRY(hipDeviceSynchronize(), "key preparation");
  ctx->has_keys = true;
  return CKKS_OK;
}

int ckks_encrypt_pixels(ckks_ctx *ctx, const uint8_t *d_px, uint64_t n, const uint64_t seed[2],
                        uint64_t first_index, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_encrypt_pixels");
  int rc = check_keys(ctx);
  if (rc) return rc;
  if (!seed || !out) return fail(CKKS_EINVAL, "seed/out is NULL");
  if (n && !d_px) return fail(CKKS_EINVAL, "pixel pointer is NULL");
  if (n > 0xFFFFFFFFull) return fail(CKKS_EINVAL, "at most 2^32-1 pixels per call");
  if ((rc = check_out(ctx, out, n, (uint32_t)ctx->prm.L))) return rc;
  out->count = n;
  out->level = (uint32_t)ctx->prm.L;
  out->scale = ctx->scale;
  if (n == 0) return CKKS_OK;
  DeviceGuard g(ctx->device);
  EncJob job;
  job.px = d_px;
  job.n = n;
  job.first_index = first_index;
  job.seed0 = seed[0];
  job.seed1 = seed[1];
  job.out = out->data;
  const uint64_t grid = std::min<uint64_t>(n, 1u << 24);
  HIP_TRY(launch_encrypt(ctx, job, grid, as_stream(stream)), "encrypt launch");
  return CKKS_OK;
}

int ckks_cache_build(ckks_ctx *ctx, const ckks_cache_desc *desc, const uint8_t *d_scan, uint64_t n_scan,
                     const uint64_t cache_seed[2], ckks_cache **out, void *stream) {
  TraceRange trace_range_("ckks_cache_build");
  int rc = check_keys(ctx);
  if (rc) return rc;
  if (!desc || !cache_seed || !out) return fail(CKKS_EINVAL, "desc/seed/out is NULL");
  *out = nullptr;
  const int kind = desc->kind;
  uint32_t n_slots = 0;
  std::vector<uint32_t> vals;
  std::vector<uint64_t> ts;
  std::vector<int16_t> slot_of(256, -1);
  if (kind == CKKS_CACHE_RADIX) {
    const uint32_t r = desc->base, D = desc->digits;
    // one digit would leave no radix randomness (Sec. 3.3 draws one bit per radix above the
    // lowest), so every pixel value would map to one fixed ciphertext
    if (r < 2 || r > 256 || D < 2 || D > (uint32_t)kMaxDigits) return fail(CKKS_ECACHE, "radix base must be in [2,256], digits in [2,8]");
    uint64_t pw = 1;
    for (uint32_t i = 0; i + 1 < D; i++) pw *= r;
    if (pw > 255) return fail(CKKS_ECACHE, "base^(digits-1) = %llu exceeds 255", (unsigned long long)pw);
    if (pw * r < 256) return fail(CKKS_ECACHE, "base^digits must be >= 256 to cover every pixel");
    n_slots = D + 1;
    vals.push_back(0);
    ts.push_back(0);
    pw = 1;
    for (uint32_t i = 0; i < D; i++) {
      vals.push_back((uint32_t)pw);
      ts.push_back(1 + i);
      pw *= r;
    }
  } else if (kind == CKKS_CACHE_VALUE_TOPK || kind == CKKS_CACHE_VALUE_FULL) {
    if (desc->zero_pool < 1 || desc->zero_pool > 4096) return fail(CKKS_ECACHE, "zero_pool must be in [1, 4096]");
    if (kind == CKKS_CACHE_VALUE_TOPK) {
      if (desc->topk < 1 || desc->topk > 256) return fail(CKKS_ECACHE, "topk must be in [1, 256]");
      if (n_scan && !d_scan) return fail(CKKS_EINVAL, "scan pixels are NULL");
      if (n_scan > 0xFFFFFFFFull) return fail(CKKS_EINVAL, "at most 2^32-1 scan pixels");
      n_slots = desc->topk;
      vals.assign(n_slots, 0);
      ts.assign(n_slots, 0);
    } else {
      n_slots = 256;
      for (uint32_t v = 0; v < 256; v++) {
        vals.push_back(v);
        ts.push_back(256 + v);
        slot_of[v] = (int16_t)v;
      }
    }
  } else {
    return fail(CKKS_ECACHE, "unknown cache kind %d", kind);
  }
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  ckks_cache *c = new ckks_cache();
  c->ctx = ctx;
  c->key_epoch = ctx->key_epoch;
  c->device = ctx->device;
  c->kind = kind;
  c->base = desc->base;
  c->digits = desc->digits;
  c->topk = desc->topk;
  c->pool = (kind == CKKS_CACHE_RADIX) ? 0 : desc->zero_pool;
  c->n_slots = n_slots;
  const uint64_t S = ct_words(ctx, (uint32_t)ctx->prm.L);
  hipError_t e = dev_alloc(&c->entries, (size_t)n_slots * S);
  if (e == hipSuccess && c->pool) e = dev_alloc(&c->pool_cts, (size_t)c->pool * S);
  if (e == hipSuccess) e = dev_alloc(&c->slot_of, 256);
  if (e == hipSuccess) e = dev_alloc(&c->vals, n_slots);
  if (e == hipSuccess) e = dev_alloc(&c->ts, n_slots);
  if (e == hipSuccess) e = dev_alloc(&c->count, 1);
  if (e != hipSuccess) {
    ckks_cache_destroy(c);
    return fail(CKKS_ENOMEM, "cache allocation failed: %s", hipGetErrorString(e));
  }
  // setup arrays are copied synchronously, before any work is enqueued on the stream
  const uint32_t count = n_slots;
  e = upload(c->slot_of, slot_of);
  if (e == hipSuccess) e = upload(c->vals, vals);
  if (e == hipSuccess) e = upload(c->ts, ts);
  if (e == hipSuccess) e = hipMemcpy(c->count, &count, sizeof(count), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ckks_cache_destroy(c);
    return hip_fail(e, "cache setup copy");
  }
  uint32_t *hist = nullptr;
  if (kind == CKKS_CACHE_VALUE_TOPK) {
    e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&hist), 256 * sizeof(uint32_t), ctx->pool, st);
    if (e == hipSuccess) e = launch_histogram_topk(ctx, d_scan, n_scan, desc->topk, hist, c, st);
    if (e == hipSuccess) e = hipFreeAsync(hist, st);
  }
  if (e == hipSuccess) {
    EncJob job;
    job.vals = c->vals;
    job.ts = c->ts;
    job.list_count = c->count;
    job.n = n_slots;
    job.seed0 = cache_seed[0];
    job.seed1 = cache_seed[1];
    job.out = c->entries;
    e = launch_encrypt(ctx, job, n_slots, st);
  }
  if (e == hipSuccess && c->pool) {
    // pool member u = Enc(0) at Philox index 512 + u
    std::vector<uint32_t> zv(c->pool, 0);
    std::vector<uint64_t> zt(c->pool);
    for (uint32_t u = 0; u < c->pool; u++) zt[u] = 512 + (uint64_t)u;
    uint32_t *d_zv = nullptr;
    uint64_t *d_zt = nullptr;
    e = dev_alloc(&d_zv, c->pool);
    if (e == hipSuccess) e = dev_alloc(&d_zt, c->pool);
    if (e == hipSuccess) e = upload(d_zv, zv);
    if (e == hipSuccess) e = upload(d_zt, zt);
    if (e == hipSuccess) {
      EncJob job;
      job.vals = d_zv;
      job.ts = d_zt;
      job.n = c->pool;
      job.seed0 = cache_seed[0];
      job.seed1 = cache_seed[1];
      job.out = c->pool_cts;
      e = launch_encrypt(ctx, job, c->pool, st);
    }
    // the temporary arrays are released once the stream has consumed them
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (d_zv) (void)hipFree(d_zv);
    if (d_zt) (void)hipFree(d_zt);
  }
  if (e != hipSuccess) {
    ckks_cache_destroy(c);
    return hip_fail(e, "cache build");
  }
  *out = c;
  return CKKS_OK;
}

void ckks_cache_destroy(ckks_cache *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  void *ptrs[] = {c->entries, c->pool_cts, c->slot_of, c->vals, c->ts, c->count};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

int ckks_cache_entries(ckks_cache *cache, uint32_t *n_entries) {
  if (!cache || !n_entries) return fail(CKKS_EINVAL, "cache/n_entries is NULL");
  DeviceGuard g(cache->device);
  HIP_TRY(hipDeviceSynchronize(), "cache build");
  HIP_TRY(hipMemcpy(n_entries, cache->count, sizeof(uint32_t), hipMemcpyDeviceToHost), "cache count");
  return CKKS_OK;
}

int ckks_cache_export(ckks_cache *cache, uint32_t *host_values, uint64_t *host_entries, uint64_t *host_pool) {
  uint32_t n = 0;
  int rc = ckks_cache_entries(cache, &n);
  if (rc) return rc;
  DeviceGuard g(cache->device);
  const size_t S = (size_t)ct_words(cache->ctx, (uint32_t)cache->ctx->prm.L);
  if (host_values) HIP_TRY(hipMemcpy(host_values, cache->vals, n * sizeof(uint32_t), hipMemcpyDeviceToHost), "cache values");
  if (host_entries)
    HIP_TRY(hipMemcpy(host_entries, cache->entries, (size_t)n * S * sizeof(uint64_t), hipMemcpyDeviceToHost), "cache entries");
  if (host_pool && cache->pool)
    HIP_TRY(hipMemcpy(host_pool, cache->pool_cts, (size_t)cache->pool * S * sizeof(uint64_t), hipMemcpyDeviceToHost),
            "cache pool");
  return CKKS_OK;
}

int ckks_cache_import(ckks_ctx *ctx, const ckks_cache_desc *desc, uint32_t n_entries, const uint32_t *host_values,
                      const uint64_t *host_entries, const uint64_t *host_pool, ckks_cache **out) {
  int rc = check_keys(ctx);
  if (rc) return rc;
  if (!desc || !out || !host_values || !host_entries) return fail(CKKS_EINVAL, "desc/out/values/entries is NULL");
  *out = nullptr;
  const int kind = desc->kind;
  const uint32_t n = n_entries;
  std::vector<int16_t> slot_of(256, -1);
  if (kind == CKKS_CACHE_RADIX) {
    const uint32_t r = desc->base, D = desc->digits;
    if (r < 2 || r > 256 || D < 2 || D > (uint32_t)kMaxDigits) return fail(CKKS_ECACHE, "radix base must be in [2,256], digits in [2,8]");
    uint64_t top = 1;
    for (uint32_t i = 0; i + 1 < D; i++) top *= r;
    if (top > 255 || top * r < 256) return fail(CKKS_ECACHE, "base^(digits-1) must be <= 255 and base^digits >= 256");
    if (n != D + 1) return fail(CKKS_ECACHE, "a radix cache has digits + 1 = %u entries, got %u", D + 1, n);
    uint64_t pw = 1;
    for (uint32_t i = 0; i < n; i++) {
      const uint64_t want = i == 0 ? 0 : pw;
      if (host_values[i] != want) return fail(CKKS_ECACHE, "radix entry %u must encrypt %llu", i, (unsigned long long)want);
      if (i) pw *= r;
    }
  } else if (kind == CKKS_CACHE_VALUE_TOPK || kind == CKKS_CACHE_VALUE_FULL) {
    if (desc->zero_pool < 1 || desc->zero_pool > 4096) return fail(CKKS_ECACHE, "zero_pool must be in [1, 4096]");
    if (!host_pool) return fail(CKKS_EINVAL, "a value cache needs its pool of encrypted zeros");
    if (kind == CKKS_CACHE_VALUE_FULL && n != 256) return fail(CKKS_ECACHE, "a full cache has 256 entries, got %u", n);
    if (kind == CKKS_CACHE_VALUE_TOPK && (desc->topk < 1 || desc->topk > 256 || n < 1 || n > desc->topk))
      return fail(CKKS_ECACHE, "a top-k cache has 1..topk entries (topk <= 256), got %u", n);
    for (uint32_t i = 0; i < n; i++) {
      const uint32_t v = host_values[i];
      if (v > 255 || slot_of[v] >= 0) return fail(CKKS_ECACHE, "entry values must be distinct pixel values (entry %u)", i);
      if (kind == CKKS_CACHE_VALUE_FULL && v != i) return fail(CKKS_ECACHE, "full-cache entry %u must encrypt %u", i, i);
      slot_of[v] = (int16_t)i;
    }
  } else {
    return fail(CKKS_ECACHE, "unknown cache kind %d", kind);
  }
  const uint32_t npool = kind == CKKS_CACHE_RADIX ? 0 : desc->zero_pool;
  const size_t N = (size_t)ctx->N, L = (size_t)ctx->prm.L, S = 2 * L * N;
  auto canonical = [&](const uint64_t *ct) {
    for (size_t p = 0; p < 2; p++)
      for (size_t i = 0; i < L; i++)
        for (size_t j = 0; j < N; j++)
          if (ct[(p * L + i) * N + j] >= ctx->prm.q[i]) return false;
    return true;
  };
  for (uint32_t i = 0; i < n; i++)
    if (!canonical(host_entries + (size_t)i * S)) return fail(CKKS_EINVAL, "entry %u has a residue that is not canonical", i);
  for (uint32_t u = 0; u < npool; u++)
    if (!canonical(host_pool + (size_t)u * S)) return fail(CKKS_EINVAL, "pool member %u has a residue that is not canonical", u);
  DeviceGuard g(ctx->device);
  ckks_cache *c = new ckks_cache();
  c->ctx = ctx;
  c->key_epoch = ctx->key_epoch;
  c->device = ctx->device;
  c->kind = kind;
  c->base = desc->base;
  c->digits = desc->digits;
  c->topk = desc->topk;
  c->pool = npool;
  c->n_slots = n;
  std::vector<uint32_t> vals(host_values, host_values + n);
  std::vector<uint64_t> ts(n);
  for (uint32_t i = 0; i < n; i++) ts[i] = kind == CKKS_CACHE_RADIX ? i : 256 + (uint64_t)vals[i];
  hipError_t e = dev_alloc(&c->entries, (size_t)n * S);
  if (e == hipSuccess && npool) e = dev_alloc(&c->pool_cts, (size_t)npool * S);
  if (e == hipSuccess) e = dev_alloc(&c->slot_of, 256);
  if (e == hipSuccess) e = dev_alloc(&c->vals, n);
  if (e == hipSuccess) e = dev_alloc(&c->ts, n);
  if (e == hipSuccess) e = dev_alloc(&c->count, 1);
  if (e != hipSuccess) {
    ckks_cache_destroy(c);
    return fail(CKKS_ENOMEM, "cache allocation failed: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(c->entries, host_entries, (size_t)n * S * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && npool)
    e = hipMemcpy(c->pool_cts, host_pool, (size_t)npool * S * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = upload(c->slot_of, slot_of);
  if (e == hipSuccess) e = upload(c->vals, vals);
  if (e == hipSuccess) e = upload(c->ts, ts);
  if (e == hipSuccess) e = hipMemcpy(c->count, &n, sizeof(n), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ckks_cache_destroy(c);
    return hip_fail(e, "cache upload");
  }
  *out = c;
  return CKKS_OK;
}

int ckks_encrypt_cached(ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint64_t n,
                        const uint64_t seed[2], uint64_t first_index, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_encrypt_cached");
  int rc = check_keys(ctx);
  if (rc) return rc;
  if ((rc = check_cache(ctx, cache))) return rc;
  if (!seed || !out) return fail(CKKS_EINVAL, "seed/out is NULL");
  if (n && !d_px) return fail(CKKS_EINVAL, "pixel pointer is NULL");
  if (n > 0xFFFFFFFFull) return fail(CKKS_EINVAL, "at most 2^32-1 pixels per call");
  if ((rc = check_out(ctx, out, n, (uint32_t)ctx->prm.L))) return rc;
  out->count = n;
  out->level = (uint32_t)ctx->prm.L;
  out->scale = ctx->scale;
  if (n == 0) return CKKS_OK;
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  void *ws = nullptr;
  WsLease lease(ctx, st);
  HIP_TRY(lease.get(cached_ws_bytes(cache, n), &ws), "workspace alloc");
  HIP_TRY(encrypt_cached_ws(ctx, cache, d_px, n, seed[0], seed[1], first_index, out->data, ws, st, true),
          "cached encryption");
  return CKKS_OK;
}

int ckks_encrypt_cached_noalloc(ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint64_t n,
                                const uint64_t seed[2], uint64_t first_index, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_encrypt_cached_noalloc");
  int rc = check_keys(ctx);
  if (rc) return rc;
  if ((rc = check_cache(ctx, cache))) return rc;
  if (!seed || !out) return fail(CKKS_EINVAL, "seed/out is NULL");
  if (n && !d_px) return fail(CKKS_EINVAL, "pixel pointer is NULL");
  if (n > 0xFFFFFFFFull) return fail(CKKS_EINVAL, "at most 2^32-1 pixels per call");
  const uint64_t need = cached_ws_bytes(cache, n);
  if (need > kNoAllocScratchBytes)
    return fail(CKKS_ENOMEM_BUDGET, "%llu pixels need %llu bytes of scratch, the fixed array holds %llu",
                (unsigned long long)n, (unsigned long long)need, (unsigned long long)kNoAllocScratchBytes);
  if ((rc = check_out(ctx, out, n, (uint32_t)ctx->prm.L))) return rc;
  if (!ctx->noalloc_scratch) return fail(CKKS_EDEVICE, "the fixed scratch array has no device address");
  out->count = n;
  out->level = (uint32_t)ctx->prm.L;
  out->scale = ctx->scale;
  if (n == 0) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(encrypt_cached_ws(ctx, cache, d_px, n, seed[0], seed[1], first_index, out->data, ctx->noalloc_scratch,
                            as_stream(stream), false),
          "cached encryption");
  return CKKS_OK;
}

uint64_t ckks_encrypt_cached_noalloc_max_pixels(const ckks_cache *cache) {
  if (!cache) return 0;
  uint64_t lo = 0, hi = 0xFFFFFFFFull;
  while (lo < hi) {  // largest n whose scratch fits (cached_ws_bytes grows with n)
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (cached_ws_bytes(cache, mid) <= kNoAllocScratchBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

static bool overlaps(const uint64_t *a, uint64_t an, const uint64_t *b, uint64_t bn) {
  return a < b + bn && b < a + an;
}

static int binary_common(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if ((rc = check_batch(ctx, a, "a")) || (rc = check_batch(ctx, b, "b"))) return rc;
  if (!out) return fail(CKKS_EINVAL, "out is NULL");
  if (a->count != b->count) return fail(CKKS_EINVAL, "counts differ (%llu vs %llu)", (unsigned long long)a->count, (unsigned long long)b->count);
  if (a->level != b->level) return fail(CKKS_ELEVEL, "levels differ (%u vs %u)", a->level, b->level);
  if (a->scale != b->scale) return fail(CKKS_ESCALE, "scales differ (%.17g vs %.17g)", a->scale, b->scale);
  return check_out(ctx, out, a->count, a->level);
}

int ckks_add(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_add");
  int rc = binary_common(ctx, a, b, out);
  if (rc) return rc;
  const ckks_ct_batch av = *a;
  out->count = av.count;
  out->level = av.level;
  out->scale = av.scale;
  if (!av.count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_add_sub(ctx, av.data, b->data, out->data, av.count, (int)av.level, false, as_stream(stream)), "add");
  return CKKS_OK;
}

int ckks_sub(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_sub");
  int rc = binary_common(ctx, a, b, out);
  if (rc) return rc;
  const ckks_ct_batch av = *a;
  out->count = av.count;
  out->level = av.level;
  out->scale = av.scale;
  if (!av.count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_add_sub(ctx, av.data, b->data, out->data, av.count, (int)av.level, true, as_stream(stream)), "sub");
  return CKKS_OK;
}

int ckks_mul(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_mul");
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if ((rc = check_batch(ctx, a, "a")) || (rc = check_batch(ctx, b, "b"))) return rc;
  if (!ctx->has_relin) return fail(CKKS_ESTATE, "no key-switching keys: call ckks_relin_keygen first");
  if (!out) return fail(CKKS_EINVAL, "out is NULL");
  if (a->count != b->count) return fail(CKKS_EINVAL, "counts differ (%llu vs %llu)", (unsigned long long)a->count, (unsigned long long)b->count);
  if (a->level != b->level) return fail(CKKS_ELEVEL, "levels differ (%u vs %u)", a->level, b->level);
  const double ns = a->scale * b->scale;
  if (!isfinite(ns)) return fail(CKKS_ESCALE, "product scale overflows");
  if ((rc = check_out(ctx, out, a->count, a->level))) return rc;
  const uint64_t words = a->count * ct_words(ctx, a->level);
  for (const ckks_ct_batch *in : {a, b})
    if (a->count && in->data != out->data && overlaps(in->data, words, out->data, words))
      return fail(CKKS_EINVAL, "product output overlaps an input other than exactly");
  const ckks_ct_batch av = *a;
  const uint64_t *bd = b->data;
  out->count = av.count;
  out->level = av.level;
  out->scale = ns;
  if (!av.count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  void *ws = nullptr;
  WsLease lease(ctx, st);
  HIP_TRY(lease.get(mul_scratch_words(av.count, (int)av.level, ctx->N) * sizeof(uint64_t), &ws), "workspace alloc");
  HIP_TRY(launch_mul(ctx, av.data, bd, out->data, av.count, (int)av.level, static_cast<uint64_t *>(ws), st), "mul");
  return CKKS_OK;
}

int ckks_mul_const(ckks_ctx *ctx, const ckks_ct_batch *a, double c, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_mul_const");
  int rc = check_ctx(ctx);
  if (rc || (rc = check_batch(ctx, a, "a"))) return rc;
  if ((rc = check_out(ctx, out, a->count, a->level))) return rc;
  std::vector<uint64_t> K;
  double ns = 0;
  if ((rc = const_multiplier(ctx, a->level, a->scale, c, K, &ns))) return rc;
  const ckks_ct_batch av = *a;
  out->count = av.count;
  out->level = av.level;
  out->scale = ns;
  if (!av.count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_mul_const(ctx, av.data, out->data, av.count, (int)av.level, K.data(), as_stream(stream)), "mul_const");
  return CKKS_OK;
}

int ckks_add_const(ckks_ctx *ctx, ckks_ct_batch *a, const double *d_b, double b, void *stream) {
  TraceRange trace_range_("ckks_add_const");
  int rc = check_ctx(ctx);
  if (rc || (rc = check_batch(ctx, a, "a"))) return rc;
  if (!d_b && !isfinite(b)) return fail(CKKS_EINVAL, "b is not finite");
  if (!a->count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_add_const(ctx, a->data, a->count, (int)a->level, a->scale, d_b, b, as_stream(stream)), "add_const");
  return CKKS_OK;
}

int ckks_rescale(ckks_ctx *ctx, const ckks_ct_batch *a, ckks_ct_batch *out, void *stream) {
  TraceRange trace_range_("ckks_rescale");
  int rc = check_ctx(ctx);
  if (rc || (rc = check_batch(ctx, a, "a"))) return rc;
  if (a->level < 2) return fail(CKKS_ELEVEL, "rescale needs level >= 2");
  if ((rc = check_out(ctx, out, a->count, a->level - 1))) return rc;
  const uint64_t nin = a->count * ct_words(ctx, a->level), nout = a->count * ct_words(ctx, a->level - 1);
  if (a->count && overlaps(a->data, nin, out->data, nout)) return fail(CKKS_EINVAL, "rescale output overlaps its input");
  const ckks_ct_batch av = *a;
  out->count = av.count;
  out->level = av.level - 1;
  out->scale = av.scale / (double)ctx->prm.q[av.level - 1];
  if (!av.count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_rescale(ctx, av.data, out->data, av.count, (int)av.level, as_stream(stream)), "rescale");
  return CKKS_OK;
}

int ckks_mean_filter(ckks_ctx *ctx, const ckks_ct_batch *img, uint32_t H, uint32_t W, uint32_t k, ckks_ct_batch *out,
                     void *stream) {
  TraceRange trace_range_("ckks_mean_filter");
  int rc = check_ctx(ctx);
  if (rc || (rc = check_batch(ctx, img, "img"))) return rc;
  if (k != 1 && k != 3 && k != 5 && k != 7) return fail(CKKS_EUNSUPPORTED, "window k must be 1, 3, 5 or 7");
  if (img->level < 2 || img->level > 8) return fail(CKKS_ELEVEL, "mean filter needs 2 <= level <= 8");
  if ((uint64_t)H * W != img->count) return fail(CKKS_EINVAL, "H*W (%llu) != count (%llu)", (unsigned long long)H * W, (unsigned long long)img->count);
  if ((rc = check_out(ctx, out, img->count, img->level - 1))) return rc;
  const uint64_t nin = img->count * ct_words(ctx, img->level), nout = img->count * ct_words(ctx, img->level - 1);
  if (img->count && overlaps(img->data, nin, out->data, nout)) return fail(CKKS_EINVAL, "filter output overlaps its input");
  std::vector<uint64_t> K;
  double s1 = 0;
  // 1/k^2 always in the scaled form rint(q_{level-1} / k^2), so the rescale restores the scale
  if ((rc = const_multiplier(ctx, img->level, img->scale, 1.0 / (double)(k * k), K, &s1, true))) return rc;
  const ckks_ct_batch iv = *img;
  out->count = iv.count;
  out->level = iv.level - 1;
  out->scale = s1 / (double)ctx->prm.q[iv.level - 1];
  if (!iv.count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_mean_filter(ctx, iv.data, out->data, H, W, 0, H, k, (int)iv.level, K.data(), as_stream(stream)),
          "mean filter");
  return CKKS_OK;
}

int ckks_decrypt_pixels(ckks_ctx *ctx, const ckks_ct_batch *in, double *d_out, void *stream) {
  TraceRange trace_range_("ckks_decrypt_pixels");
  int rc = check_keys(ctx);
  if (rc || (rc = check_batch(ctx, in, "in"))) return rc;
  if (in->count && !d_out) return fail(CKKS_EINVAL, "d_out is NULL");
  if (!in->count) return CKKS_OK;
  DeviceGuard g(ctx->device);
  HIP_TRY(launch_decrypt(ctx, in->data, in->count, (int)in->level, in->scale, d_out, in->level >= 2 ? 2 : 1,
                         as_stream(stream)),
          "decrypt");
  return CKKS_OK;
}

int ckks_stream_sync(ckks_ctx *ctx, void *stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  HIP_TRY(hipStreamSynchronize(as_stream(stream)), "stream synchronize");
  HIP_TRY(hipGetLastError(), "earlier launch");
  return CKKS_OK;
}

int ckks_stream_status(ckks_ctx *ctx, void *stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  const hipError_t q = hipStreamQuery(as_stream(stream));
  if (q == hipErrorNotReady) return CKKS_PENDING;
  HIP_TRY(q, "stream query");
  HIP_TRY(hipGetLastError(), "earlier launch");
  return CKKS_OK;
}

}  // extern "C"
