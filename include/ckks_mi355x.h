/*
 * ckks_mi355x.h -- C ABI of the MI355X (gfx950) pixel-level CKKS library.
 *
 * Implements the data-parallel path of iCHEETAH (arXiv 2409.03568): per-pixel
 * CKKS encryption (Sec. 2.2.2), the cached encryption of Sec. 3.2 with the
 * randomness of Sec. 3.3, the homomorphic operations of Sec. 2.2.3 and the pixel
 * operations of Sec. 4.4 (mean filter, brightness), and decryption.
 *
 * General conventions
 *  - Every function returns an int status: CKKS_OK (0) or a negative CKKS_E*
 *    code; ckks_last_error() returns a thread-local message for the last failure.
 *    No C++ exception crosses this boundary.
 *  - Pointers whose name starts with d_ (and the data field of ckks_ct_batch) are
 *    DEVICE pointers on the context's GPU; host_ pointers are host memory.
 *  - Ownership: the caller owns every pixel, ciphertext and output buffer; the
 *    library owns the context, keys, tables and caches (freed by *_destroy).  No
 *    caller pointer is kept after the enqueued work has completed.
 *  - Asynchrony: compute calls validate their arguments synchronously, then
 *    enqueue on `stream` (a hipStream_t; NULL = the null stream) and return.
 *    Temporary device buffers of a call (cache metadata, tile buffers) are taken from
 *    a stream-ordered memory pool owned by the context, on the call's stream; the pool
 *    keeps freed memory for later calls and returns it when the context is destroyed.
 *    Calls on different streams may run concurrently once keys and caches exist;
 *    two calls writing the same buffer must be ordered by the caller.
 *  - Ciphertext layout (coefficient domain, canonical residues in [0, q_i)):
 *      data[ct][poly 0..1][limb 0..level-1][coefficient 0..N-1], uint64.
 *    A batch shares one level and one scale.
 *  - Output descriptors: on input, out->count is 0 (the caller vouches for the buffer's
 *    size) or the number of ciphertexts the buffer holds at level out->level (0 = the
 *    result's level); a buffer with fewer bytes than the result needs is CKKS_EINVAL
 *    before anything is enqueued.  On success count, level and scale describe the result.
 *  - Keys: ckks_keygen and ckks_keys_import replace the keys of a context.  Key-switching
 *    keys, caches, batch plans and servers made under the old keys are then invalid: the
 *    product needs a new ckks_relin_keygen, and the others return CKKS_ESTATE.
 *  - Determinism: ciphertext t of an encryption call equals the result for pixel
 *    index first_index + t computed alone, bit for bit, whatever the batch size,
 *    stream or tiling: all randomness comes from Philox4x64-10 (Salmon et al.,
 *    SC'11) keyed by the 2-word seed with counter (index, tag, block, 0).
 */
#ifndef CKKS_MI355X_H
#define CKKS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define CKKS_OK 0
#define CKKS_EINVAL (-1)        /* bad argument (null pointer, size, unsupported value) */
#define CKKS_ENOMEM (-2)        /* device allocation failed */
#define CKKS_ENOMEM_BUDGET (-3) /* request larger than a configured byte budget */
#define CKKS_EDEVICE (-4)       /* HIP runtime error (launch, copy, earlier asynchronous fault) */
#define CKKS_ELEVEL (-5)        /* operand levels differ, or level too low for the operation */
#define CKKS_ESCALE (-6)        /* operand scales differ */
#define CKKS_ECACHE (-7)        /* cache kind / descriptor mismatch, or pixel not representable */
#define CKKS_EUNSUPPORTED (-8)  /* parameter outside what the kernels implement */
#define CKKS_ESTATE (-9)        /* keys not generated or imported yet, or replaced since */
#define CKKS_ECANCELED (-10)    /* a server job was cancelled before it was admitted */
#define CKKS_EIO (-11)          /* a file could not be read or written */
#define CKKS_PENDING 1          /* ckks_stream_status: work is still running (not an error) */

typedef struct ckks_ctx ckks_ctx;
typedef struct ckks_cache ckks_cache;

/* CKKS parameters (Sec. 2.2, Table 1: ring dimension N, modulus Q, scale Delta;
 * Sec. 4.2 uses N = 2^12, Q ~ 2^109 and a ternary secret).
 *  log_n       N = 2^log_n; the kernels implement 11 <= log_n <= 14.
 *  num_primes  L, the number of RNS primes (1..16); Q = q_0 ... q_{L-1}.
 *  prime_bits  every q_i has exactly this many bits, 20 <= prime_bits <= 50
 *              (the modular arithmetic is exact FP64, which needs q < 2^50).
 *  log_scale   Delta = 2^log_scale.  Pixel coefficients must stay below q_{L-1}/2:
 *              256 * 2^(log_scale + 1 - log_n) < q_{L-1} is required.
 *  sigma       standard deviation of the discrete Gaussian errors (0 = no noise).
 *  gauss_bound tail cut B of the Gaussian; 0 selects floor(6 sigma).  B <= 63.
 *  primes      NULL selects the L largest primes below 2^prime_bits that are
 *              1 mod 2N, in descending order; otherwise L caller-chosen primes
 *              (each 1 mod 2N, exactly prime_bits bits, distinct), copied.      */
typedef struct ckks_params {
  uint32_t log_n;
  uint32_t num_primes;
  uint32_t prime_bits;
  uint32_t log_scale;
  double sigma;
  uint32_t gauss_bound;
  uint32_t reserved;
  const uint64_t *primes;
} ckks_params;

/* A batch of ciphertexts: data is a device pointer to count * ckks_ct_bytes(level) bytes. */
typedef struct ckks_ct_batch {
  uint64_t *data;
  uint64_t count;
  uint32_t level;
  uint32_t reserved;
  double scale;
} ckks_ct_batch;

/* Cache kinds of Sec. 3.2. */
#define CKKS_CACHE_RADIX 1      /* Enc(0) and Enc(r^i), i < digits; pixels combined from base-r digits */
#define CKKS_CACHE_VALUE_TOPK 2 /* scanning-based: the topk most frequent values of a scan image */
#define CKKS_CACHE_VALUE_FULL 3 /* full caching: Enc(v) for every v in 0..255 */

/* base, digits: radix caches (2 <= base <= 256, 2 <= digits <= 8, base^digits >= 256,
 *              base^(digits-1) <= 255; one digit is refused: the radix randomness of
 *              Sec. 3.3 draws one bit per radix above the lowest, so with a single digit
 *              every pixel value would map to one fixed ciphertext).
 * topk:        VALUE_TOPK (1..256).
 * zero_pool:   VALUE_* caches: size n of the pool of encrypted zeros added to every cached
 *              pixel (Sec. 3.3 randomness pool), 1..4096.                                  */
typedef struct ckks_cache_desc {
  int32_t kind;
  uint32_t base;
  uint32_t digits;
  uint32_t topk;
  uint32_t zero_pool;
} ckks_cache_desc;

/* ---- host-only queries (no GPU needed) ---- */

/* Message for the last failing call on this thread ("" if none). */
const char *ckks_last_error(void);

/* Resolve a parameter set without touching the GPU: writes the L primes that a
 * context would use to host_primes[L] and the Gaussian bound actually used to
 * *gauss_bound (either may be NULL).  Errors: CKKS_EINVAL, CKKS_EUNSUPPORTED. */
int ckks_params_resolve(const ckks_params *params, uint64_t *host_primes, uint32_t *gauss_bound);

/* Host tables a context would upload, for inspection:
 *   ckks_host_cdt_table: 2B cumulative thresholds of the Gaussian (Sec. 2.2.1 error
 *     distribution; sample = -B + #{k : w >= T[k]} for a Philox word w) -> host_out[2B];
 *   ckks_host_encode_table: T_j = 2^(log_scale+1-log_n) cos(pi j / N), j < N, the
 *     closed-form inverse embedding of a pixel placed in slot 0 (Sec. 2.2) -> host_out[N]. */
int ckks_host_cdt_table(const ckks_params *params, uint64_t *host_out, uint32_t capacity);
int ckks_host_encode_table(const ckks_params *params, double *host_out, uint64_t capacity);

/* ---- context ---- */

/* Create a context on HIP device `device`: computes primes, roots of unity, NTT
 * twiddles and the encoding / Gaussian tables and uploads them.  *out receives the
 * context (owned by the library).  Errors: CKKS_EINVAL, CKKS_EUNSUPPORTED,
 * CKKS_ENOMEM, CKKS_EDEVICE. */
int ckks_context_create(const ckks_params *params, int device, ckks_ctx **out);
/* Wait for all work of the context and free it.  NULL is ignored. */
void ckks_context_destroy(ckks_ctx *ctx);

/* Tuning of the NTT kernels (encryption, decryption, keys, ciphertext product): each
 * thread of a workgroup holds values_per_thread ring coefficients (8, 16 or 32), so a
 * workgroup has N / values_per_thread threads (at most 1024: 8 needs N <= 8192).  The
 * setter applies to all of them (ckks_autotune chooses per kernel); the getter reports
 * the encryption kernel's.  Results are identical for every setting; only speed differs.
 * CKKS_EINVAL for other values.  The default is 8 where allowed, else 16. */
int ckks_context_set_ntt_width(ckks_ctx *ctx, uint32_t values_per_thread);
int ckks_context_get_ntt_width(const ckks_ctx *ctx, uint32_t *values_per_thread);

/* Bytes of one ciphertext at `level` (2 * level * N * 8); 0 for a bad level. */
uint64_t ckks_ct_bytes(const ckks_ctx *ctx, uint32_t level);
/* Context parameters: N, L, Delta and the primes (host_primes[L], may be NULL). */
int ckks_context_info(const ckks_ctx *ctx, uint32_t *log_n, uint32_t *num_primes, double *scale,
                      uint64_t *host_primes);

/* ---- keys (Sec. 2.2.2, key generation steps 1-2) ---- */

/* Generate s (ternary), e (Gaussian), a_i (uniform mod q_i) from Philox keyed by seed
 * (counter index 0; tags 16, 17, 32+i) and set pk = (-a*s + e, a), on the GPU.
 * Synchronous: returns after the keys are ready.  The key-switching keys of the
 * ciphertext product are generated separately (ckks_relin_keygen). */
int ckks_keygen(ckks_ctx *ctx, const uint64_t seed[2]);
/* Copy the keys out: host_s[N] (int64 in {-1,0,1}), host_pk[2][L][N]. Either may be NULL. */
int ckks_keys_export(ckks_ctx *ctx, int64_t *host_s, uint64_t *host_pk);
/* Install keys produced elsewhere (s[N] in {-1,0,1}; pk[2][L][N] canonical residues). */
int ckks_keys_import(ckks_ctx *ctx, const int64_t *host_s, const uint64_t *host_pk);

/* Key-switching keys of s^2 for relinearization (Sec. 2.2.3, hybrid key switching
 * with one special prime qP and one digit per limb).  qP is the largest prime
 * congruent to 1 mod 2N below 2^bits that is not one of the q_i.  Key i (i < L), in
 * each prime p_j of q_0..q_{L-1}, qP (j = L):
 *   b_ij = -a_ij * s + e_i + [j == i] (qP mod q_i) s^2 (mod p_j),  a_ij uniform mod p_j,
 * with e_i Gaussian from Philox (seed, 0, 48 + i) and a_ij by rejection from
 * (seed, 0, 64 + 32 i + j) as in ckks_keygen.  Requires keys (CKKS_ESTATE);
 * CKKS_EUNSUPPORTED if no such qP exists.  Synchronous; allocates the keys on first
 * use (2 * L * (L+1) * 2 * N * 8 bytes with their NTT-domain copies). */
int ckks_relin_keygen(ckks_ctx *ctx, const uint64_t seed[2]);
/* Copy the key-switching keys out as host_evk[L][L+1][2][N] (b then a; canonical
 * residues) and the special prime.  Either pointer may be NULL.  CKKS_ESTATE without
 * ckks_relin_keygen. */
int ckks_relin_keys_export(ckks_ctx *ctx, uint64_t *host_evk, uint64_t *host_special_prime);

/* ---- encryption ---- */

/* Plain per-pixel encryption (Sec. 2.2.2): for t < n, with v ternary and e0, e1
 * Gaussian drawn from Philox keyed by seed at counter index first_index + t (tags 1,
 * 2, 3), and m the slot-0 encoding of pixel d_px[t] at scale Delta:
 *   c0 = v*pk0 + e0 + m,  c1 = v*pk1 + e1   (mod q_i, every limb).
 * out->data must hold n ciphertexts of level L; on success out->count = n,
 * out->level = L, out->scale = Delta.  n = 0 is a no-op. */
int ckks_encrypt_pixels(ckks_ctx *ctx, const uint8_t *d_px, uint64_t n, const uint64_t seed[2],
                        uint64_t first_index, ckks_ct_batch *out, void *stream);

/* Build a cache (Sec. 3.2) under cache_seed:
 *  RADIX:      entries Enc(0) (index 0) and Enc(base^i) (index 1+i), i < digits;
 *  VALUE_TOPK: histogram of d_scan[n_scan] on the GPU, the topk most frequent values
 *              (count descending, value ascending, only values that occur), each
 *              Enc(v) at index 256+v;
 *  VALUE_FULL: Enc(v) at index 256+v for all 256 values (d_scan ignored);
 *  VALUE_*:    a pool of zero_pool encrypted zeros, member u at index 512+u.
 * Entries are plain encryptions exactly as ckks_encrypt_pixels computes them.  The
 * call enqueues on `stream`; the cache is usable by later work on the same stream
 * (synchronize before using it on another stream).  *out owns the device memory. */
int ckks_cache_build(ckks_ctx *ctx, const ckks_cache_desc *desc, const uint8_t *d_scan, uint64_t n_scan,
                     const uint64_t cache_seed[2], ckks_cache **out, void *stream);
void ckks_cache_destroy(ckks_cache *cache);
/* Number of cached value entries (RADIX: digits + 1; VALUE_FULL: 256; VALUE_TOPK: the
 * number of distinct values kept, which waits for the build on the stream). */
int ckks_cache_entries(ckks_cache *cache, uint32_t *n_entries);
/* Copy a built cache to host memory (waits for the build).  host_values[n] receives the
 * plaintext value of each entry and host_entries[n][2][L][N] the entries, n as reported by
 * ckks_cache_entries (RADIX: entry 0 is Enc(0), entry 1+i is Enc(base^i)); host_pool
 * receives the zero_pool encrypted zeros of a value cache.  Any pointer may be NULL. */
int ckks_cache_export(ckks_cache *cache, uint32_t *host_values, uint64_t *host_entries, uint64_t *host_pool);
/* Install a cache built elsewhere -- full caching is prepared offline (Sec. 3.2), so a
 * cache exported earlier (or computed by another implementation) can be loaded instead of
 * rebuilt.  desc gives the kind and its parameters as for ckks_cache_build;
 * host_values[n_entries] and host_entries[n_entries][2][L][N] are laid out as
 * ckks_cache_export writes them (RADIX: n_entries = digits + 1 with values 0, 1, base, ...;
 * VALUE_FULL: 256 entries with values 0..255; VALUE_TOPK: 1..topk distinct values);
 * host_pool[zero_pool][2][L][N] holds a value cache's encrypted zeros (NULL for RADIX).
 * The entries must be encryptions under the context's current keys (the library cannot
 * check that); residues must be canonical (CKKS_EINVAL).  Synchronous: the data are
 * copied to device memory owned by the new cache before the call returns. */
int ckks_cache_import(ckks_ctx *ctx, const ckks_cache_desc *desc, uint32_t n_entries, const uint32_t *host_values,
                      const uint64_t *host_entries, const uint64_t *host_pool, ckks_cache **out);

/* Cached encryption of pixel d_px[t], index first_index + t, under the job seed:
 *  RADIX (Sec. 3.2 + 3.3): c = Enc(0) + sum_i d_i Enc(base^i) over the base-`base`
 *    digits d_i of the pixel, then for i = 1..digits-1, if bit i-1 of auxiliary
 *    Philox word 1 (tag 4) is set, c += Enc(base^i) - base * Enc(base^(i-1)).
 *  VALUE_* (Sec. 3.2 + 3.3): a cached value p gives c = Enc(p) + Z_u with
 *    u = floor(zero_pool * w / 2^64), w = auxiliary word 0; a value that is not
 *    cached is encrypted in full exactly like ckks_encrypt_pixels.
 * Output as for ckks_encrypt_pixels.  Its per-pixel metadata goes to a scratch buffer
 * that the context keeps for this stream (see "Per-stream scratch" below). */
int ckks_encrypt_cached(ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint64_t n,
                        const uint64_t seed[2], uint64_t first_index, ckks_ct_batch *out, void *stream);

/* The same cached encryption for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): it calls no
 * hipMalloc, hipFree or allocating routine.  Its per-pixel metadata lives in a fixed
 * device array of 32 MiB that the library holds on each GPU it runs on until the process
 * ends (ckks_encrypt_cached_noalloc_max_pixels gives the largest n for a cache: about
 * 2.7 million pixels for a value cache, 2 million for a radix cache); a larger n is
 * CKKS_ENOMEM_BUDGET before anything is enqueued.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (on different streams, or from different
 * threads without ordering) race and may produce wrong ciphertexts: order them.  Results
 * equal ckks_encrypt_cached bit for bit. */
int ckks_encrypt_cached_noalloc(ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint64_t n,
                                const uint64_t seed[2], uint64_t first_index, ckks_ct_batch *out, void *stream);
uint64_t ckks_encrypt_cached_noalloc_max_pixels(const ckks_cache *cache);

/* ---- homomorphic operations (Sec. 2.2.3) ---- */

/* out = a + b (ckks_add) or a - b (ckks_sub), residue-wise.  a and b must have the
 * same count and level (CKKS_ELEVEL) and exactly equal scales (CKKS_ESCALE).  out->data
 * may alias a->data or b->data; out->count/level/scale are set. */
int ckks_add(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out, void *stream);
int ckks_sub(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out, void *stream);

/* Relinearized product out = a * b (Sec. 2.2.3; the squared difference of image
 * matching, Sec. 4.4.3), ciphertext by ciphertext:
 *   (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1) in each q_j;
 *   acc = sum_i d2_i * key_i in q_0..q_{level-1} and qP, d2_i the limb-i residues taken
 *         as integers in [0, q_i);
 *   out_k = d_k + (acc_k - [acc_k]_qP) * qP^-1 (mod q_j), [.]_qP the centered residue.
 * a and b must have the same count and level (CKKS_ELEVEL); scales may differ and
 * out->scale = a->scale * b->scale at the same level (ckks_rescale brings it back).
 * Requires ckks_relin_keygen (CKKS_ESTATE).  out->data may equal a->data or b->data;
 * any other overlap is CKKS_EINVAL.  Uses min(count, 2048) * (2 level + 2) * N * 8
 * bytes of scratch that the context keeps for this stream (see "Per-stream scratch"
 * below). */
int ckks_mul(ckks_ctx *ctx, const ckks_ct_batch *a, const ckks_ct_batch *b, ckks_ct_batch *out, void *stream);

/* Per-stream scratch (ckks_encrypt_cached, ckks_mul): the context keeps one device buffer
 * for each stream these calls were given, so that calls queued on a stream reuse it
 * without waiting on the host.  A buffer grows (by 1.5x, in 2 MiB steps) when a call
 * needs more; growing first waits on the host for that stream's previous use.  Buffers
 * of at most 16 streams are kept: a call on a further stream first releases the least
 * recently used one, after waiting on the host for its last use.  All are freed by
 * ckks_context_destroy.  Calls that enqueue on one context are serialized on the host
 * for the short time they enqueue. */

/* out = c * a.  An integer-valued c multiplies exactly and keeps the scale; any other c
 * multiplies by K = rint(c * q_{level-1}) and sets out->scale = a->scale * q_{level-1}, so
 * that ckks_rescale restores the scale.  out->data may alias a->data. */
int ckks_mul_const(ckks_ctx *ctx, const ckks_ct_batch *a, double c, ckks_ct_batch *out, void *stream);

/* In place: add the plaintext b, encoded like a pixel (slot 0) at the batch's scale,
 * m_j = rint(((b * scale) * 2^(1-log_n)) * cos(pi j / N)), to c0 of every ciphertext.
 * d_b (nullable) gives one b per ciphertext; otherwise the scalar b is used.
 * Brightness (Sec. 4.4.2) and the watermark (Sec. 4.4.4). */
int ckks_add_const(ckks_ctx *ctx, ckks_ct_batch *a, const double *d_b, double b, void *stream);

/* Rescale (Sec. 2.2.3): divide by q = q_{level-1} with rounding, floor((x + floor(q/2)) / q),
 * and drop that limb; out->level = level - 1, out->scale = scale / q.  CKKS_ELEVEL if
 * level < 2.  out->data must not overlap a->data. */
int ckks_rescale(ckks_ctx *ctx, const ckks_ct_batch *a, ckks_ct_batch *out, void *stream);

/* ---- image operations (Sec. 4.4) ---- */

/* k x k mean filter (Sec. 4.4.1) of an H x W image of ciphertexts in row-major order
 * (img->count == H * W): out(y,x) = rescale(K * sum of in(clamp(y+dy), clamp(x+dx)) over
 * |dy|, |dx| <= k/2), borders clamped to the edge, with 1/k^2 represented as
 * K = rint(q_{level-1} / k^2) at scale * q_{level-1}, so out->scale = img->scale.  For k > 1
 * this is bit-identical to the k^2 - 1 additions, ckks_mul_const(1/k^2) and ckks_rescale.  k in {1, 3, 5, 7}; 2 <= level <= 8
 * (CKKS_EUNSUPPORTED / CKKS_ELEVEL otherwise).  out has level - 1; out->data must not
 * overlap img->data. */
int ckks_mean_filter(ckks_ctx *ctx, const ckks_ct_batch *img, uint32_t H, uint32_t W, uint32_t k,
                     ckks_ct_batch *out, void *stream);

/* ---- decryption (Sec. 2.2.2) ---- */

/* d_out[t] = slot 0 of decode(c0 + c1*s) (Sec. 2.2.2 decryption): sum_j x_j cos(pi j/N) / scale,
 * where x_j is the centered integer of the decrypted coefficient j.  At level >= 2 x_j is
 * the CRT lift of limbs 0 and 1, x_j = x0_j + q_0 k_j with x0_j centered mod q_0 and
 * k_j = [(d1_j - x0_j) q_0^-1] centered mod q_1: exact while every |x_j| < q_0 q_1 / 2, so a
 * coefficient past q_0/2 (a sum of a few hundred pixels at N = 4096, Delta = 2^30)
 * still decodes correctly.  At level 1 only limb 0 exists: exact while |x_j| < q_0/2,
 * which the library cannot check.  d_out is a device double[count]. */
int ckks_decrypt_pixels(ckks_ctx *ctx, const ckks_ct_batch *in, double *d_out, void *stream);

/* ---- streams ---- */

/* Wait for all work enqueued on `stream` and report any asynchronous device error. */
int ckks_stream_sync(ckks_ctx *ctx, void *stream);
/* Non-blocking: CKKS_OK when all work enqueued on `stream` has completed, CKKS_PENDING (a
 * positive value) while some is still running, CKKS_EDEVICE for an asynchronous device
 * error. */
int ckks_stream_status(ckks_ctx *ctx, void *stream);

/* ---- autotuning ----
 * Times the NTT kernels (encryption, Sec. 2.2.2: one forward and two inverse
 * transforms per limb; decryption: one forward and one inverse on limb 0) at each
 * supported register blocking (8, 16 or 32 values per thread) on trial_cts synthetic
 * ciphertexts, and, once ckks_relin_keygen has run, the relinearized product
 * (Sec. 2.2.3) of trial_cts pairs; keeps the fastest width for each kernel on this
 * context.  Then times the launch shapes of the HBM-bound kernels: the row-wise
 * kernels (ciphertext addition, Sec. 2.2.3, standing for every row-wise kernel:
 * subtraction, constants, rescaling, radix gather) at 0 (one workgroup per row), 2, 4,
 * 8 and 16 workgroups per compute unit, and the value-cache gather (Sec. 3.2) at 2, 4,
 * 8, 16 and 32, on trial_cts synthetic ciphertexts; keeps the fastest of each.  Reports
 * every timing.  The choices change speed only, never results.  Enqueues on the null
 * stream and synchronizes; allocates and frees its own scratch buffers.
 */
typedef struct {
  uint32_t encrypt_width, decrypt_width;  /* chosen values per thread */
  uint32_t trial_cts, mul_width;          /* mul_width 0: product not timed (no keys) */
  double encrypt_ms[3], decrypt_ms[3];    /* best of 3 runs: [0] 8, [1] 16, [2] 32 values per thread */
  double mul_ms[3];                       /* the same for the product (INFINITY if not timed) */
  uint32_t row_wgs_per_cu, gather_wgs_per_cu; /* chosen launch shapes */
  double row_ms[5];                       /* best of 3 runs at 0, 2, 4, 8, 16 workgroups per CU */
  double gather_ms[5];                    /* best of 3 runs at 2, 4, 8, 16, 32 workgroups per CU */
} ckks_tune_report;

int ckks_autotune(ckks_ctx *ctx, uint32_t trial_cts, ckks_tune_report *out);

/* Launch shapes of the HBM-bound kernels, in workgroups per compute unit: row_wgs for
 * the row-wise kernels (0..64; 0 = one workgroup per ciphertext row, the default) and
 * gather_wgs for the value-cache gather (1..64; default 8).  Results are identical for
 * every setting.  CKKS_EINVAL outside those ranges. */
int ckks_context_set_launch_shapes(ckks_ctx *ctx, uint32_t row_wgs, uint32_t gather_wgs);
int ckks_context_get_launch_shapes(const ckks_ctx *ctx, uint32_t *row_wgs, uint32_t *gather_wgs);

/* Persistence of the tuned settings (the three register blockings and the two launch
 * shapes) in a text file at `path`, one line per (device architecture, compute units,
 * log N, number of primes): ckks_tune_save writes this context's current settings,
 * replacing its line or adding one and keeping the others (written to a temporary file
 * and renamed, so a concurrent reader sees the old file or the new one; concurrent
 * writers may lose each other's lines).  ckks_tune_load applies the line that matches
 * this context and sets *found to 1, or leaves the settings and sets *found to 0 when
 * the file or the line is absent.  Errors: CKKS_EINVAL (NULL arguments, or a matching
 * line with settings this context does not support), CKKS_EIO (file not readable or
 * writable; the message names the system error). */
int ckks_tune_save(const ckks_ctx *ctx, const char *path);
int ckks_tune_load(ckks_ctx *ctx, const char *path, int *found);

/* ---- batched images ----
 * Encrypts many images packed in one flat pixel array (image i = pixels
 * [seg_end[i-1], seg_end[i])), adds each image's brightness constant b_i
 * (add_const, Sec. 4.4.2: encode(b_i) in slot 0 of c0), and decrypts every ciphertext
 * (Sec. 2.2.2) -- the batched form of encrypt -> brighten -> decrypt.  Ciphertexts are
 * written, each in full (all limbs) before it is decrypted, into a ring buffer of
 * chunk_cts ciphertexts owned by the plan, so device memory stays bounded whatever the
 * batch size.  The cache metadata of the whole batch comes first, so hits are grouped by
 * pool member and cache slot over all images (each pair's entries are read from L2 for
 * all its pixels); then one persistent launch assembles every ciphertext -- entry + pool
 * member for a cached value, full encryption for a miss or for every pixel without a
 * cache -- with the brightness fused in, writes it to the ring (a workgroup reuses its
 * slots in turn) and decrypts it from the registers that hold its limb-0 rows.  With a
 * VALUE_FULL cache the launch has no encryption path and needs only the decryption's LDS
 * and registers, so several workgroups share a CU.  (Where limb 0 alone does not decode
 * exactly, chunks of chunk_cts ciphertexts are produced and then decrypted from the ring
 * with the two-limb lift.)  Ciphertexts equal ckks_encrypt_cached / ckks_encrypt_pixels
 * followed by ckks_add_const, bit for bit; the decrypted values equal ckks_decrypt_pixels
 * of those ciphertexts bit for bit when the context's encryption and decryption use the
 * same NTT width (the decoded sum's rounding follows the workgroup shape), otherwise to a
 * few units in the last place.  A plan runs one batch at a time.
 * With use_graph, the whole chunk sequence is captured once into a HIP graph and
 * replayed while ckks_batch_run is called again with the same arguments.
 */
typedef struct ckks_batch_plan ckks_batch_plan;

typedef struct {
  uint64_t chunk_cts;  /* ciphertexts per ring-buffer chunk (>= 1) */
  uint32_t use_graph;  /* 1 = capture the chunk sequence in a HIP graph and replay it */
  uint32_t reserved;
} ckks_batch_config;

/* cache: a VALUE_TOPK / VALUE_FULL cache of ctx, or NULL for plain encryption. */
int ckks_batch_plan_create(ckks_ctx *ctx, const ckks_cache *cache, const ckks_batch_config *cfg,
                           ckks_batch_plan **out);

/* d_px: n pixels (device).  host_seg_end: n_seg ascending image ends, the last = n.
 * host_seg_b: n_seg brightness constants, |b * scale * 2^(1 - log N)| < 2^50.
 * d_out: n doubles (device), the decrypted pixel + b values.  Ciphertext t uses Philox
 * index first_index + t.  cts_out (nullable): when given, its data (device memory for n
 * ciphertexts of level L; count/level as for other outputs) receives every brightened
 * ciphertext instead of the plan's ring buffer, and count/level/scale are set.
 * Decryption decodes limb 0 when a worst-case bound on the coefficients of a pixel plus
 * brightness (with the encryption errors bounded by the Gaussian tail cut) stays below
 * q_0/2, as it does at every configured parameter set, else the two-limb lift of
 * ckks_decrypt_pixels.  Enqueued on `stream`.  CKKS_ESTATE if the keys changed after the
 * plan was made. */
int ckks_batch_run(ckks_batch_plan *plan, const uint8_t *d_px, uint64_t n, const uint64_t *host_seg_end,
                   const double *host_seg_b, uint32_t n_seg, const uint64_t seed[2], uint64_t first_index,
                   double *d_out, ckks_ct_batch *cts_out, void *stream);

void ckks_batch_plan_destroy(ckks_batch_plan *plan);

/* ---- streamed image pipeline ----
 * Encrypts an H x W image (plain, or with a radix / value cache, Sec. 2.2.2 / Sec. 3.2),
 * applies the k x k clamp-edge mean filter (Sec. 4.4.1) and decrypts, in tiles of
 * tile_rows output rows, so that only a few tiles of ciphertexts exist at any time.
 * streams = 1 (the faster mode) runs the tiles one after another on the caller's stream
 * and keeps the encrypted rows in a ring of tile_rows + 2 (k/2) rows: each tile encrypts
 * only the rows it adds, so every pixel is encrypted once.  With streams = 3, encryption,
 * filtering and decryption run on three streams of the context with two buffers per
 * stage, so tile t+1 can be encrypted while tile t is filtered and tile t-1 decrypted;
 * each tile then encrypts its k/2 halo rows above and below again (the same ciphertexts
 * as a whole-image encryption, since every ciphertext depends only on its pixel and
 * global index), and the caller's stream waits for all of it.  Results
 * equal ckks_encrypt_* -> ckks_mean_filter -> ckks_decrypt_pixels on the whole image, bit
 * for bit.  Tile buffers come from the context's scratch pool on the caller's stream.
 * Calls on one context with streams = 3 must not overlap (they share the stage streams).
 */
typedef struct {
  uint32_t tile_rows;  /* output rows per tile (>= 1) */
  uint32_t streams;    /* 1 or 3 */
  uint32_t filter_k;   /* 1, 3, 5 or 7 */
  uint32_t reserved;
} ckks_pipeline_config;

/* d_px: H*W pixels; d_out: H*W doubles (decrypted filtered pixels); both device. */
int ckks_image_pipeline(ckks_ctx *ctx, const ckks_cache *cache, const uint8_t *d_px, uint32_t H, uint32_t W,
                        const uint64_t seed[2], uint64_t first_index, const ckks_pipeline_config *cfg, double *d_out,
                        void *stream);

/* ---- serving runtime ----
 * A server runs whole image jobs -- encrypt every pixel (plain or cached, Sec. 2.2.2 /
 * Sec. 3.2), apply the k x k mean filter (Sec. 4.4.1), decrypt (Sec. 2.2.2) -- for
 * requests that arrive while earlier ones are still on the GPU.  A dispatcher thread
 * owned by the server admits queued jobs in arrival order as soon as one of
 * `max_inflight` slots (each a HIP stream of its own) is free and a contiguous range of
 * the job's device bytes is free in the server's arena (one device allocation of
 * `hbm_budget_bytes` made at creation).  While the oldest queued job waits for arena
 * space, younger jobs that fit may start ahead of it, at most `max_bypass` of them per
 * queued job (0 = strict arrival order), so no job waits forever.  Admitted jobs run
 * concurrently on their streams.
 * A job runs in row tiles (as ckks_image_pipeline with one stream): its device bytes
 * (ckks_job_bytes) are its pixels, its decrypted values and the buffers of one tile -- a
 * ring of tile + 2 (k/2) encrypted rows, the filtered rows, cache metadata -- with the
 * tile height the largest whose buffers fit `tile_bytes` (0 = the whole image as one
 * tile), so a large image does not hold most of the arena while smaller jobs wait.  A
 * job's results do not depend on which other jobs run beside it, nor on the tiling: its
 * ciphertexts are fixed by (job_seed, first_index), and every kernel's result is
 * independent of the launch that computes it.
 */
typedef struct ckks_server ckks_server;

typedef struct {
  uint64_t hbm_budget_bytes;  /* arena size; jobs larger than this are refused at submission */
  uint32_t max_inflight;      /* slots (streams), 1..64 */
  uint32_t filter_k;          /* mean-filter window: 1, 3, 5, 7; 0 = no filter (decrypt the encryption) */
  const ckks_cache *cache;    /* cache for encryption, NULL = plain encryption; must outlive the server */
  uint64_t max_job_pixels;    /* pinned staging sized for this many pixels per slot at creation (0 = on demand) */
  uint64_t tile_bytes;        /* cap on one job's tile buffers (0 = whole image) */
  uint32_t max_bypass;        /* younger jobs that may start ahead of a waiting one (0 = none) */
  uint32_t reserved;          /* 0 */
} ckks_server_config;

typedef struct {
  uint64_t job_id;
  int32_t status;             /* CKKS_OK or the CKKS_E* code of the failed step */
  uint32_t height, width;
  double t_submit_us;         /* host steady clock, microseconds since the server was created */
  double t_admit_us;
  double t_done_us;           /* when the dispatcher saw the job's last copy complete */
  double gpu_ms;              /* device time from the job's first to its last operation */
} ckks_job_result;

typedef struct {
  uint64_t submitted, completed, failed, queued, inflight;
  uint64_t arena_bytes, inflight_bytes, peak_inflight_bytes;
  uint32_t peak_inflight_jobs, reserved;
  uint64_t canceled;
  uint64_t backfilled;        /* jobs started ahead of an older waiting job */
} ckks_server_stats;

/* Creates a server and starts its dispatcher.  Needs keys on ctx; ctx (and cache) must
 * outlive the server.  ENOMEM if the arena cannot be allocated. */
int ckks_server_create(ckks_ctx *ctx, const ckks_server_config *cfg, ckks_server **out);

/* Queues one job of H*W pixels (host_px, row-major uint8).  host_px is copied before the
 * call returns; host_out (H*W doubles, the decrypted filtered pixels) must stay valid
 * until the job's result has been returned by ckks_server_poll.  Ciphertext t uses Philox
 * index first_index + t under job_seed.  ENOMEM_BUDGET if the job can never fit. */
int ckks_server_submit(ckks_server *srv, const uint8_t *host_px, uint32_t H, uint32_t W, const uint64_t job_seed[2],
                       uint64_t first_index, double *host_out, uint64_t *job_id);

/* Arena bytes a job of H x W pixels takes in a server with this cache, filter window and
 * tile_bytes (0 for H*W = 0 or a NULL context). */
uint64_t ckks_job_bytes(const ckks_ctx *ctx, const ckks_cache *cache, uint32_t H, uint32_t W, uint32_t filter_k,
                        uint64_t tile_bytes);

/* Cancels a job that is still queued: it is never admitted, and ckks_server_poll returns
 * it with status CKKS_ECANCELED.  CKKS_ESTATE if it has already been admitted (it then
 * runs to completion), CKKS_EINVAL for an unknown id. */
int ckks_server_cancel(ckks_server *srv, uint64_t job_id);

/* Failure injection, for testing a client's failure handling: when the (still queued) job
 * is admitted, none of its work is enqueued and it finishes with `status` (a negative
 * CKKS_E* code), as if one of its steps had failed; the jobs beside it are unaffected.
 * CKKS_ESTATE if the job is not queued. */
int ckks_server_inject_failure(ckks_server *srv, uint64_t job_id, int32_t status);

/* Returns up to `max` finished jobs (oldest first), waiting up to wait_ms milliseconds
 * (0 = do not wait, negative = until at least one is available or nothing is pending). */
int ckks_server_poll(ckks_server *srv, ckks_job_result *out, uint32_t max, uint32_t *n_out, int32_t wait_ms);

/* Blocks until every submitted job has finished (results stay available to poll). */
int ckks_server_drain(ckks_server *srv);

int ckks_server_stats_get(ckks_server *srv, ckks_server_stats *out);

/* Stops the dispatcher after the running jobs finish; queued jobs are dropped. */
void ckks_server_destroy(ckks_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* CKKS_MI355X_H */
