/* A C program using the library only through include/ckks_mi355x.h and the HIP runtime:
 * keys, plain and value-cached encryption of a 24 x 20 image, the 3x3 mean filter,
 * decryption, and the error path of a bad call.  Checks the decrypted pixels against the
 * plaintext filter and prints "OK" (run by tests/test_gpu_c_program.py). */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ckks_mi355x.h"

#define CHECK(c)                                                                  \
  do {                                                                            \
    if (!(c)) {                                                                   \
      fprintf(stderr, "FAILED %s at line %d: %s\n", #c, __LINE__, ckks_last_error()); \
      exit(1);                                                                    \
    }                                                                             \
  } while (0)

enum { H = 24, W = 20, K = 3 };

int main(void) {
  ckks_params prm = {12, 3, 36, 30, 3.2, 0, 0, NULL};
  ckks_ctx *ctx = NULL;
  CHECK(ckks_context_create(&prm, 0, &ctx) == CKKS_OK);
  const uint64_t key_seed[2] = {11, 12}, job[2] = {13, 14}, cache_seed[2] = {15, 16};
  CHECK(ckks_keygen(ctx, key_seed) == CKKS_OK);
  uint8_t px[H * W];
  for (int i = 0; i < H * W; i++) px[i] = (uint8_t)((i * 37 + i / W * 11) % 256);
  const uint64_t n = H * W, S = ckks_ct_bytes(ctx, 3), S2 = ckks_ct_bytes(ctx, 2);
  uint8_t *d_px = NULL;
  uint64_t *d_ct = NULL, *d_flt = NULL;
  double *d_dec = NULL;
  CHECK(hipMalloc((void **)&d_px, n) == hipSuccess);
  CHECK(hipMalloc((void **)&d_ct, n * S) == hipSuccess);
  CHECK(hipMalloc((void **)&d_flt, n * S2) == hipSuccess);
  CHECK(hipMalloc((void **)&d_dec, n * sizeof(double)) == hipSuccess);
  CHECK(hipMemcpy(d_px, px, n, hipMemcpyHostToDevice) == hipSuccess);
  /* plaintext 3x3 clamp-edge box filter */
  double box[H * W];
  for (int y = 0; y < H; y++)
    for (int x = 0; x < W; x++) {
      double s = 0;
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          int yy = y + dy < 0 ? 0 : (y + dy >= H ? H - 1 : y + dy);
          int xx = x + dx < 0 ? 0 : (x + dx >= W ? W - 1 : x + dx);
          s += px[yy * W + xx];
        }
      box[y * W + x] = s / 9.0;
    }
  ckks_cache_desc desc = {CKKS_CACHE_VALUE_TOPK, 0, 0, 16, 8};
  ckks_cache *cache = NULL;
  CHECK(ckks_cache_build(ctx, &desc, d_px, n, cache_seed, &cache, NULL) == CKKS_OK);
  for (int pass = 0; pass < 2; pass++) {
    ckks_ct_batch ct = {d_ct, n, 3, 0, 0.0};
    if (pass == 0)
      CHECK(ckks_encrypt_pixels(ctx, d_px, n, job, 0, &ct, NULL) == CKKS_OK);
    else
      CHECK(ckks_encrypt_cached(ctx, cache, d_px, n, job, 0, &ct, NULL) == CKKS_OK);
    CHECK(ct.count == n && ct.level == 3);
    ckks_ct_batch flt = {d_flt, n, 2, 0, 0.0};
    CHECK(ckks_mean_filter(ctx, &ct, H, W, K, &flt, NULL) == CKKS_OK);
    CHECK(flt.level == 2);
    CHECK(ckks_decrypt_pixels(ctx, &flt, d_dec, NULL) == CKKS_OK);
    CHECK(ckks_stream_sync(ctx, NULL) == CKKS_OK);
    double dec[H * W];
    CHECK(hipMemcpy(dec, d_dec, sizeof(dec), hipMemcpyDeviceToHost) == hipSuccess);
    double err = 0;
    for (int i = 0; i < H * W; i++) err = fmax(err, fabs(dec[i] - box[i]));
    CHECK(err < 1e-3);
  }
  /* an error path: a filter window that is not odd */
  ckks_ct_batch ct = {d_ct, n, 3, 0, 0.0}, flt = {d_flt, n, 2, 0, 0.0};
  ct.scale = flt.scale = 0.0;
  CHECK(ckks_encrypt_pixels(ctx, d_px, n, job, 0, &ct, NULL) == CKKS_OK);
  CHECK(ckks_mean_filter(ctx, &ct, H, W, 4, &flt, NULL) != CKKS_OK && ckks_last_error()[0] != 0);
  ckks_cache_destroy(cache);
  CHECK(hipFree(d_px) == hipSuccess && hipFree(d_ct) == hipSuccess && hipFree(d_flt) == hipSuccess &&
        hipFree(d_dec) == hipSuccess);
  ckks_context_destroy(ctx);
  printf("OK\n");
  return 0;
}
