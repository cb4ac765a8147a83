/* Runs every oracle entry point once at small sizes, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py).  Checks a few results on the
 * way, but its purpose is to exercise the code paths under the sanitizers; prints "OK". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/ckks_oracle.h"

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__); \
      exit(1);                                                 \
    }                                                          \
  } while (0)

static void run(int log_n, int L, int bits, int log_scale) {
  orc_params P;
  CHECK(orc_params_init(&P, log_n, L, bits, log_scale, 3.2, 0, NULL) == 0);
  const int N = 1 << log_n;
  const size_t S = (size_t)2 * L * N;
  const uint64_t seed[2] = {1, 2}, job[2] = {3, 4}, cs[2] = {5, 6};
  int64_t *s = malloc(sizeof(int64_t) * N);
  uint64_t *pk = malloc(sizeof(uint64_t) * 2 * L * N);
  orc_keygen(&P, seed, s, pk);
  uint64_t *a = malloc(sizeof(uint64_t) * S), *b = malloc(sizeof(uint64_t) * S), *c = malloc(sizeof(uint64_t) * S);
  orc_encrypt(&P, pk, 200.0, job, 7, a);
  orc_encrypt(&P, pk, 50.0, job, 8, b);
  int err = 0;
  CHECK(orc_decrypt(&P, s, a, L, (double)(1ull << log_scale), &err) > 199.0 && err == 0);
  orc_add(&P, a, b, c, L);
  orc_sub(&P, a, b, c, L);
  double sc = 0;
  CHECK(orc_mul_const(&P, a, L, (double)(1ull << log_scale), 0.25, c, &sc) == 0);
  uint64_t *r = malloc(sizeof(uint64_t) * S);
  double sc2 = 0;
  CHECK(orc_rescale(&P, c, L, sc, r, &sc2) == 0);
  CHECK(orc_add_const(&P, a, L, (double)(1ull << log_scale), 3.0) == 0);
  uint64_t *d = malloc(sizeof(uint64_t) * L * N);
  int64_t *x = malloc(sizeof(int64_t) * N);
  orc_decrypt_coeffs(&P, s, a, L, d);
  CHECK(orc_decode_centered(&P, d, L, x) == 0);
  /* caches */
  uint64_t *ent = malloc(sizeof(uint64_t) * 3 * S);
  orc_radix_entries(&P, pk, 16, 2, cs, ent);
  CHECK(orc_radix_encrypt(&P, ent, 16, 2, 255, job, 9, c) == 0);
  uint8_t px[64];
  for (int i = 0; i < 64; i++) px[i] = (uint8_t)(i * 37 % 11);
  uint64_t h[256];
  orc_histogram(px, 64, h);
  int vals[256];
  const int nv = orc_topk(h, 8, vals);
  CHECK(nv == 8);
  uint64_t *pool = malloc(sizeof(uint64_t) * 2 * S);
  orc_pool_entry(&P, pk, 0, cs, pool);
  orc_pool_entry(&P, pk, 1, cs, pool + S);
  orc_value_entry(&P, pk, vals[0], cs, b);
  orc_value_encrypt(&P, pk, b, pool, 2, vals[0], job, 10, c);
  orc_value_encrypt(&P, pk, NULL, pool, 2, 99, job, 11, c);
  /* batch encryption, filter, batch decryption */
  uint64_t *img = malloc(sizeof(uint64_t) * 12 * S);
  orc_encrypt_batch(&P, pk, px, 12, job, 0, img);
  for (int k = 1; k <= 5; k += 2)
    for (int y = 0; y < 3; y++)
      for (int xx = 0; xx < 4; xx++)
        CHECK(orc_mean_filter_pixel(&P, img, 3, 4, L, (double)(1ull << log_scale), k, y, xx, c, &sc) == 0);
  double dec[12];
  int nerr = 0;
  orc_decrypt_batch(&P, s, img, 12, L, (double)(1ull << log_scale), dec, &nerr);
  CHECK(nerr == 0);
  /* product with relinearization */
  if (P.qP) {
    uint64_t *evk = malloc(sizeof(uint64_t) * (size_t)L * (L + 1) * 2 * N);
    orc_relin_keygen(&P, s, seed, evk);
    uint64_t *tens = malloc(sizeof(uint64_t) * 3 * L * N);
    orc_tensor(&P, a, a, L, tens);
    uint64_t *acc = malloc(sizeof(uint64_t) * 2 * (L + 1) * N);
    orc_key_switch(&P, evk, tens + (size_t)2 * L * N, L, acc);
    orc_mod_down(&P, acc, L, c);
    orc_mul(&P, evk, a, b, L, c);
    free(evk);
    free(tens);
    free(acc);
  }
  /* transforms and samplers */
  uint64_t *u = malloc(sizeof(uint64_t) * N), *v = malloc(sizeof(uint64_t) * N), *w = malloc(sizeof(uint64_t) * N);
  orc_sample_uniform(seed, 0, 40, N, P.q[0], u);
  orc_sample_uniform(seed, 1, 40, N, P.q[0], v);
  orc_negacyclic_mul(u, v, w, N, P.q[0], P.psi[0]);
  uint64_t *w2 = malloc(sizeof(uint64_t) * N);
  orc_negacyclic_schoolbook(u, v, w2, N, P.q[0]);
  CHECK(memcmp(w, w2, sizeof(uint64_t) * N) == 0);
  int64_t *g = malloc(sizeof(int64_t) * N);
  orc_sample_gauss(&P, seed, 0, 2, g);
  orc_sample_ternary(seed, 0, 1, N, g);
  double *T = malloc(sizeof(double) * N);
  orc_encode_table(log_n, log_scale, T);
  orc_encode(&P, 17.0, x);
  free(s), free(pk), free(a), free(b), free(c), free(r), free(d), free(x), free(ent), free(pool), free(img);
  free(u), free(v), free(w), free(w2), free(g), free(T);
}

int main(void) {
  run(5, 2, 30, 20);
  run(6, 3, 36, 25);
  run(10, 3, 36, 30);
  printf("OK\n");
  return 0;
}
