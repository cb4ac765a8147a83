/*
 * ckks_oracle.h -- plain, slow CPU reference of pixel-level CKKS encryption with
 * caching (iCHEETAH, arXiv 2409.03568).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP implementation.
 *
 * Conventions (readings of the paper, frozen here):
 *  - Ring R_q = Z_q[X]/(X^N+1) in RNS form, Q = q_0 ... q_{L-1}, each q_i = 1 mod 2N
 *    (Sec. 2.2, "CKKS"; Sec. 2.2.1, "RLWE").
 *  - A ciphertext is stored [poly 0..1][limb 0..level-1][coeff 0..N-1] as uint64
 *    canonical residues in [0, q_i), coefficient domain.
 *  - Public key pk = (pk0, pk1) = (-a*s + e, a); encryption c0 = v*pk0 + e0 + m,
 *    c1 = v*pk1 + e1; decryption m' = c0 + c1*s.  This is Sec. 2.2.2 ("CKKS Basics")
 *    with the sign convention that makes its decryption equation hold (the printed
 *    key and encryption equations use a and b inconsistently).
 *  - Randomness is Philox4x64-10 (Salmon et al., SC'11), counter (t, tag, block, 0),
 *    key = 2-word seed.  Word j of a stream is word j%4 of block j/4.
 */
#ifndef CKKS_ORACLE_H
#define CKKS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LIMBS 16
#define ORC_MAX_B 64

/* Stream tags (counter word 1). */
enum {
  ORC_TAG_V = 1, ORC_TAG_E0 = 2, ORC_TAG_E1 = 3, ORC_TAG_AUX = 4,
  ORC_TAG_SK = 16, ORC_TAG_EK = 17, ORC_TAG_A0 = 32,
  ORC_TAG_RK_E0 = 48, /* + digit i: error of key-switching key i */
  ORC_TAG_RK_A0 = 64  /* + 32 digit + prime index: uniform part of key-switching key i */
};
/* Cache entry indices t under the cache seed. */
enum { ORC_RADIX_BASE_T = 0, ORC_VALUE_BASE_T = 256, ORC_POOL_BASE_T = 512 };

typedef struct {
  int log_n;                /* N = 2^log_n */
  int L;                    /* number of RNS primes */
  int log_scale;            /* Delta = 2^log_scale */
  int B;                    /* Gaussian tail bound; 0 = no noise */
  double sigma;             /* Gaussian standard deviation */
  uint64_t q[ORC_MAX_LIMBS];   /* primes, descending */
  uint64_t psi[ORC_MAX_LIMBS]; /* a primitive 2N-th root of unity mod q_i */
  uint64_t cdt[2 * ORC_MAX_B]; /* cumulative table, 2B entries */
  uint64_t qP;                 /* special prime of key switching (not one of the q_i) */
  uint64_t psiP;               /* a primitive 2N-th root of unity mod qP */
} orc_params;

/* ---- parameters ---- */
int orc_gen_primes(int log_n, int bits, int L, uint64_t *q);
uint64_t orc_primitive_2n_root(uint64_t q, int log_n);
int orc_cdt_table(double sigma, int B, uint64_t *T);
int orc_params_init(orc_params *P, int log_n, int L, int bits, int log_scale,
                    double sigma, int B, const uint64_t *primes);

/* ---- randomness ---- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t orc_stream_word(const uint64_t key[2], uint64_t t, uint64_t tag, uint64_t j);
int64_t orc_ternary(uint64_t w);
int64_t orc_gauss(uint64_t w, const uint64_t *T, int B);
void orc_sample_ternary(const uint64_t key[2], uint64_t t, uint64_t tag, int N, int64_t *out);
void orc_sample_gauss(const orc_params *P, const uint64_t key[2], uint64_t t, uint64_t tag, int64_t *out);
void orc_sample_uniform(const uint64_t key[2], uint64_t t, uint64_t tag, int N, uint64_t q, uint64_t *out);

/* ---- ring arithmetic ---- */
void orc_negacyclic_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *c, int N, uint64_t q);
void orc_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *c, int N, uint64_t q, uint64_t psi);

/* ---- CKKS ---- */
void orc_encode_table(int log_n, int log_scale, double *T);
void orc_encode(const orc_params *P, double value, int64_t *m);
void orc_keygen(const orc_params *P, const uint64_t seed[2], int64_t *s, uint64_t *pk);
void orc_encrypt(const orc_params *P, const uint64_t *pk, double value, const uint64_t seed[2],
                 uint64_t t, uint64_t *ct);
void orc_decrypt_coeffs(const orc_params *P, const int64_t *s, const uint64_t *ct, int level, uint64_t *d);
int orc_decode_centered(const orc_params *P, const uint64_t *d, int level, int64_t *x);
double orc_decrypt(const orc_params *P, const int64_t *s, const uint64_t *ct, int level, double scale, int *err);

void orc_add(const orc_params *P, const uint64_t *a, const uint64_t *b, uint64_t *out, int level);
void orc_sub(const orc_params *P, const uint64_t *a, const uint64_t *b, uint64_t *out, int level);
int orc_mul_const(const orc_params *P, const uint64_t *a, int level, double scale, double c,
                  uint64_t *out, double *out_scale);
int orc_add_const(const orc_params *P, uint64_t *a, int level, double scale, double b);
int orc_rescale(const orc_params *P, const uint64_t *in, int level, double scale, uint64_t *out,
                double *out_scale);

/* ---- ciphertext multiplication (Sec. 2.2.3: tensor product, relinearization) ----
 * Relinearization is RNS hybrid key switching with the special prime qP and one digit per
 * ciphertext prime.  Key-switching key i (i < L) has, for every prime p_j of
 * {q_0..q_{L-1}, qP} (j = L is qP), the pair
 *   ( -a_ij * s + e_i + [j == i] (qP mod q_i) s^2 ,  a_ij )  mod p_j,
 * i.e. (-a s + e_i + qP g_i s^2, a) mod qP*Q with g_i = 1 mod q_i, 0 mod q_j (j != i).
 * a_ij: uniform stream (seed, 0, ORC_TAG_RK_A0 + 32 i + j); e_i: Gaussian stream
 * (seed, 0, ORC_TAG_RK_E0 + i), the same integers in every prime.
 * Layout evk[i][j][2][N], canonical residues, coefficient domain.                       */
void orc_relin_keygen(const orc_params *P, const int64_t *s, const uint64_t seed[2], uint64_t *evk);
/* d[3][level][N] = (a0 b0, a0 b1 + a1 b0, a1 b1) per limb (negacyclic products). */
void orc_tensor(const orc_params *P, const uint64_t *a, const uint64_t *b, int level, uint64_t *d);
/* acc[2][level+1][N]: sum over digits i < level of (d2 limb i, lifted to p_j) * key i,
 * for the primes q_0..q_{level-1} then qP (index level). */
void orc_key_switch(const orc_params *P, const uint64_t *evk, const uint64_t *d2, int level, uint64_t *acc);
/* out[2][level][N] = (x - [x]_qP) / qP mod q_j for the value x with residues acc[k][.][.]
 * ([x]_qP centered), i.e. x / qP rounded to nearest. */
void orc_mod_down(const orc_params *P, const uint64_t *acc, int level, uint64_t *out);
/* out = (d0, d1) + ModDown(KeySwitch(d2)): the relinearized product, scale sa * sb. */
void orc_mul(const orc_params *P, const uint64_t *evk, const uint64_t *a, const uint64_t *b, int level,
             uint64_t *out);

/* ---- caching (Sec. 3.2) and randomness (Sec. 3.3) ---- */
void orc_radix_entries(const orc_params *P, const uint64_t *pk, int r, int D, const uint64_t cache_seed[2],
                       uint64_t *entries);
int orc_radix_encrypt(const orc_params *P, const uint64_t *entries, int r, int D, int p,
                      const uint64_t job_seed[2], uint64_t t, uint64_t *out);
void orc_histogram(const uint8_t *px, uint64_t n, uint64_t *h);
int orc_topk(const uint64_t *h, int k, int *values);
void orc_value_entry(const orc_params *P, const uint64_t *pk, int value, const uint64_t cache_seed[2],
                     uint64_t *ct);
void orc_pool_entry(const orc_params *P, const uint64_t *pk, int u, const uint64_t cache_seed[2], uint64_t *ct);
uint32_t orc_pool_pick(const uint64_t job_seed[2], uint64_t t, uint32_t npool);
void orc_value_encrypt(const orc_params *P, const uint64_t *pk, const uint64_t *value_ct, const uint64_t *pool,
                       uint32_t npool, int p, const uint64_t job_seed[2], uint64_t t, uint64_t *out);

/* ---- image operations (Sec. 4.4) ---- */
int orc_mean_filter_pixel(const orc_params *P, const uint64_t *img, int H, int W, int level, double scale,
                          int k, int y, int x, uint64_t *out, double *out_scale);

/* ---- batches (OpenMP over independent ciphertexts) ---- */
void orc_encrypt_batch(const orc_params *P, const uint64_t *pk, const uint8_t *px, uint64_t n,
                       const uint64_t seed[2], uint64_t first_index, uint64_t *out);
void orc_decrypt_batch(const orc_params *P, const int64_t *s, const uint64_t *cts, uint64_t n, int level,
                       double scale, double *out, int *nerr);
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
