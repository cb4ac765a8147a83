// Selects the per-ring-degree launchers of the NTT path.
#include "internal.hpp"

namespace ckks {

#define CKKS_DECLARE_RING(LOGN)                                                                              \
  hipError_t launch_encrypt_##LOGN(const ckks_ctx *, const EncJob &, uint64_t, hipStream_t);                 \
  hipError_t launch_cached_fused_##LOGN(const ckks_ctx *, const FusedJob &, bool, hipStream_t);              \
  hipError_t launch_keygen_##LOGN(const ckks_ctx *, uint64_t, uint64_t, hipStream_t);                        \
  hipError_t launch_keys_prepare_##LOGN(const ckks_ctx *, hipStream_t);                                      \
  hipError_t launch_decrypt_##LOGN(const ckks_ctx *, const uint64_t *, uint64_t, int, double, double *, int,   \
                                   hipStream_t, uint64_t);                                                    \
  hipError_t launch_relin_keygen_##LOGN(const ckks_ctx *, uint64_t, uint64_t, hipStream_t);                  \
  hipError_t launch_relin_prepare_##LOGN(const ckks_ctx *, hipStream_t);                                     \
  hipError_t launch_mul_##LOGN(const ckks_ctx *, const uint64_t *, const uint64_t *, uint64_t *, uint64_t, int, \
                               uint64_t *, hipStream_t);
CKKS_DECLARE_RING(11)
CKKS_DECLARE_RING(12)
CKKS_DECLARE_RING(13)
CKKS_DECLARE_RING(14)

#define CKKS_RING_SWITCH(FN, ...)                      \
  switch (c->prm.log_n) {                              \
    case 11: return FN##_11(c, __VA_ARGS__);           \
    case 12: return FN##_12(c, __VA_ARGS__);           \
    case 13: return FN##_13(c, __VA_ARGS__);           \
    case 14: return FN##_14(c, __VA_ARGS__);           \
    default: return hipErrorInvalidValue;              \
  }

hipError_t launch_encrypt(const ckks_ctx *c, const EncJob &job, uint64_t grid, hipStream_t stream) {
  CKKS_RING_SWITCH(launch_encrypt, job, grid, stream)
}
hipError_t launch_cached_fused(const ckks_ctx *c, const FusedJob &job, bool misses, hipStream_t stream) {
  CKKS_RING_SWITCH(launch_cached_fused, job, misses, stream)
}
hipError_t launch_keygen(const ckks_ctx *c, uint64_t seed0, uint64_t seed1, hipStream_t stream) {
  CKKS_RING_SWITCH(launch_keygen, seed0, seed1, stream)
}
hipError_t launch_keys_prepare(const ckks_ctx *c, hipStream_t stream) { CKKS_RING_SWITCH(launch_keys_prepare, stream) }
hipError_t launch_decrypt(const ckks_ctx *c, const uint64_t *cts, uint64_t n, int level, double scale, double *out,
                          int limbs, hipStream_t stream, uint64_t max_grid) {
  CKKS_RING_SWITCH(launch_decrypt, cts, n, level, scale, out, limbs, stream, max_grid)
}
hipError_t launch_relin_keygen(const ckks_ctx *c, uint64_t seed0, uint64_t seed1, hipStream_t stream) {
  CKKS_RING_SWITCH(launch_relin_keygen, seed0, seed1, stream)
}
hipError_t launch_relin_prepare(const ckks_ctx *c, hipStream_t stream) { CKKS_RING_SWITCH(launch_relin_prepare, stream) }
hipError_t launch_mul(const ckks_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n, int level,
                      uint64_t *scratch, hipStream_t stream) {
  CKKS_RING_SWITCH(launch_mul, a, b, out, n, level, scratch, stream)
}

}  // namespace ckks
