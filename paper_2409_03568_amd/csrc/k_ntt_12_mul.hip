// Kernels of the NTT path for N = 2^12: ciphertext product and its keys (see k_ntt_impl.hpp).
#include "k_ntt_impl.hpp"
CKKS_DEFINE_RING_MUL(12)
