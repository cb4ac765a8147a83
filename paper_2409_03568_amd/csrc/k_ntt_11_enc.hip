// Kernels of the NTT path for N = 2^11: encryption, keys and decryption (see k_ntt_impl.hpp).
#include "k_ntt_impl.hpp"
CKKS_DEFINE_RING_ENC(11)
