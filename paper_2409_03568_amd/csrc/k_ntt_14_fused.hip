// Kernels of the NTT path for N = 2^14: fused cached encryption (see k_ntt_impl.hpp).
#include "k_ntt_impl.hpp"
CKKS_DEFINE_RING_FUSED(14)
