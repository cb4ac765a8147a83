// Philox4x64-10 counter-based generator and the samplers built on it.
//
// Philox (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128-bit
// multiplies by fixed odd constants, xor-ed with the Weyl-sequence round keys.
// Every random value of the scheme is a word of the stream keyed by a 2-word seed at
// counter (t, tag, block, 0): word j of stream (t, tag) is word j mod 4 of block j/4.
// Tags: 1 = v, 2 = e0, 3 = e1 (encryption randomness, Sec. 2.2.2), 4 = auxiliary
// (cache randomness, Sec. 3.3), 16 = secret key, 17 = key error, 32+i = a_i.
#pragma once
#include "modarith.hpp"

namespace ckks {

enum : uint32_t {
  kTagV = 1, kTagE0 = 2, kTagE1 = 3, kTagAux = 4, kTagSk = 16, kTagEk = 17, kTagA0 = 32
};

struct Philox4 {
  uint64_t w[4];
};

// The key (k0, k1) must be uniform across the wavefront (it is a seed of the launch).
CKKS_HD Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#if defined(__HIP_DEVICE_COMPILE__)
  // Every call of a launch has the same key; without this the compiler forms all twenty
  // round keys once per kernel and keeps them in scalar registers throughout, which
  // spills.  Here each call forms them as it goes (two scalar adds per round).
  asm volatile("" : "+s"(k0), "+s"(k1));
#endif
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  Philox4 o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

// Ternary value floor(3w / 2^64) - 1 in {-1, 0, 1}: the word range split at
// ceil(2^64/3) and ceil(2^65/3).
CKKS_HD int ternary_of(uint64_t w) {
  return (int)(w >= 0x5555555555555556ULL) + (int)(w >= 0xAAAAAAAAAAAAAAABULL) - 1;
}

// Gaussian value -B + #{k < 2B : w >= T[k]} by a branch-free binary search over a
// 128-entry table whose unused tail is all-ones (never counted: the count is capped
// at 2B, and an all-ones word already counts every real entry).
constexpr int kCdtSlots = 128;
CKKS_HD int gauss_of(uint64_t w, const uint64_t *T, int B) {
  int pos = 0;
#pragma unroll
  for (int step = kCdtSlots / 2; step >= 1; step >>= 1) pos += (T[pos + step - 1] <= w) ? step : 0;
  pos = pos < 2 * B ? pos : 2 * B;
  return pos - B;
}

}  // namespace ckks
