// Exact modular arithmetic for RNS primes q < 2^50, shared by host and device code.
//
// Residues inside the NTT are held in IEEE doubles as exact signed integers.  The
// product a*w is split into h = fl(a*w) and the exact rounding error l = fma(a,w,-h);
// the quotient c = rint(h/q) comes from one fma against 1/q with the 1.5*2^52
// rounding constant; h - c*q and the final sum are exact because both are
// integers below 2^53.  This is the FMA-based modular product of van der Hoeven,
// Lecerf and Quintin ("Modular SIMD arithmetic in Mathemagix", 2014), used with
// signed (lazy) representatives: outputs are congruent to the true product and
// bounded in magnitude, and a separate reduction brings values back near [-q/2, q/2].
//
// Bounds (q < 2^50, 1/q rounded to nearest):
//   reduce(x):     |x| < 2^52      ->  x' = x (mod q), |x'| <= q/2 + 1
//                  |x| < 2^53      ->  x' = x (mod q), |x'| <= q/2 + 2 (x an exact integer)
//   mulmod(a, w):  |a*w/q| < 2^51  ->  r = a*w (mod q), |r| <= q/2 + |a*w| 2^-52 + 1
// The NTT keeps forward-transform values below 2^52 and inverse-transform values below
// 2^51 by reducing after the stages its compile-time schedule selects (ntt.hpp), which
// satisfies both preconditions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CKKS_HD __host__ __device__ __forceinline__

namespace ckks {

constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52

struct ModF {
  double q;     // the prime, exactly
  double qinv;  // fl(1/q)
};

// x - q*rint(x/q): congruent to x, |result| <= q/2 + 1 for |x| < 2^52.
CKKS_HD double reduce(double x, double q, double qinv) {
  const double c = __builtin_fma(x, qinv, kRound) - kRound;
  return __builtin_fma(-c, q, x);
}

// a*w mod q as a signed representative (see the bounds above).
CKKS_HD double mulmod(double a, double w, double q, double qinv) {
  const double h = a * w;
  const double l = __builtin_fma(a, w, -h);
  const double c = __builtin_fma(h, qinv, kRound) - kRound;
  const double r = __builtin_fma(-c, q, h);
  return r + l;
}

// canonical representative in [0, q) of an integer-valued x with |x| < 2^52.
CKKS_HD double canon(double x, double q, double qinv) {
  const double r = reduce(x, q, qinv);
  return r < 0.0 ? r + q : r;
}

// centered representative in (-q/2, q/2] of an integer-valued x with |x| < 2^52.
CKKS_HD double center(double x, double q, double qinv) {
  double r = reduce(x, q, qinv);
  r = (r > 0.5 * q) ? r - q : r;
  r = (r <= -0.5 * q) ? r + q : r;
  return r;
}

// Cooley-Tukey butterfly (X, Y) -> (X + W*Y, X - W*Y).
CKKS_HD void ct_butterfly(double &X, double &Y, double W, double q, double qinv) {
  const double t = mulmod(Y, W, q, qinv);
  Y = X - t;
  X = X + t;
}

// Gentleman-Sande butterfly (X, Y) -> (X + Y, (X - Y)*W).
CKKS_HD void gs_butterfly(double &X, double &Y, double W, double q, double qinv) {
  const double d = X - Y;
  X = X + Y;
  Y = mulmod(d, W, q, qinv);
}

// ---------------------------------------------------------------------------
// conversions between canonical uint64 residues (< 2^52) and exact doubles
// ---------------------------------------------------------------------------
// For an integer 0 <= x < 2^52 the double 2^52 + x is exact and its bit pattern is that
// of 2^52 with x in the low 52 (mantissa) bits, so each conversion is one integer and
// one floating-point operation.
constexpr double kTwo52 = 4503599627370496.0;
constexpr uint64_t kTwo52Bits = 0x4330000000000000ull;

CKKS_HD double u64_to_f64(uint64_t x) { return __builtin_bit_cast(double, x | kTwo52Bits) - kTwo52; }

// x integer-valued in [0, 2^52)
CKKS_HD uint64_t f64_to_u64(double x) { return __builtin_bit_cast(uint64_t, x + kTwo52) - kTwo52Bits; }

// ---------------------------------------------------------------------------
// 64-bit integer helpers for canonical uint64 residues (elementwise kernels)
// ---------------------------------------------------------------------------
CKKS_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
  const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
  const uint64_t p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
  const uint64_t mid = (p00 >> 32) + (uint32_t)p01 + (uint32_t)p10;
  return p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

// 128-bit product as a chain of four 32x32+64 multiply-adds (one v_mad_u64_u32 each):
// with t = a0 b0, u = a1 b0 + hi(t), v = a0 b1 + lo(u), w = a1 b1 + hi(u) (none of which
// overflows 64 bits), a*b = lo(t) + 2^32 v + 2^64 w, so lo = (v << 32) | lo(t) and
// hi = w + hi(v).
CKKS_HD void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t t = (uint64_t)a0 * b0;
  const uint64_t u = (uint64_t)a1 * b0 + (t >> 32);
  const uint64_t v = (uint64_t)a0 * b1 + (uint32_t)u;
  const uint64_t w = (uint64_t)a1 * b1 + (u >> 32);
  lo = (v << 32) | (uint32_t)t;
  hi = w + (v >> 32);
}

CKKS_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  const uint64_t s = a + b;
  return s >= q ? s - q : s;
}

CKKS_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + (q - b); }

// Shoup multiplication by a fixed w < q with wp = floor(w * 2^64 / q): exact a*w mod q
// for any a < 2^64 (Harvey, "Faster arithmetic for number-theoretic transforms", 2014).
CKKS_HD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  const uint64_t hi = mulhi64(a, wp);
  const uint64_t r = a * w - hi * q;
  return r >= q ? r - q : r;
}

// x mod q for a signed x with |x| < 2^62 and q < 2^50, using a double quotient estimate.
CKKS_HD uint64_t mod_i64(int64_t x, uint64_t q, double qinv) {
  const int64_t c = (int64_t)((double)x * qinv);
  int64_t r = x - c * (int64_t)q;
  while (r < 0) r += (int64_t)q;
  while (r >= (int64_t)q) r -= (int64_t)q;
  return (uint64_t)r;
}

// residue of an integer-valued double of any magnitude: |x| = M * 2^e with M < 2^53.
CKKS_HD uint64_t residue_of_double(double x, uint64_t q, double qinv) {
  const double ax = x < 0 ? -x : x;
  uint64_t r;
  if (ax < 4503599627370496.0) {  // 2^52: the value is its own integer
    r = mod_i64((int64_t)ax, q, qinv);
  } else {
    int e;
    const double m = frexp(ax, &e);
    uint64_t M = (uint64_t)ldexp(m, 53);
    r = M % q;
    // multiply by 2^(e-53) mod q by doubling
    for (int i = 0; i < e - 53; i++) r = add_mod(r, r, q);
  }
  return (x < 0 && r != 0) ? q - r : r;
}

}  // namespace ckks
