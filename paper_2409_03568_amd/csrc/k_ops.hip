// Elementwise homomorphic operations (Sec. 2.2.3) and the fused mean filter (Sec. 4.4.1)
// on canonical uint64 residues.  All of these are bound by HBM bandwidth: each kernel
// streams its ciphertexts once with 16-byte accesses, one workgroup per N-coefficient
// row ([ct][poly][limb] rows), and keeps the per-limb constants in registers.
#include <atomic>

#include "internal.hpp"
#include "modarith.hpp"
#include "philox.hpp"

namespace ckks {

constexpr int kRowThreads = 256;

struct RowConsts {
  uint64_t q[kMaxL];
  uint64_t K[kMaxL];   // multiplier per limb
  uint64_t Kp[kMaxL];  // its Shoup companion
};

// out = a +/- b, rows of N residues; row r has limb r % level.
template <bool SUB>
__global__ void __launch_bounds__(kRowThreads)
    k_add_sub(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b, uint64_t *__restrict__ out,
              uint64_t rows, int level, int log_n, RowConsts rc) {
  const int N = 1 << log_n;
  for (uint64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const uint64_t q = rc.q[row % (uint64_t)level];
    const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(a + row * N);
    const ulonglong2 *pb = reinterpret_cast<const ulonglong2 *>(b + row * N);
    ulonglong2 *po = reinterpret_cast<ulonglong2 *>(out + row * N);
    for (int i = threadIdx.x; i < N / 2; i += kRowThreads) {
      const ulonglong2 x = pa[i], y = pb[i];
      ulonglong2 z;
      z.x = SUB ? sub_mod(x.x, y.x, q) : add_mod(x.x, y.x, q);
      z.y = SUB ? sub_mod(x.y, y.y, q) : add_mod(x.y, y.y, q);
      po[i] = z;
    }
  }
}

// out = K_limb * a (Shoup multiplication by the per-limb constant).
__global__ void __launch_bounds__(kRowThreads)
    k_mul_const(const uint64_t *__restrict__ a, uint64_t *__restrict__ out, uint64_t rows, int level, int log_n,
                RowConsts rc) {
  const int N = 1 << log_n;
  for (uint64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int l = (int)(row % (uint64_t)level);
    const uint64_t q = rc.q[l], K = rc.K[l], Kp = rc.Kp[l];
    const ulonglong2 *pa = reinterpret_cast<const ulonglong2 *>(a + row * N);
    ulonglong2 *po = reinterpret_cast<ulonglong2 *>(out + row * N);
    for (int i = threadIdx.x; i < N / 2; i += kRowThreads) {
      const ulonglong2 x = pa[i];
      ulonglong2 z;
      z.x = mul_shoup(x.x, K, Kp, q);
      z.y = mul_shoup(x.y, K, Kp, q);
      po[i] = z;
    }
  }
}

// c0 += encode(b) at scale `scale` (slot 0): m_j = rint(f cos(pi j / N)), f = (b*scale) 2^(1-log_n).
// Rows are the c0 rows only: row r is ciphertext r / level, limb r % level.
__global__ void __launch_bounds__(kRowThreads)
    k_add_const(uint64_t *__restrict__ a, uint64_t rows, int level, int log_n, double scale,
                const double *__restrict__ d_b, double b, const double *__restrict__ cosj,
                const LimbConsts *__restrict__ lcp) {
  const LimbConsts &lc = *lcp;
  const int N = 1 << log_n;
  for (uint64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const uint64_t ct = row / (uint64_t)level;
    const int l = (int)(row % (uint64_t)level);
    const double bb = d_b ? d_b[ct] : b;
    const double f = ldexp(bb * scale, 1 - log_n);
    const double q = lc.q[l], qinv = lc.qinv[l];
    const uint64_t qi = lc.qi[l];
    uint64_t *c0 = a + (ct * 2 * (uint64_t)level + (uint64_t)l) * N;
    const bool small = fabs(f) < 4503599627370496.0;  // then |m_j| < 2^52: exact FP64 residue
    for (int j = threadIdx.x; j < N; j += kRowThreads) {
      const double m = __builtin_rint(f * cosj[j]);
      const uint64_t r = small ? (uint64_t)canon(m, q, qinv) : residue_of_double(m, qi, qinv);
      c0[j] = add_mod(c0[j], r, qi);
    }
  }
}

// Rescale by q_last = q_{level-1}: r = (c_last + h) mod q_last, h = floor(q_last/2);
// c'_i = (c_i + h - r) * q_last^-1 mod q_i for i < level-1.  One thread per coefficient.
struct RescaleConsts {
  uint64_t q[kMaxL];
  uint64_t h_mod[kMaxL];    // h mod q_i
  uint64_t qlinv[kMaxL];    // q_last^-1 mod q_i
  uint64_t qlinv_p[kMaxL];  // Shoup companion
  uint64_t qlast, h;
};

__global__ void __launch_bounds__(kRowThreads)
    k_rescale(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint64_t polys, int level, int log_n,
              RescaleConsts rc) {
  const int N = 1 << log_n;
  const int nl = level - 1;
  for (uint64_t p = blockIdx.x; p < polys; p += gridDim.x) {
    const uint64_t *src = in + p * (uint64_t)level * N;
    uint64_t *dst = out + p * (uint64_t)nl * N;
    for (int j = threadIdx.x; j < N; j += kRowThreads) {
      const uint64_t r = add_mod(src[(size_t)nl * N + j], rc.h, rc.qlast);
      for (int i = 0; i < nl; i++) {
        const uint64_t qi = rc.q[i];
        const uint64_t ri = r >= qi ? r - qi : r;  // r < q_last < 2 q_i
        const uint64_t num = sub_mod(add_mod(src[(size_t)i * N + j], rc.h_mod[i], qi), ri, qi);
        dst[(size_t)i * N + j] = mul_shoup(num, rc.qlinv[i], rc.qlinv_p[i], qi);
      }
    }
  }
}

// Fused k x k mean filter with clamped borders: out(y,x) = rescale(K * sum of the window).
// Thread (x-tile, poly, j) owns XT adjacent output columns of coefficient j and walks down
// output rows y_begin..y_end-1 of the image (written as rows 0.. of out), keeping the
// horizontal window sums of the last k rows in a ring; the vertical sum is updated by
// adding the row that enters and subtracting the row that leaves.  Image row y is read
// from row y mod fc.ring of `in` (a buffer of whole rows: the image itself, or a ring of
// rows that a tiled pipeline refills as it moves down).  Arithmetic is exact FP64 on signed representatives:
//   a horizontal sum of k <= 7 canonical residues is below 7q < 2^53 and is reduced to
//   |h| <= q/2 + 2; the vertical sum of k such values stays below 3.5q + 14 < 2^52; the
//   product with the centered multiplier K (|K| <= q/2) has |v K / q| < 1.75q < 2^51, so
//   mulmod applies and returns |m| < 0.94q; the rescale numerator m_i + h - r stays below
//   2.5 * 2^50 and its product with the centered q_last^-1 is canonicalised at the end.
// Since every step is exact modular arithmetic the result equals the sum, multiplication
// and rescale applied one after another.
struct FilterConsts {
  double q[kMaxL], qinv[kMaxL];
  double K[kMaxL];      // K = rint(q_last / k^2) mod q_i, centered
  double qlinv[kMaxL];  // q_last^-1 mod q_i, centered
  double h;             // floor(q_last / 2)
  uint32_t ring;        // rows of the input buffer: image row y is buffer row y mod ring
};

constexpr int kFilterWaves = 8;
// s_waitcnt immediate that waits for every outstanding vector memory operation of the wave
// (vmcnt 0; expcnt and lgkmcnt at their maxima, i.e. not waited for)
constexpr int kWaitVmcnt0 = 0x0F70;
// cache-policy operand of a load: non-temporal
constexpr int kCpolNonTemporal = 2;
constexpr int kFilterThreads = 64 * kFilterWaves;

// Columns of one image row that a workgroup stages in LDS (its 8 waves' output columns and
// the halos on both sides), and the staging buffers' bytes (two rows, 64 coefficients).
template <int KW, int LV, int XT>
constexpr int filter_stage_cols() {
  return kFilterWaves * XT + 2 * (KW / 2);
}
template <int KW, int LV, int XT>
constexpr size_t filter_lds_bytes() {
  return 2 * (size_t)filter_stage_cols<KW, LV, XT>() * LV * 64 * sizeof(double);
}

template <int KW, int LV, int XT>
__global__ void __launch_bounds__(kFilterThreads)
    k_mean_filter(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint32_t H, uint32_t W, uint32_t y_begin,
                  uint32_t y_end, int log_n, uint32_t groups, FilterConsts fc) {
  constexpr int RAD = KW / 2, XC = XT + 2 * RAD;
  constexpr int XW = filter_stage_cols<KW, LV, XT>(), NV = XW * LV;  // staged columns, 64-word vectors per row
  static_assert(NV % 2 == 0, "a staging load moves two vectors");
  const int N = 1 << log_n;
  // logical workgroup lb = (64-coefficient chunk jc, poly, tile group g), g fastest; its
  // wave w takes column tile kFilterWaves * g + w.  The workgroup stages each input row's
  // columns (its waves' output columns and the halos) once in LDS, loaded straight from
  // HBM into LDS with non-temporal loads one row ahead of use, and its waves read their
  // columns from there: the image streams past the caches without displacing what other
  // kernels keep in them (cache entries between calls), and the halo columns two waves
  // share are read from HBM once.
  extern __shared__ uint64_t stage[];  // [2][NV][64] residues: row buffers, alternating
  const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const uint32_t g = lb % groups;
  const uint32_t rest = lb / groups;
  const int poly = (int)(rest & 1);
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
  const uint64_t jc = (uint64_t)(rest >> 1) * 64;
  // a wave past the right edge reads clamped columns and writes nothing, but takes part
  // in the staging and the workgroup's barriers
  const uint64_t xw0 = (uint64_t)g * kFilterWaves * XT;  // first output column of the workgroup
  const uint64_t x0 = xw0 + (uint64_t)wv * XT;            // first output column of this wave
  const uint64_t ct_stride = (uint64_t)2 * LV * N;
  const uint64_t pbase = (uint64_t)poly * LV * N + jc;
  const int64_t y_last = (int64_t)y_end - 1 + RAD;  // last input row the workgroup needs
  // Loads input row yy into buffer b: vector v = (staged column v / LV, limb v % LV) is
  // the 64 coefficients of that limb of image column xw0 + v / LV - RAD (clamped); each
  // load instruction moves two vectors, 16 bytes per lane.
  auto stage_row = [&](int64_t yy, int b) {
    const uint32_t yi = (uint32_t)(yy < 0 ? 0 : (yy >= (int64_t)H ? H - 1 : yy));
    const uint64_t y = yi < fc.ring ? yi : yi % fc.ring;
    uint64_t *sb = stage + (size_t)b * NV * 64;
    for (int pr = wv; pr < NV / 2; pr += kFilterWaves) {
      const int v = 2 * pr + (lane >> 5);
      const int col = v / LV, i = v % LV;
      const int64_t xx = (int64_t)xw0 + col - RAD;
      const uint64_t xc = (uint64_t)(xx < 0 ? 0 : (xx >= (int64_t)W ? (int64_t)W - 1 : xx));
      const uint64_t *p = in + (y * W + xc) * ct_stride + pbase + (size_t)i * N + 2 * (lane & 31);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)p,
                                       (__attribute__((address_space(3))) void *)(sb + (size_t)pr * 128), 16, 0,
                                       kCpolNonTemporal);
    }
  };
  const uint64_t out_stride = (uint64_t)2 * (LV - 1) * N;
  const uint64_t out_base = (uint64_t)poly * (LV - 1) * N + jc + lane;
  int buf = 0;
  stage_row((int64_t)y_begin - RAD, 0);
  // horizontal sums of input row yy (staged in buffer buf) for the XT output columns
  auto hsum = [&](int64_t yy, double (&h)[XT][LV]) {
    // this wave's staging loads are complete (the wait also covers its output stores);
    // after the barrier all waves' are, and every wave has finished reading the other buffer
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (yy + 1 <= y_last) stage_row(yy + 1, buf ^ 1);
    const uint64_t *sb = stage + (size_t)buf * NV * 64;
    double c[XC][LV];
#pragma unroll
    for (int d = 0; d < XC; d++)
#pragma unroll
      for (int i = 0; i < LV; i++) c[d][i] = u64_to_f64(sb[((wv * XT + d) * LV + i) * 64 + lane]);
    buf ^= 1;
#pragma unroll
    for (int t = 0; t < XT; t++) {
#pragma unroll
      for (int i = 0; i < LV; i++) {
        double s = c[t][i];
#pragma unroll
        for (int d = 1; d < KW; d++) s += c[t + d][i];
        h[t][i] = reduce(s, fc.q[i], fc.qinv[i]);
      }
    }
  };
  double ring[KW][XT][LV];
  double v[XT][LV];
#pragma unroll
  for (int t = 0; t < XT; t++)
#pragma unroll
    for (int i = 0; i < LV; i++) v[t][i] = 0.0;
#pragma unroll
  for (int d = 0; d < KW; d++) {
    hsum((int64_t)y_begin + d - RAD, ring[d]);
#pragma unroll
    for (int t = 0; t < XT; t++)
#pragma unroll
      for (int i = 0; i < LV; i++) v[t][i] += ring[d][t][i];
  }
  const double ql = fc.q[LV - 1], qlinv = fc.qinv[LV - 1];
  for (uint32_t y0 = y_begin; y0 < y_end; y0 += KW) {
#pragma unroll
    for (int s = 0; s < KW; s++) {
      const uint32_t y = y0 + s;
      if (y >= y_end) break;
#pragma unroll
      for (int t = 0; t < XT; t++) {
        if (x0 + t >= W) break;
        const double r = canon(mulmod(v[t][LV - 1], fc.K[LV - 1], ql, qlinv) + fc.h, ql, qlinv);
        uint64_t *o = out + ((uint64_t)(y - y_begin) * W + x0 + t) * out_stride + out_base;
#pragma unroll
        for (int i = 0; i < LV - 1; i++) {
          const double m = mulmod(v[t][i], fc.K[i], fc.q[i], fc.qinv[i]);
          const double z = mulmod(m + fc.h - r, fc.qlinv[i], fc.q[i], fc.qinv[i]);
          __builtin_nontemporal_store(f64_to_u64(canon(z, fc.q[i], fc.qinv[i])), o + (size_t)i * N);
        }
      }
      // slide the window: ring slot s holds row y - RAD; replace it by row y + RAD + 1
      if (y + 1 < y_end) {
        double nh[XT][LV];
        hsum((int64_t)y + RAD + 1, nh);
#pragma unroll
        for (int t = 0; t < XT; t++)
#pragma unroll
          for (int i = 0; i < LV; i++) {
            v[t][i] = (v[t][i] - ring[s][t][i]) + nh[t][i];
            ring[s][t][i] = nh[t][i];
          }
      }
    }
  }
  // no staging load may still be writing this workgroup's LDS when it ends
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_add_sub(const ckks_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n,
                          int level, bool sub, hipStream_t st) {
  RowConsts rc{};
  for (int i = 0; i < level; i++) rc.q[i] = c->prm.q[(size_t)i];
  const uint64_t rows = n * 2 * (uint64_t)level;
  if (sub)
    hipLaunchKernelGGL(k_add_sub<true>, dim3(row_grid(c, rows)), dim3(kRowThreads), 0, st, a, b, out, rows, level,
                       c->prm.log_n, rc);
  else
    hipLaunchKernelGGL(k_add_sub<false>, dim3(row_grid(c, rows)), dim3(kRowThreads), 0, st, a, b, out, rows, level,
                       c->prm.log_n, rc);
  return hipGetLastError();
}

hipError_t launch_mul_const(const ckks_ctx *c, const uint64_t *a, uint64_t *out, uint64_t n, int level,
                            const uint64_t *K, hipStream_t st) {
  RowConsts rc{};
  for (int i = 0; i < level; i++) {
    rc.q[i] = c->prm.q[(size_t)i];
    rc.K[i] = K[i];
    rc.Kp[i] = host::shoup_companion(K[i], rc.q[i]);
  }
  const uint64_t rows = n * 2 * (uint64_t)level;
  hipLaunchKernelGGL(k_mul_const, dim3(row_grid(c, rows)), dim3(kRowThreads), 0, st, a, out, rows, level, c->prm.log_n,
                     rc);
  return hipGetLastError();
}

hipError_t launch_add_const(const ckks_ctx *c, uint64_t *a, uint64_t n, int level, double scale, const double *d_b,
                            double b, hipStream_t st) {
  const uint64_t rows = n * (uint64_t)level;
  hipLaunchKernelGGL(k_add_const, dim3(row_grid(c, rows)), dim3(kRowThreads), 0, st, a, rows, level, c->prm.log_n, scale,
                     d_b, b, c->dev.cosj, c->d_lc);
  return hipGetLastError();
}

static void rescale_consts(const ckks_ctx *c, int level, uint64_t *q, uint64_t *h_mod, uint64_t *qlinv,
                           uint64_t *qlinv_p, uint64_t *qlast, uint64_t *h) {
  *qlast = c->prm.q[(size_t)level - 1];
  *h = *qlast / 2;
  for (int i = 0; i < level - 1; i++) {
    q[i] = c->prm.q[(size_t)i];
    h_mod[i] = *h % q[i];
    qlinv[i] = host::inv_mod(*qlast % q[i], q[i]);
    qlinv_p[i] = host::shoup_companion(qlinv[i], q[i]);
  }
}

hipError_t launch_rescale(const ckks_ctx *c, const uint64_t *a, uint64_t *out, uint64_t n, int level,
                          hipStream_t st) {
  RescaleConsts rc{};
  rescale_consts(c, level, rc.q, rc.h_mod, rc.qlinv, rc.qlinv_p, &rc.qlast, &rc.h);
  const uint64_t polys = n * 2;
  hipLaunchKernelGGL(k_rescale, dim3(row_grid(c, polys)), dim3(kRowThreads), 0, st, a, out, polys, level, c->prm.log_n,
                     rc);
  return hipGetLastError();
}

// Output columns per thread: enough to share the k - 1 halo columns, few enough that the
// ring of k * XT * LV sums stays in registers.
template <int KW, int LV>
constexpr int filter_xt() {
  return KW * LV <= 16 ? 2 : 1;
}

template <int KW, int LV>
static hipError_t filter_t(const uint64_t *in, uint64_t *out, uint32_t H, uint32_t W, uint32_t y0, uint32_t y1,
                           int log_n, const FilterConsts &fc, hipStream_t st) {
  constexpr int XT = filter_xt<KW, LV>();
  constexpr size_t lds = filter_lds_bytes<KW, LV, XT>();
  static_assert(lds <= 160 * 1024, "staging buffers exceed a CU's LDS");
  const uint64_t tiles = ((uint64_t)W + XT - 1) / XT;
  const uint64_t groups = (tiles + kFilterWaves - 1) / kFilterWaves;
  const uint64_t blocks = groups * 2 * (((uint64_t)1 << log_n) / 64);
  if (blocks > 0xffffffffull) return hipErrorInvalidValue;
  if constexpr (lds > 64 * 1024) {
    // once per kernel and device (also keeps the call out of graph captures after the first launch)
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 63;
    const uint64_t bit = 1ull << dev;
    if (!(done.load(std::memory_order_acquire) & bit)) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_mean_filter<KW, LV, XT>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      done.fetch_or(bit, std::memory_order_acq_rel);
    }
  }
  hipLaunchKernelGGL((k_mean_filter<KW, LV, XT>), dim3((uint32_t)blocks), dim3(kFilterThreads), lds, st, in, out, H,
                     W, y0, y1, log_n, (uint32_t)groups, fc);
  return hipGetLastError();
}

template <int KW>
static hipError_t filter_level(int level, const uint64_t *in, uint64_t *out, uint32_t H, uint32_t W, uint32_t y0,
                               uint32_t y1, int log_n, const FilterConsts &fc, hipStream_t st) {
  switch (level) {
    case 2: return filter_t<KW, 2>(in, out, H, W, y0, y1, log_n, fc, st);
    case 3: return filter_t<KW, 3>(in, out, H, W, y0, y1, log_n, fc, st);
    case 4: return filter_t<KW, 4>(in, out, H, W, y0, y1, log_n, fc, st);
    case 5: return filter_t<KW, 5>(in, out, H, W, y0, y1, log_n, fc, st);
    case 6: return filter_t<KW, 6>(in, out, H, W, y0, y1, log_n, fc, st);
    case 7: return filter_t<KW, 7>(in, out, H, W, y0, y1, log_n, fc, st);
    case 8: return filter_t<KW, 8>(in, out, H, W, y0, y1, log_n, fc, st);
    default: return hipErrorInvalidValue;
  }
}

static double centered_double(uint64_t x, uint64_t q) {
  return x > q / 2 ? -(double)(q - x) : (double)x;
}

hipError_t launch_mean_filter(const ckks_ctx *c, const uint64_t *in, uint64_t *out, uint32_t H, uint32_t W,
                              uint32_t y0, uint32_t y1, uint32_t k, int level, const uint64_t *K, hipStream_t st,
                              uint32_t ring_rows) {
  FilterConsts fc{};
  fc.ring = ring_rows ? ring_rows : H;
  const uint64_t qlast = c->prm.q[(size_t)level - 1];
  for (int i = 0; i < level; i++) {
    const uint64_t qi = c->prm.q[(size_t)i];
    fc.q[i] = (double)qi;
    fc.qinv[i] = 1.0 / (double)qi;
    fc.K[i] = centered_double(K[i] % qi, qi);
    if (i < level - 1) fc.qlinv[i] = centered_double(host::inv_mod(qlast % qi, qi), qi);
  }
  fc.h = (double)(qlast / 2);
  const int log_n = c->prm.log_n;
  switch (k) {
    case 1: return filter_level<1>(level, in, out, H, W, y0, y1, log_n, fc, st);
    case 3: return filter_level<3>(level, in, out, H, W, y0, y1, log_n, fc, st);
    case 5: return filter_level<5>(level, in, out, H, W, y0, y1, log_n, fc, st);
    case 7: return filter_level<7>(level, in, out, H, W, y0, y1, log_n, fc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ckks
