// cfs_device.hpp -- device building blocks of the chaos game on gfx950.
//
// One lane carries one point (Section 1 / Section 3 of the paper: every point
// is independent; per-thread state is a handful of values).  The map table
// lives in LDS and is gathered per lane by the drawn index, so there is no
// per-lane branching on the index for affine maps; composed transforms are
// compile-time kinds, so the whole wave takes the same path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cfs_params.hpp"

namespace cfs {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds; each
// multiplies words 0 and 2 by the two round constants into 64-bit products
// (one v_mad_u64_u32 each), xors the high halves with words 1/3 and the key,
// and moves the low halves; the key advances by the Weyl constants.  The key
// is wave-uniform, so its bumps stay on the scalar unit.
// ---------------------------------------------------------------------------
struct Block4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block4 philox10(uint32_t x0, uint32_t x1, uint32_t x2,
                                           uint32_t x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t m0 = static_cast<uint64_t>(0xD2511F53u) * x0;
    const uint64_t m1 = static_cast<uint64_t>(0xCD9E8D57u) * x2;
    const uint32_t y0 = static_cast<uint32_t>(m1 >> 32) ^ x1 ^ k0;
    const uint32_t y2 = static_cast<uint32_t>(m0 >> 32) ^ x3 ^ k1;
    x1 = static_cast<uint32_t>(m1);
    x3 = static_cast<uint32_t>(m0);
    x0 = y0;
    x2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block4{x0, x1, x2, x3};
}

__device__ __forceinline__ uint32_t word_of(const Block4 &b, int j) {
  return j == 0 ? b.w0 : (j == 1 ? b.w1 : (j == 2 ? b.w2 : b.w3));
}

// Initial point: tag 1, block 0; coordinate c = (word c >> 8) * 2^-24.
template <typename real, int DIM>
__device__ __forceinline__ void initial_point(uint32_t pid, uint32_t instance,
                                              uint32_t k0, uint32_t k1, real p[DIM]) {
  const Block4 w = philox10(pid, 0u, instance, 1u, k0, k1);
  const real s = static_cast<real>(1.0 / 16777216.0);
  p[0] = static_cast<real>(w.w0 >> 8) * s;
  p[1] = static_cast<real>(w.w1 >> 8) * s;
  if constexpr (DIM == 3) p[2] = static_cast<real>(w.w2 >> 8) * s;
}

// Starting position of point n: the initial point of a fresh game, or, for
// a continued run, the position stored in `state` after the steps already
// taken (lanes past the run's end read nothing and take zeros).
template <typename real, int DIM>
__device__ __forceinline__ void start_point(const RunArgs &ra, uint32_t pid, uint32_t n,
                                            bool active, const void *state, real p[DIM]) {
  if (ra.iter_block) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) p[c] = static_cast<real>(0);
    if (active) {
      const real *s = static_cast<const real *>(state) + static_cast<size_t>(n) * DIM;
#pragma unroll
      for (int c = 0; c < DIM; ++c) p[c] = s[c];
    }
  } else {
    initial_point<real, DIM>(pid, ra.instance, ra.k0, ra.k1, p);
  }
}

// ---------------------------------------------------------------------------
// Selection.  Equal probabilities: k = floor(u n / 2^32) (one mul_hi).
// Otherwise k = the number of finite thresholds <= u (the inverse CDF),
// found with a guide table (Chen and Asau, 1974): the top kGuideBits bits of
// u name a bucket whose entry holds lo = #{thresholds <= bucket start} and
// hi = #{thresholds <= bucket end}; k = lo + #{i in [lo, hi) : th[i] <= u},
// and lo == hi for all but at most n - 1 buckets.  Same result as a search
// over all thresholds, in one LDS read for most draws.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int select_equal(uint32_t u, uint32_t n) {
  return static_cast<int>(__umulhi(u, n));
}

__device__ __forceinline__ int select_table(uint32_t u, const uint32_t *__restrict__ th) {
  const uint32_t g = th[kMaxMaps + (u >> (32 - kGuideBits))];
  int k = static_cast<int>(g & 0xFFFFu);
  const int hi = static_cast<int>(g >> 16);
  for (int i = k; i < hi; ++i) k += th[i] <= u ? 1 : 0;
  return k;
}

// SEL: kSelTable, kSelEqual (compile-time rule) or kSelRuntime (equal when
// n_search == 0; used where one kernel serves systems of both kinds).
constexpr int kSelTable = 0;
constexpr int kSelEqual = 1;
constexpr int kSelRuntime = 2;

template <int SEL>
__device__ __forceinline__ int select_index(uint32_t u, const uint32_t *th, int n_maps, int n_search) {
  if constexpr (SEL == kSelEqual) {
    return select_equal(u, static_cast<uint32_t>(n_maps));
  } else if constexpr (SEL == kSelTable) {
    return select_table(u, th);
  } else {
    return n_search == 0 ? select_equal(u, static_cast<uint32_t>(n_maps)) : select_table(u, th);
  }
}

// ---------------------------------------------------------------------------
// Map table rows in LDS.  2D rows are 8 values: a00 a01 a10 a11 b0 b1, the
// map kind (1 = circle) and padding; 3D rows hold A row-major then b.
// ---------------------------------------------------------------------------
template <typename real, int DIM>
struct RowStride {
  static constexpr int value = (DIM == 2) ? 8 : 12;
};

__device__ __forceinline__ float atan2_r(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double atan2_r(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ void sincos_m(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ __forceinline__ void sincos_m(double a, double *s, double *c) { sincos(a, s, c); }

// The circle map of Section 3's circle equation (reading in cfs.h): radius
// sqrt(v), angle pi (u + f) for u = |p|^2 and v = polar angle / (2 pi).
template <typename real>
__device__ __forceinline__ void circle_map(real f, real p[2]) {
  const real two_pi = static_cast<real>(6.283185307179586476925286766559);
  const real u = p[0] * p[0] + p[1] * p[1];
  real th = atan2_r(p[1], p[0]);
  if (th < static_cast<real>(0)) th += two_pi;
  const real r2 = sqrt(th / two_pi);
  const real th2 = static_cast<real>(0.5) * two_pi * (u + f);
  real s, c;
  sincos_m(th2, &s, &c);
  p[0] = r2 * c;
  p[1] = r2 * s;
}

// Apply map k.  `flags & kFlagCircle` (uniform) says whether any map is not
// affine; the branch on the kind then diverges only where a wave holds both.
template <typename real, int DIM>
__device__ __forceinline__ void apply_map(const real *__restrict__ table, int k, real p[DIM],
                                          int flags = 0) {
  const real *r = table + k * RowStride<real, DIM>::value;
  if constexpr (DIM == 2) {
    if ((flags & kFlagCircle) && r[6] != static_cast<real>(0)) {
      circle_map<real>(r[4], p);
      return;
    }
    // two fused multiply-adds per coordinate
    const real x = p[0], y = p[1];
    p[0] = fma(r[0], x, fma(r[1], y, r[4]));
    p[1] = fma(r[2], x, fma(r[3], y, r[5]));
  } else {
    const real x = p[0], y = p[1], z = p[2];
    p[0] = fma(r[0], x, fma(r[1], y, fma(r[2], z, r[9])));
    p[1] = fma(r[3], x, fma(r[4], y, fma(r[5], z, r[10])));
    p[2] = fma(r[6], x, fma(r[7], y, fma(r[8], z, r[11])));
  }
}

// Systems whose maps all share one linear part A (the similarity maps of the
// Sierpinski triangle, the square and the Menger sponge): A is uniform over
// the workgroup and kept in registers, and only the translation b_k is
// gathered from LDS by the drawn index (a third or a quarter of the bytes of
// a whole row).  With A = s I (kLinScalar) the map is one FMA per
// coordinate, fma(s, p_i, b_i): the general map's FMAs with the zero
// entries add exact zeros, so the result is the same (the host takes this
// form only without negative-zero translations, whose sign the zero
// products could change).
template <typename real, int DIM>
struct SharedLinear {
  real a[DIM * DIM];
};

template <typename real, int DIM>
__device__ __forceinline__ SharedLinear<real, DIM> shared_linear(const MapTable<DIM> &mt) {
  SharedLinear<real, DIM> A;
#pragma unroll
  for (int i = 0; i < DIM * DIM; ++i) A.a[i] = static_cast<real>(mt.coef[i]);
  return A;
}

template <typename real, int DIM, int LIN>
__device__ __forceinline__ void apply_shared_map(const real *__restrict__ btab,
                                                 const SharedLinear<real, DIM> &A, int k,
                                                 real p[DIM]) {
  const real *b = btab + k * BRowStride<DIM>::value;
  if constexpr (LIN == kLinScalar) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) p[c] = fma(A.a[0], p[c], b[c]);
  } else if constexpr (DIM == 2) {
    const real x = p[0], y = p[1];
    p[0] = fma(A.a[0], x, fma(A.a[1], y, b[0]));
    p[1] = fma(A.a[2], x, fma(A.a[3], y, b[1]));
  } else {
    const real x = p[0], y = p[1], z = p[2];
    p[0] = fma(A.a[0], x, fma(A.a[1], y, fma(A.a[2], z, b[0])));
    p[1] = fma(A.a[3], x, fma(A.a[4], y, fma(A.a[5], z, b[1])));
    p[2] = fma(A.a[6], x, fma(A.a[7], y, fma(A.a[8], z, b[2])));
  }
}

__device__ inline void load_sincos_table();

// Copy the kernel-argument map table into LDS rows of type `real`, the
// selection thresholds and their guide; FP64 kernels (TRIG) also fill the
// sine/cosine table of sincos_f64.
// SHARED: the translations-only table of a shared-linear-part system
// (BRowStride values per map) instead of whole rows.
template <typename real, int DIM, bool TRIG = (sizeof(real) == sizeof(double)), bool SHARED = false>
__device__ __forceinline__ void load_table(const MapTable<DIM> &mt, real *table,
                                           uint32_t *th) {
  constexpr int S = RowStride<real, DIM>::value;
  constexpr int C = DIM * (DIM + 1);
  if constexpr (SHARED) {
    constexpr int BS = BRowStride<DIM>::value;
    for (int i = threadIdx.x; i < mt.n_maps * BS; i += blockDim.x) {
      const int m = i / BS, c = i % BS;
      table[i] = c < DIM ? static_cast<real>(mt.coef[m * C + DIM * DIM + c]) : static_cast<real>(0);
    }
  }
  for (int i = threadIdx.x; !SHARED && i < mt.n_maps * S; i += blockDim.x) {
    const int m = i / S, c = i % S;
    real v = static_cast<real>(0);
    if constexpr (DIM == 2) {
      if (c < 6)
        v = static_cast<real>(mt.coef[m * C + c]);
      else if (c == 6)
        v = static_cast<real>((mt.circle_mask >> m) & 1ull);
    } else {
      v = static_cast<real>(mt.coef[m * C + c]);
    }
    table[i] = v;
  }
  const int n_th = mt.n_search > 0 ? mt.n_search - 1 : 0;
  for (int i = threadIdx.x; i < n_th; i += blockDim.x) th[i] = mt.thresh[i];
  // guide buckets from the (uniform) thresholds in the kernel arguments
  for (int b = threadIdx.x; b < kGuide; b += blockDim.x) {
    const uint32_t first = static_cast<uint32_t>(b) << (32 - kGuideBits);
    const uint32_t last = first | ((1u << (32 - kGuideBits)) - 1u);
    uint32_t lo = 0, hi = 0;
    for (int i = 0; i < n_th; ++i) {
      lo += mt.thresh[i] <= first ? 1u : 0u;
      hi += mt.thresh[i] <= last ? 1u : 0u;
    }
    th[kMaxMaps + b] = lo | (hi << 16);
  }
  if constexpr (TRIG) load_sincos_table();
}

// ---------------------------------------------------------------------------
// Composed transforms on the copy q of p (p is never modified).
// ---------------------------------------------------------------------------
// FP64 sine and cosine for the transforms, by table and angle addition.
// k = rint(128 a / pi) and r = a - k pi/128 by Cody and Waite's reduction
// (Software Manual for the Elementary Functions, 1980) with a three-part
// constant whose first two parts have 33 significant bits (exact products
// for |k| < 2^20), so |r| <= pi/256.  sin r and cos r are their Taylor series
// to degree 5 and 6 (truncation below 1e-17), and
//   sin a = S_j cos r + C_j sin r,  cos a = C_j cos r - S_j sin r,
// with (S_j, C_j) = (sin, cos)(j pi/128), j = k mod 256, from a table in LDS
// that every workgroup of an FP64 kernel fills once with the library routine
// (load_table does it).  Arguments with |a| >= 25000, infinite or NaN take
// the library's sincos in a function of its own (its registers stay out of
// the calling loop); no lane of the workloads here does.
constexpr int kSinCosTable = 256;
__shared__ double2 s_sincos[kSinCosTable];

// Out of line (the rare wide-angle case), returning in registers: results
// passed back through memory would leave loads in flight at the join with
// the inline path, and the wait for them (the memory counter is in order)
// would also wait for every store the kernel has in flight, such as the
// binned splat's record writes.
__device__ __noinline__ double2 sincos_f64_wide(double a) {
  double sn, cs;
  sincos(a, &sn, &cs);
  return make_double2(sn, cs);
}

__device__ inline void load_sincos_table() {
  for (int i = threadIdx.x; i < kSinCosTable; i += blockDim.x) {
    const double x = fma(static_cast<double>(i), 0x1.921fb54400000p-6,
                         static_cast<double>(i) * 0x1.0b4611a600000p-40);
    double sn, cs;
    sincos(x, &sn, &cs);
    s_sincos[i] = make_double2(sn, cs);
  }
}

__device__ __forceinline__ void sincos_f64(double a, double *sn, double *cs) {
  if (!(fabs(a) < 25000.0)) {
    const double2 w = sincos_f64_wide(a);
    *sn = w.x;
    *cs = w.y;
    return;
  }
  const double k = rint(a * 40.743665431525205956834243423364);
  double r = fma(-k, 0x1.921fb54400000p-6, a);
  r = fma(-k, 0x1.0b4611a600000p-40, r);
  r = fma(-k, 0x1.3198a2e037073p-75, r);
  const double2 t = s_sincos[static_cast<int>(k) & (kSinCosTable - 1)];
  const double z = r * r;
  const double sr = fma(r * z, fma(z, 1.0 / 120.0, -1.0 / 6.0), r);
  const double cr = fma(z, fma(z, fma(z, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  *sn = fma(t.x, cr, t.y * sr);
  *cs = fma(t.y, cr, -(t.x * sr));
}

// FP64 square root for the transforms (a radius that feeds an angle or a
// scale): the hardware reciprocal square root estimate, one coupled Newton
// step on (sqrt a, 1 / (2 sqrt a)) and a final residual correction, which
// lands within an ulp or two; a <= 1e-300 gives 0.
__device__ __forceinline__ double sqrt_f64(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y;
  double h = 0.5 * y;
  const double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double d = fma(-g, g, a);
  g = fma(d, h, g);
  return a > 1e-300 ? g : 0.0;
}

// FP64 reciprocal for the camera's perspective divide: the hardware estimate
// and two Newton steps (within an ulp or two of 1 / a; one estimate and four
// FMAs in place of the two correctly rounded divisions' longer sequences).
// 0 gives infinity, whose projection is then dropped with the depth test.
__device__ __forceinline__ double rcp_f64(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  r = fma(r, fma(-a, r, 1.0), r);
  return r;
}

__device__ __forceinline__ float rcp_r(float a) { return 1.0f / a; }
__device__ __forceinline__ double rcp_r(double a) { return rcp_f64(a); }
__device__ __forceinline__ void sincos_r(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ __forceinline__ void sincos_r(double a, double *s, double *c) { sincos_f64(a, s, c); }
__device__ __forceinline__ float sqrt_r(float a) { return sqrtf(a); }
__device__ __forceinline__ double sqrt_r(double a) { return sqrt_f64(a); }
__device__ __forceinline__ float cos_r(float a) { return cosf(a); }
__device__ __forceinline__ double cos_r(double a) { return cos(a); }

template <typename real, int FINAL, int DIM, typename P = float>
__device__ __forceinline__ void final_transform(const P *__restrict__ fp, const real p[DIM],
                                                real q[2], real *depth) {
  if constexpr (FINAL == kFinalSwirl) {
    const real cx = fp[0], cy = fp[1], kappa = fp[2], tx = fp[3], ty = fp[4];
    const real dx = p[0] - cx, dy = p[1] - cy;
    const real r = sqrt_r(dx * dx + dy * dy);
    real s, c;
    sincos_r(kappa * r, &s, &c);
    q[0] = cx + tx + (c * dx - s * dy);
    q[1] = cy + ty + (s * dx + c * dy);
  } else if constexpr (FINAL == kFinalStretch) {
    q[0] = static_cast<real>(fp[0]) * p[0];
    q[1] = p[1] - static_cast<real>(fp[1]) * cos_r(p[0]);
  } else if constexpr (FINAL == kFinalRing) {
    const real ri = fp[0], ro = fp[1];
    const real r2 = p[0] * p[0] + p[1] * p[1];
    const real R = sqrt_r(ri * ri + (ro * ro - ri * ri) * r2);
    if (r2 > static_cast<real>(0)) {
      const real r = sqrt_r(r2);
      q[0] = R * (p[0] / r);
      q[1] = R * (p[1] / r);
    } else {
      q[0] = R;
      q[1] = static_cast<real>(0);
    }
  } else if constexpr (FINAL == kFinalTwistCamera) {
    const real wx = p[0] - static_cast<real>(fp[1]);
    const real wy = p[1] - static_cast<real>(fp[2]);
    const real wz = p[2] - static_cast<real>(fp[3]);
    real s, c;
    sincos_r(static_cast<real>(fp[0]) * wy, &s, &c);
    const real tx = c * wx - s * wz;
    const real tz = s * wx + c * wz;
    const real vx = fp[4] * tx + fp[5] * wy + fp[6] * tz + fp[7];
    const real vy = fp[8] * tx + fp[9] * wy + fp[10] * tz + fp[11];
    const real vz = fp[12] * tx + fp[13] * wy + fp[14] * tz + fp[15];
    const real inv = rcp_r(vz);
    q[0] = static_cast<real>(fp[16]) * vx * inv;
    q[1] = static_cast<real>(fp[17]) * vy * inv;
    *depth = vz;
  } else {
    q[0] = p[0];
    q[1] = p[1];
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b to XCD
// b mod 8) and every XCD has an L2 of its own.  Kernels whose neighbouring
// items share cache lines of their input (the runs of adjacent image tiles
// are adjacent in every chunk of records) take item xcd_item(b, n) instead of
// b: XCD x then works through one contiguous range of the n items.  A
// bijection of [0, n) for every n.
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t n) {
  const uint32_t x = b & 7u, j = b >> 3, q = n >> 3, r = n & 7u;
  return x * q + (x < r ? x : r) + j;
}

// Pixel of q in the window, or -1 when it is dropped (outside or NaN).
template <typename real>
__device__ __forceinline__ int bin_pixel(const real q[2], const Window &w, int *ix_out) {
  const real fx = (q[0] - static_cast<real>(w.lo[0])) * static_cast<real>(w.scale[0]);
  const real fy = (q[1] - static_cast<real>(w.lo[1])) * static_cast<real>(w.scale[1]);
  if (!(fx >= static_cast<real>(0) && fx < static_cast<real>(w.width))) return -1;
  if (!(fy >= static_cast<real>(0) && fy < static_cast<real>(w.height))) return -1;
  const int ix = static_cast<int>(fx);
  const int iy = static_cast<int>(fy);
  *ix_out = ix;
  return iy * w.width + ix;
}

}  // namespace cfs
