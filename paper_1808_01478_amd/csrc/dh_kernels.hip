// gfx950 kernels of libdisthist: staging, the LDS-histogram pair kernel,
// output zeroing, out-of-range counts and the per-pair probe.
//
// The pair kernel is persistent: a grid of a few workgroups per CU drains a
// work list of (frame, histogram, bin window, i-block, j-range) items through
// an atomic counter. Per item, every lane keeps R i-particles in registers;
// the workgroup streams the j-range through a double-buffered LDS tile with
// coalesced loads, and every wave reads each j as a uniform (broadcast) LDS
// load. Each pair's bin is counted with one ds_add_u32 into a u32 LDS
// sub-histogram (Sec. 2.4: groups of processing units share a private
// histogram; Sec. 3.2.3: partial histograms in on-chip memory). Lanes whose
// pair must not count (out of range, j <= i on a diagonal block, ragged
// i-block tail) are steered by a clamp to a per-lane discard slot past the
// bin window instead of a branch, so the atomic is issued without divergence
// and discarded pairs never collide on one address. When the histogram,
// window or frame changes, or before any u32 slot could wrap, the workgroup
// sums its copies and adds them to the uint64 output with global atomics
// (Sec. 3.1: u32 private histograms flushed into a u64 global one).
//
// Histograms too wide for LDS either run as bin windows (one LDS window per
// item, the shared-memory kernel's sweeps of Sec. 3.2.3) or, in the global
// mode, count every in-range pair with one uint64 atomic straight into the
// output (the global-memory kernel of Sec. 3.2.2); the host picks the mode.
#include "dh_internal.h"

#include <algorithm>
#include <type_traits>

namespace dh {
namespace {

template <typename T>
struct V4;
template <>
struct V4<float> { using type = float4; };
template <>
struct V4<double> { using type = double4; };

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// s_waitcnt immediates (gfx9 encoding: vmcnt bits [3:0] and [15:14], expcnt
// [6:4], lgkmcnt [11:8]); a field at its maximum does not wait.
constexpr int kWaitVm0 = 0x0F70;    // vmcnt(0)
constexpr int kWaitLgkm0 = 0xC07F;  // lgkmcnt(0)
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

// --------------------------------------------------------------------------
// Distance arithmetic
// --------------------------------------------------------------------------

__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }

// binary64, canonical op sequence (Algorithm 1 with Eq. 5), no contraction.
struct Geo64 {
  double s, L0, L1, L2, iL0, iL1, iL2;
  double ax, bx, by, cx, cy, cz, h11, h12, h13, h22, h23, h33;
  const double (*shift)[3];
};

__device__ __forceinline__ Geo64 load_geo64(const FrameParams *F) {
  Geo64 g;
  g.s = uni(F->s);
  g.L0 = uni(F->L[0]); g.L1 = uni(F->L[1]); g.L2 = uni(F->L[2]);
  g.iL0 = uni(F->iL[0]); g.iL1 = uni(F->iL[1]); g.iL2 = uni(F->iL[2]);
  g.ax = uni(F->ax); g.bx = uni(F->bx); g.by = uni(F->by);
  g.cx = uni(F->cx); g.cy = uni(F->cy); g.cz = uni(F->cz);
  g.h11 = uni(F->h11); g.h12 = uni(F->h12); g.h13 = uni(F->h13);
  g.h22 = uni(F->h22); g.h23 = uni(F->h23); g.h33 = uni(F->h33);
  g.shift = F->shift64;
  return g;
}

// Fractional coordinates B^-1 x of a point (the rows of Eq. 5's reduction
// applied to a position instead of a difference).
__device__ __forceinline__ void frac64(double x, double y, double z, const Geo64 &g,
                                       double (&sg)[3]) {
  sg[0] = fma(z, g.h13, fma(y, g.h12, x * g.h11));
  sg[1] = fma(z, g.h23, y * g.h22);
  sg[2] = z * g.h33;
}

// Correctly rounded binary64 square root (IEEE-754 sqrt) for every
// argument. The candidate y comes from v_rsq_f64 refined by one Goldschmidt
// step and two Newton corrections with fused residuals, which leaves y within
// half an ulp plus a tiny fraction of sqrt(q): at most one ulp from the
// correctly rounded root. Tuckerman's rounding test then settles the last
// bit. With u = ulp(y) and the remainder r = q - y*y (one fma), sqrt(q) lies
// above the midpoint y + u/2 iff r > u*y, and below the midpoint under y iff
// r <= -u*y (-u*y/2 when y is a power of two, whose lower neighbour is only
// u/2 away): q and y*y are multiples of u*u, so r is too, and the midpoint
// conditions r < u*y + u*u/4 and r > -u*y + u*u/4 reduce to those
// thresholds. The thresholds and the next multiples of u*u beyond them are
// representable, so the comparisons are exact even where the fma rounds r.
// Arguments below 2^-767 are scaled by 2^1024 (exactly) so that the
// iteration and the remainder stay in the normal range, and the root is
// scaled back by 2^-512; 0, +inf and NaN are returned as IEEE sqrt returns
// them.
__device__ __forceinline__ double sqrt_cr(double q) {
  const bool tiny = q < 0x1p-767;
  const double qs = tiny ? ldexp(q, 1024) : q;
  const double y0 = __builtin_amdgcn_rsq(qs);
  double g = qs * y0;
  double h = 0.5 * y0;
  const double e = fma(-h, g, 0.5);
  h = fma(h, e, h);
  g = fma(g, e, g);
  double d = fma(-g, g, qs);
  g = fma(d, h, g);
  d = fma(-g, g, qs);
  double y = fma(d, h, g);
  const double r = fma(-y, y, qs);
  const uint64_t yb = static_cast<uint64_t>(__double_as_longlong(y));
  // y = f * 2^ex with f in [1/2, 1); y is normal here
  const int ex = static_cast<int>((yb >> 52) & 0x7ff) - 1022;
  const double uy = ldexp(y, ex - 53);  // ulp(y) * y, exact
  const bool pow2 = (yb & 0xFFFFFFFFFFFFFull) == 0;
  const double low = pow2 ? -0.5 * uy : -uy;
  const uint64_t step = r > uy ? 1ull : (r <= low ? ~0ull : 0ull);
  y = __longlong_as_double(static_cast<long long>(yb + step));
  if (tiny) y = ldexp(y, -512);
  if (qs > 0.0 && qs <= 0x1.fffffffffffffp+1023) return y;
  return q == 0.0 ? q : (q > 0.0 ? q : __builtin_nan(""));
}

// The scaled distance t = sqrt(q) * s from a short root: v_rsq_f64 (relative
// error at most 2^-23, the precision the ISA states for it) and one
// Goldschmidt step, with s folded into the step's last fma (g s (1 + e)
// instead of (g (1 + e)) s: one dependent step less), give t within about
// 1.5 * 2^-46 relative plus three roundings, so it lies within 2^13 ulps of
// the canonical t (correctly rounded root times s).
// It decides the bin whenever it is farther than 2^16 ulps from every
// integer. For t < 2^20 the integers are multiples of 2^32 ulps of t, so t
// is that far from every integer when the low 32 bits of its encoding are
// at least 2^16 away from a multiple of 2^32, i.e. when lo + 2^16 (mod 2^32)
// is at least 2^17, lo being those bits (a conservative test). The caller
// keeps the smallest lo + 2^16 of its pairs per lane in `gap` (a minimum the
// compiler forms three at a time) and takes the correctly rounded root for
// all of them when any lane's gap is below 2^17 (one ballot). Every t at or above 2^20 is
// out of range, as is the canonical t, when n_bins < 2^20 - 2; with more
// bins the callers take the correctly rounded root for every pair. The
// bound holds for every normal q (all intermediates stay normal). q = 0
// gives t = 0 * inf = NaN, whose encoding ends in 32 zero bits, so the test
// flags it; so it does for a subnormal q if v_rsq_f64 flushed it (q * inf,
// then inf - inf). Otherwise, for subnormal q the canonical t is below
// 2^-511 s, under 2^-11 when s < 2^500 (the callers take the correctly
// rounded root for every pair beyond that), and the short root, within a
// few ulps of it, falls in bin 0 as well. A NaN t (q = +inf or NaN) counts
// out of range like the canonical one.
__device__ __forceinline__ double t_fast64(double q, double s, uint32_t &gap) {
  const double y = __builtin_amdgcn_rsq(q);
  const double g = q * y;
  const double h = 0.5 * y;
  const double e = fma(-h, g, 0.5);
  const double gs = g * s;
  const double t = fma(gs, e, gs);
  gap = min(gap, static_cast<uint32_t>(__double_as_longlong(t)) + 0x10000u);
  return t;
}

// Initial gap of a group of pairs: 0 (the correctly rounded root for every
// pair) when the histogram has 2^20 - 2 bins or more or s is huge (big_bins,
// see run_item), else no pair yet.
__device__ __forceinline__ uint32_t gap_init(bool big_bins) { return big_bins ? 0u : ~0u; }

// Whether any lane of the wave has a pair whose short t may lie near an
// integer (a uniform answer).
__device__ __forceinline__ bool any_near(uint32_t gap) {
  return __builtin_amdgcn_ballot_w64(gap < 0x20000u) != 0;
}

// t with the canonical arithmetic for one pair: the short root, or, when any
// lane of the wave needs it, the correctly rounded one (a uniform branch).
__device__ __forceinline__ double t_guarded64(double q, double s, bool big_bins) {
  uint32_t gap = gap_init(big_bins);
  const double t = t_fast64(q, s, gap);
  if (__builtin_expect(any_near(gap), 0)) return sqrt_cr(q) * s;
  return t;
}

// d = x_j - x_i reduced by the minimum-image rule of the box kind.
template <int BOX>
__device__ __forceinline__ void reduce64(double xi, double yi, double zi, double xj, double yj,
                                         double zj, const Geo64 &g, double &dx, double &dy,
                                         double &dz) {
  dx = xj - xi;
  dy = yj - yi;
  dz = zj - zi;
  if constexpr (BOX == kBoxOrtho || BOX == kBoxCube) {
    const double n0 = rint(dx * g.iL0), n1 = rint(dy * g.iL1), n2 = rint(dz * g.iL2);
    dx = fma(-g.L0, n0, dx);
    dy = fma(-g.L1, n1, dy);
    dz = fma(-g.L2, n2, dz);
  } else if constexpr (BOX == kBoxTric || BOX == kBoxTricSearch) {
    const double sc = dz * g.h33;
    const double sb = fma(dz, g.h23, dy * g.h22);
    const double sa = fma(dz, g.h13, fma(dy, g.h12, dx * g.h11));
    const double na = rint(sa), nb = rint(sb), nc = rint(sc);
    dz = fma(-g.cz, nc, dz);
    dy = fma(-g.cy, nc, fma(-g.by, nb, dy));
    dx = fma(-g.cx, nc, fma(-g.bx, nb, fma(-g.ax, na, dx)));
  }
}

// Minimum of q over the 27 images d + S (S = 0 gives q itself). Every q is
// a sum of squares (never -0), so fmin equals the select v < q ? v : q,
// NaN included (a NaN d makes every image NaN); the minimum of such values
// does not depend on the order, so three running minima give the chain
// more independent work.
__device__ __forceinline__ double search_q64(double dx, double dy, double dz, double q,
                                             const Geo64 &g) {
  double qa = q, qb = q, qc = q;
#pragma unroll
  for (int m = 0; m < kShifts; m += 3) {
    double v[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const double vx = dx + uni(g.shift[m + u][0]);
      const double vy = dy + uni(g.shift[m + u][1]);
      const double vz = dz + uni(g.shift[m + u][2]);
      v[u] = fma(vz, vz, fma(vy, vy, vx * vx));
    }
    qa = fmin(qa, v[0]);
    qb = fmin(qb, v[1]);
    qc = fmin(qc, v[2]);
  }
  return fmin(qa, fmin(qb, qc));
}

template <int BOX>
__device__ __forceinline__ double t64(double xi, double yi, double zi, double xj, double yj,
                                      double zj, const Geo64 &g) {
  double dx, dy, dz;
  reduce64<BOX>(xi, yi, zi, xj, yj, zj, g, dx, dy, dz);
  double q = fma(dz, dz, fma(dy, dy, dx * dx));
  if constexpr (BOX == kBoxTricSearch) q = search_q64(dx, dy, dz, q, g);
  return sqrt_cr(q) * g.s;
}

// q of the canonical sequence before the root (no image search)
template <int BOX>
__device__ __forceinline__ double q64(double xi, double yi, double zi, double xj, double yj,
                                      double zj, const Geo64 &g) {
  double dx, dy, dz;
  reduce64<BOX>(xi, yi, zi, xj, yj, zj, g, dx, dy, dz);
  return fma(dz, dz, fma(dy, dy, dx * dx));
}

// binary32. Without a box the staged coordinates are x * s, so the
// Euclidean length is already t. With a periodic cell they are 32-bit
// fixed-point fractional coordinates: the wrapped difference u_j - u_i read as
// a signed integer is 2^32 times the Eq. 5 reduced fractional difference, so
// the minimum image costs one integer subtraction per axis; converting it to
// float and applying the cell matrix scaled by s / 2^32 gives t units.
struct Geo32 {
  float kx, ky, kz;                 // orthorhombic: L_c * s / 2^32
  float ry, rz;                     // orthorhombic: (L_y / L_x)^2, (L_z / L_x)^2
  float ax, bx, by, cx, cy, cz;     // triclinic: cell matrix * s / 2^32
  float nbx, nby, ncx, ncy, ncz;    // triclinic: cell matrix / a_x
  const float (*shift)[3];          // image shifts * s
};

__device__ __forceinline__ Geo32 load_geo32(const FrameParams *F) {
  Geo32 g;
  g.kx = uni(F->k32[0]); g.ky = uni(F->k32[1]); g.kz = uni(F->k32[2]);
  g.ry = uni(F->ryz32[0]); g.rz = uni(F->ryz32[1]);
  g.ax = uni(F->Bk[0]); g.bx = uni(F->Bk[1]); g.by = uni(F->Bk[2]);
  g.cx = uni(F->Bk[3]); g.cy = uni(F->Bk[4]); g.cz = uni(F->Bk[5]);
  g.nbx = uni(F->Bn[0]); g.nby = uni(F->Bn[1]); g.ncx = uni(F->Bn[2]);
  g.ncy = uni(F->Bn[3]); g.ncz = uni(F->Bn[4]);
  g.shift = F->shift32;
  return g;
}

// reduced fractional difference, units of 2^-32 of the cell vector
__device__ __forceinline__ float frac_diff(float ui, float uj) {
  return static_cast<float>(static_cast<int32_t>(__float_as_uint(uj) - __float_as_uint(ui)));
}

template <int BOX>
__device__ __forceinline__ float t32_packed(uint64_t ab_j, uint64_t neg_ab_i, float zi, float zj,
                                            const Geo32 &g);
template <int BOX>
__device__ __forceinline__ float t32_packed_c(uint64_t ab_j, uint64_t neg_ab_i, float fc,
                                              const Geo32 &g);

// Binary32 bins without a float-to-integer conversion: t + (2^23 - 1/2)
// rounded to nearest lies in [2^23, 2^24) for 1/2 <= t < 2^22, where the
// spacing is 1, so its bits minus those of 2^23 are floor(t), except at an
// integer t: that is a tie, which goes to the even neighbour, so an odd
// integer t counts one bin lower (a pair at a bin edge, inside the binary32
// tolerance). For t < 1/4 the difference is -1 (bin 0; the counting code
// maps it there); it grows monotonically with t and is at least 2^22 for
// t >= 2^22, +inf and NaN (read as unsigned). Binary32 histograms have at
// most 2^22 bins, so a pair counts iff the difference is below n_bins.
constexpr float kMagic32 = 8388607.5f;        // 2^23 - 1/2
constexpr int kGuardBytes = 16;               // >= 4 bytes per copy, 4 copies at most
constexpr uint32_t kMagicBits = 0x4B000000u;  // bits of 2^23

__device__ __forceinline__ uint32_t bin_bits32(float t) {
  return __float_as_uint(t + kMagic32);
}

// median of three unsigned values: x clamped to [lo, hi] when lo <= hi (the
// compiler forms v_med3_u32 only for constant bounds)
__device__ __forceinline__ uint32_t med3_u32(uint32_t x, uint32_t lo, uint32_t hi) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}

// min(a, b) for an a that is an arithmetic result (never a signalling NaN):
// one v_min_f64, without the canonicalisation fmin adds for arbitrary input.
// A NaN a gives b, as fmin does.
__device__ __forceinline__ double min_arith(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Minimum and maximum over the 64 lanes of a wave, as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(v, o)));
  return static_cast<uint32_t>(uni(static_cast<int>(v)));
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(v, o)));
  return static_cast<uint32_t>(uni(static_cast<int>(v)));
}

__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return uni(v);
}
__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return uni(v);
}

// Triclinic reduced vector (t units) from packed fractional words.
__device__ __forceinline__ void tric_vec32(uint64_t ab_j, uint64_t neg_ab_i, float zi, float zj,
                                           const Geo32 &g, float &dx, float &dy, float &dz) {
  const uint64_t dab = ab_j + neg_ab_i;
  const float fa = static_cast<float>(static_cast<int32_t>(static_cast<uint32_t>(dab)));
  const float fb = static_cast<float>(static_cast<int32_t>(static_cast<uint32_t>(dab >> 32)));
  const float fc = frac_diff(zi, zj);
  dx = fmaf(g.cx, fc, fmaf(g.bx, fb, g.ax * fa));
  dy = fmaf(g.cy, fc, g.by * fb);
  dz = g.cz * fc;
}

// Minimum of q over the 27 images (binary32, t units), three running minima.
__device__ __forceinline__ float search_q32(float dx, float dy, float dz, float q,
                                            const Geo32 &g) {
  float qa = q, qb = q, qc = q;
#pragma unroll
  for (int m = 0; m < kShifts; m += 3) {
    float v[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const float vx = dx + uni(g.shift[m + u][0]);
      const float vy = dy + uni(g.shift[m + u][1]);
      const float vz = dz + uni(g.shift[m + u][2]);
      v[u] = fmaf(vz, vz, fmaf(vy, vy, vx * vx));
    }
    qa = fminf(qa, v[0]);
    qb = fminf(qb, v[1]);
    qc = fminf(qc, v[2]);
  }
  return fminf(qa, fminf(qb, qc));
}

template <int BOX>
__device__ __forceinline__ float t32(float xi, float yi, float zi, float xj, float yj, float zj,
                                     const Geo32 &g) {
  if constexpr (BOX == kBoxNone) {
    const float dx = xj - xi, dy = yj - yi, dz = zj - zi;
    return __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));  // v_sqrt_f32
  } else {
    const uint64_t ai = (static_cast<uint64_t>(__float_as_uint(yi)) << 32) | __float_as_uint(xi);
    const uint64_t aj = (static_cast<uint64_t>(__float_as_uint(yj)) << 32) | __float_as_uint(xj);
    return t32_packed<BOX>(aj, 0ull - ai, zi, zj, g);
  }
}

// Periodic binary32 distance from packed fractional words: ab = (b << 32) | a
// of particle j and -(b << 32 | a) of particle i. One 64-bit addition gives
// both differences: the low word exactly, the high word lowered by one unit
// (2^-32 of a cell vector, far below binary32 rounding) when a borrows.
template <int BOX>
__device__ __forceinline__ float t32_packed(uint64_t ab_j, uint64_t neg_ab_i, float zi, float zj,
                                            const Geo32 &g) {
  return t32_packed_c<BOX>(ab_j, neg_ab_i, frac_diff(zi, zj), g);
}

// The same with the c difference given (as a float of fixed-point units).
template <int BOX>
__device__ __forceinline__ float t32_packed_c(uint64_t ab_j, uint64_t neg_ab_i, float fc,
                                              const Geo32 &g) {
  {
    const uint64_t dab = ab_j + neg_ab_i;
    const float fa = static_cast<float>(static_cast<int32_t>(static_cast<uint32_t>(dab)));
    const float fb = static_cast<float>(static_cast<int32_t>(static_cast<uint32_t>(dab >> 32)));
    if constexpr (BOX == kBoxCube) {
      return __builtin_amdgcn_sqrtf(fmaf(fc, fc, fmaf(fb, fb, fa * fa))) * g.kx;
    } else if constexpr (BOX == kBoxOrtho) {
      // q / kx^2, the y and z squares weighted by (L_y/L_x)^2 and (L_z/L_x)^2
      const float q = fmaf(fc * g.rz, fc, fmaf(fb * g.ry, fb, fa * fa));
      return __builtin_amdgcn_sqrtf(q) * g.kx;
    } else if constexpr (BOX == kBoxTric) {
      // d / (a_x s 2^-32): the cell matrix divided by a_x
      const float dx = fmaf(g.ncx, fc, fmaf(g.nbx, fb, fa));
      const float dy = fmaf(g.ncy, fc, g.nby * fb);
      const float dz = g.ncz * fc;
      return __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) * g.ax;
    } else {
      const float dx = fmaf(g.cx, fc, fmaf(g.bx, fb, g.ax * fa));
      const float dy = fmaf(g.cy, fc, g.by * fb);
      const float dz = g.cz * fc;
      float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      if constexpr (BOX == kBoxTricSearch) q = search_q32(dx, dy, dz, q, g);
      return __builtin_amdgcn_sqrtf(q);
    }
  }
}

// Bin bits (see bin_bits32) of the same distance; without the image search
// the scale (L_x or a_x times s / 2^32) and the offset are one fused
// multiply-add on the root.
template <int BOX>
__device__ __forceinline__ uint32_t bits32_packed_c(uint64_t ab_j, uint64_t neg_ab_i, float fc,
                                                    const Geo32 &g) {
  if constexpr (BOX == kBoxCube || BOX == kBoxOrtho || BOX == kBoxTric) {
    const uint64_t dab = ab_j + neg_ab_i;
    const float fa = static_cast<float>(static_cast<int32_t>(static_cast<uint32_t>(dab)));
    const float fb = static_cast<float>(static_cast<int32_t>(static_cast<uint32_t>(dab >> 32)));
    float q, k;
    if constexpr (BOX == kBoxCube) {
      q = fmaf(fc, fc, fmaf(fb, fb, fa * fa));
      k = g.kx;
    } else if constexpr (BOX == kBoxOrtho) {
      q = fmaf(fc * g.rz, fc, fmaf(fb * g.ry, fb, fa * fa));
      k = g.kx;
    } else {
      const float dx = fmaf(g.ncx, fc, fmaf(g.nbx, fb, fa));
      const float dy = fmaf(g.ncy, fc, g.nby * fb);
      const float dz = g.ncz * fc;
      q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      k = g.ax;
    }
    return __float_as_uint(fmaf(__builtin_amdgcn_sqrtf(q), k, kMagic32));
  } else {
    return bin_bits32(t32_packed_c<BOX>(ab_j, neg_ab_i, fc, g));
  }
}

// min(a, b) of two arithmetic results (never signalling NaNs), without the
// canonicalisation fmin adds; a NaN operand gives the other, as fmin does.
__device__ __forceinline__ float min_arith(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Minimum of q over the images in the search table from `base` (an octant
// row, or the 27 shift vectors), n of them (uniform), three running minima.
// Rows are padded with the zero shift, and a run past a row's end reads
// further table entries, which are images too, so the minimum is unchanged;
// images
// left out of an octant row cannot be nearer (see octant_images on the
// host), so it equals the one over all 27 images.
template <typename T>
__device__ __forceinline__ T search_oct(T dx, T dy, T dz, T q, int base, int n,
                                        const typename V4<T>::type *__restrict__ tab) {
  T qa = q, qb = q, qc = q;
  const typename V4<T>::type *row = tab + base;
  auto image = [&](int k) {
    const typename V4<T>::type S = row[k];
    const T vx = dx + S.x;
    const T vy = dy + S.y;
    const T vz = dz + S.z;
    return fmaT(vz, vz, fmaT(vy, vy, vx * vx));
  };
  int k = 0;
  for (; k + 2 < n; k += 3) {
    const T v0 = image(k), v1 = image(k + 1), v2 = image(k + 2);
    qa = min_arith(qa, v0);
    qb = min_arith(qb, v1);
    qc = min_arith(qc, v2);
  }
  for (; k < n; ++k) qa = min_arith(qa, image(k));
  return min_arith(qa, min_arith(qb, qc));
}

// Octant of a reduced binary64 vector: bit k when fractional component k is
// negative; 8 (the full list) when a component lies outside the octant boxes
// of the host (|f| beyond 1/2 plus half their slack, or NaN).
__device__ __forceinline__ int octant64(double dx, double dy, double dz, const Geo64 &g) {
  double f[3];
  frac64(dx, dy, dz, g, f);
  int code = 0;
  bool inside = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    code |= f[k] < 0.0 ? 1 << k : 0;
    inside = inside && fabs(f[k]) <= 0.5 + 0.5 * kOctSlack;
  }
  return inside ? code : 8;
}

// Octant of a reduced binary32 vector from its wrapped fixed-point
// differences (exact, within [-1/2, 1/2) of a cell vector).
__device__ __forceinline__ int octant32(uint64_t ab_j, uint64_t neg_ab_i, float zi, float zj) {
  const uint64_t dab = ab_j + neg_ab_i;
  return (static_cast<int32_t>(static_cast<uint32_t>(dab)) < 0 ? 1 : 0) |
         (static_cast<int32_t>(static_cast<uint32_t>(dab >> 32)) < 0 ? 2 : 0) |
         (static_cast<int32_t>(__float_as_uint(zj) - __float_as_uint(zi)) < 0 ? 4 : 0);
}

template <typename T>
struct Geo;
template <>
struct Geo<float> {
  using type = Geo32;
  static __device__ __forceinline__ Geo32 load(const FrameParams *F) { return load_geo32(F); }
};
template <>
struct Geo<double> {
  using type = Geo64;
  static __device__ __forceinline__ Geo64 load(const FrameParams *F) { return load_geo64(F); }
};

template <typename T, int BOX>
__device__ __forceinline__ T pair_t(T xi, T yi, T zi, T xj, T yj, T zj,
                                    const typename Geo<T>::type &g) {
  if constexpr (sizeof(T) == 4)
    return t32<BOX>(xi, yi, zi, xj, yj, zj, g);
  else
    return t64<BOX>(xi, yi, zi, xj, yj, zj, g);
}

// --------------------------------------------------------------------------
// Staging: binary64 [N][3] -> padded float4 / double4
// --------------------------------------------------------------------------

__global__ void stage64_kernel(const double *__restrict__ in, double4 *__restrict__ out,
                               int64_t n) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += step)
    out[i] = make_double4(in[3 * i], in[3 * i + 1], in[3 * i + 2], 0.0);
}

// 32-bit fixed-point image of a fractional coordinate: floor(2^32 * (f mod 1))
__device__ __forceinline__ float fixfrac(double f) {
  const double w = f - floor(f);
  const uint64_t u = static_cast<uint64_t>(w * 4294967296.0);
  return __uint_as_float(static_cast<uint32_t>(u));
}

// One staged binary32 point (see FrameParams for the formats).
template <int BOX>
__device__ __forceinline__ float4 stage_point32(double x, double y, double z,
                                                const FrameParams &p) {
  if constexpr (BOX == kBoxNone) {
    return make_float4(static_cast<float>(x * p.s), static_cast<float>(y * p.s),
                       static_cast<float>(z * p.s), 0.f);
  } else if constexpr (BOX == kBoxOrtho) {
    // c twice: the pair kernel reads (c : c) as one 64-bit word
    const float c = fixfrac(z * p.iL[2]);
    return make_float4(fixfrac(x * p.iL[0]), fixfrac(y * p.iL[1]), c, c);
  } else {
    const double fa = fma(z, p.h13, fma(y, p.h12, x * p.h11));
    const double fb = fma(z, p.h23, y * p.h22);
    const double fc = z * p.h33;
    const float c = fixfrac(fc);
    return make_float4(fixfrac(fa), fixfrac(fb), c, c);
  }
}

template <int BOX>
__global__ void stage32_kernel(const double *__restrict__ in, float4 *__restrict__ out, int64_t n,
                               FrameParams p) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += step)
    out[i] = stage_point32<BOX>(in[3 * i], in[3 * i + 1], in[3 * i + 2], p);
}

// --------------------------------------------------------------------------
// Spatially sorted binary32 staging (triclinic cells without image search)
// --------------------------------------------------------------------------
//
// The points of every species are put in the order of a Morton curve over
// their wrapped fractional coordinates (9 bits per axis), ties by input
// index, so that 64 consecutive points are close together in the cell. The
// pair kernel then finds, for most pairs of such groups, one lattice shift
// that is the Eq. 5 wrap of every pair of the two groups (see run_item).
// The order is a permutation within each species, so the histograms are
// those of the input; the sort is a bitonic network on 64-bit keys
// (species : Morton code : input index), which makes the order unique.

struct SpeciesOffsets {
  int64_t v[kMaxSpeciesStage + 1];
};

// Morton code of three 9-bit integers: bit b of axis a goes to bit 3b + a.
__device__ __forceinline__ uint64_t morton9(uint32_t a, uint32_t b, uint32_t c) {
  uint64_t m = 0;
#pragma unroll
  for (int bit = 0; bit < 9; ++bit)
    m |= (static_cast<uint64_t>((a >> bit) & 1u) << (3 * bit)) |
         (static_cast<uint64_t>((b >> bit) & 1u) << (3 * bit + 1)) |
         (static_cast<uint64_t>((c >> bit) & 1u) << (3 * bit + 2));
  return m;
}

// wrapped fractional coordinate as 32-bit fixed point (as fixfrac)
__device__ __forceinline__ uint32_t fix32(double f) {
  const double w = f - floor(f);
  return static_cast<uint32_t>(static_cast<uint64_t>(w * 4294967296.0));
}

__global__ void sort_keys_kernel(const double *__restrict__ in, int64_t n, int64_t npad,
                                 SpeciesOffsets off, int32_t k, FrameParams p,
                                 uint64_t *__restrict__ keys) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < npad;
       i += step) {
    if (i >= n) {
      keys[i] = ~0ull;
      continue;
    }
    int s = 0;
    while (s + 1 < k && off.v[s + 1] <= i) ++s;
    const double x = in[3 * i], y = in[3 * i + 1], z = in[3 * i + 2];
    const uint32_t ua = fix32(fma(z, p.h13, fma(y, p.h12, x * p.h11)));
    const uint32_t ub = fix32(fma(z, p.h23, y * p.h22));
    const uint32_t uc = fix32(z * p.h33);
    const uint64_t m = morton9(ua >> 23, ub >> 23, uc >> 23);
    keys[i] = (static_cast<uint64_t>(s) << 58) | (m << 31) | static_cast<uint64_t>(i);
  }
}

constexpr int kBitonicBlock = 2048;  // keys sorted in LDS by one workgroup of 1024

__device__ __forceinline__ void bitonic_cas(uint64_t &a, uint64_t &b, bool ascending) {
  if ((a > b) == ascending) {
    const uint64_t t = a;
    a = b;
    b = t;
  }
}

// All stages k <= kBitonicBlock of each block (first == true), or the steps
// j < kBitonicBlock of stage k (first == false), in LDS.
__global__ __launch_bounds__(1024) void bitonic_local_kernel(uint64_t *__restrict__ keys,
                                                             int64_t k_stage, int first) {
  __shared__ uint64_t sk[kBitonicBlock];
  const int t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kBitonicBlock;
  sk[t] = keys[base + t];
  sk[t + 1024] = keys[base + t + 1024];
  const int64_t k_lo = first ? 2 : k_stage, k_hi = first ? kBitonicBlock : k_stage;
  for (int64_t kk = k_lo; kk <= k_hi; kk <<= 1) {
    for (int j = kk / 2 < kBitonicBlock / 2 ? static_cast<int>(kk / 2) : kBitonicBlock / 2;
         j > 0; j >>= 1) {
      __syncthreads();
      const int lo = 2 * j * (t / j) + (t % j);
      const bool asc = ((base + lo) & kk) == 0;
      bitonic_cas(sk[lo], sk[lo + j], asc);
    }
  }
  __syncthreads();
  keys[base + t] = sk[t];
  keys[base + t + 1024] = sk[t + 1024];
}

// One step j >= kBitonicBlock of stage k over the whole array.
__global__ void bitonic_global_kernel(uint64_t *__restrict__ keys, int64_t npad, int64_t j,
                                      int64_t k_stage) {
  const int64_t half = npad / 2;
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < half;
       t += step) {
    const int64_t lo = 2 * j * (t / j) + (t % j);
    uint64_t a = keys[lo], b = keys[lo + j];
    bitonic_cas(a, b, (lo & k_stage) == 0);
    keys[lo] = a;
    keys[lo + j] = b;
  }
}

// Staged entry of the sorted position p: the fixed-point fractional words
// (a, b, c, c) as for the unsorted binary32 triclinic staging, then the
// Cartesian position of the same wrapped point relative to the cell centre,
// B (u - 1/2) with u the fixed-point fraction read back exactly, so the two
// formats describe one point.
__global__ void stage_sorted_kernel(const double *__restrict__ in,
                                    const uint64_t *__restrict__ keys, int64_t n, FrameParams p,
                                    float4 *__restrict__ out) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; q < n;
       q += step) {
    const int64_t i = static_cast<int64_t>(keys[q] & 0x7FFFFFFFull);
    const double x = in[3 * i], y = in[3 * i + 1], z = in[3 * i + 2];
    const uint32_t ua = fix32(fma(z, p.h13, fma(y, p.h12, x * p.h11)));
    const uint32_t ub = fix32(fma(z, p.h23, y * p.h22));
    const uint32_t uc = fix32(z * p.h33);
    const double va = ua * 0x1p-32 - 0.5, vb = ub * 0x1p-32 - 0.5, vc = uc * 0x1p-32 - 0.5;
    const float cx = static_cast<float>(fma(p.cx, vc, fma(p.bx, vb, p.ax * va)));
    const float cy = static_cast<float>(fma(p.cy, vc, p.by * vb));
    const float cz = static_cast<float>(p.cz * vc);
    out[2 * q] = make_float4(__uint_as_float(ua), __uint_as_float(ub), __uint_as_float(uc),
                             __uint_as_float(uc));
    out[2 * q + 1] = make_float4(cx, cy, cz, 0.f);
  }
}

// binary64: the input point of the sorted position q, unchanged.
__global__ void stage_sorted64_kernel(const double *__restrict__ in,
                                      const uint64_t *__restrict__ keys, int64_t n,
                                      double4 *__restrict__ out) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; q < n;
       q += step) {
    const int64_t i = static_cast<int64_t>(keys[q] & 0x7FFFFFFFull);
    out[q] = make_double4(in[3 * i], in[3 * i + 1], in[3 * i + 2], 0.0);
  }
}

// Batched staging: blockIdx.y selects the frame.
template <int PREC>
__global__ void stage_batch_kernel(const FrameParams *__restrict__ frames) {
  const FrameParams &p = frames[blockIdx.y];
  // spatially sorted frames are staged by their own sort
  if (p.box == kBoxTricSorted) return;
  const int64_t n = p.n_points;
  const double *__restrict__ in = p.in;
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += step) {
    const double x = in[3 * i], y = in[3 * i + 1], z = in[3 * i + 2];
    if constexpr (PREC == 1) {
      static_cast<double4 *>(const_cast<void *>(p.coords))[i] = make_double4(x, y, z, 0.0);
    } else {
      float4 v;
      if (p.box == kBoxNone)
        v = stage_point32<kBoxNone>(x, y, z, p);
      else if (p.box == kBoxOrtho || p.box == kBoxCube)
        v = stage_point32<kBoxOrtho>(x, y, z, p);
      else
        v = stage_point32<kBoxTric>(x, y, z, p);
      static_cast<float4 *>(const_cast<void *>(p.coords))[i] = v;
    }
  }
}

// Batched zeroing of every frame's histograms, plus the work counters.
__global__ void zero_batch_kernel(const FrameParams *__restrict__ frames, int32_t *counters,
                                  int32_t n_counters) {
  const FrameParams &p = frames[blockIdx.y];
  const int64_t n = static_cast<int64_t>(p.n_hist) * p.n_bins;
  const int64_t i0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (blockIdx.y == 0 && i0 < n_counters) counters[i0] = 0;
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = i0; i < n; i += step) p.out[i] = 0ull;
}

// Batched out-of-range counts: blockIdx.x = histogram, blockIdx.y = frame.
__global__ void oor_batch_kernel(const FrameParams *__restrict__ frames) {
  __shared__ unsigned long long part[256];
  const FrameParams &p = frames[blockIdx.y];
  const int h = blockIdx.x;
  if (p.oor == nullptr || h >= p.n_hist) return;
  unsigned long long v = 0;
  for (int b = threadIdx.x; b < p.n_bins; b += blockDim.x)
    v += p.out[static_cast<size_t>(h) * p.n_bins + b];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.oor[h] = p.pairs[h] - part[0];
}

// --------------------------------------------------------------------------
// Pair kernel
// --------------------------------------------------------------------------

// Adds the LDS copies of bins [0, count) into out[] and clears every slot.
// Copies are interleaved bin-major: slot b of copy c is word b * copies + c.
__device__ __forceinline__ void flush_hist(uint32_t *hist, const PairKernelArgs &a,
                                           const FrameParams *F, int hist_idx, int sweep) {
  const int n_bins = uni(F->n_bins);
  const int win = uni(F->win);
  const int b_lo = sweep * win;
  const int count = min(win, n_bins - b_lo);
  uint64_t *out = F->out + static_cast<size_t>(hist_idx) * n_bins + b_lo;
  // the whole stride: slots past the window may hold counts of out-of-range
  // pairs of unclamped items, and the next frame may use a wider window
  const int clear = a.stride;
  uint64_t in_range = 0;
  for (int b = threadIdx.x; b < clear; b += blockDim.x) {
    uint64_t v = 0;
    // bin 0 also takes the guard words below the histogram (binary32 bin -1)
    uint32_t *p = hist + (b == 0 ? -a.copies : b * a.copies);
    for (int c = 0; c < (b == 0 ? 2 : 1) * a.copies; ++c) {
      v += p[c];
      p[c] = 0u;
    }
    if (b < count && v != 0) {
      atomicAdd(reinterpret_cast<unsigned long long *>(out + b),
                static_cast<unsigned long long>(v));
      in_range += v;
    }
  }
  if (uni(F->oor_by_flush)) {
    // the out-of-range count is the pair count less every flushed count: one
    // subtraction per wave
    for (int o = 32; o > 0; o >>= 1) in_range += __shfl_xor(in_range, o);
    if ((threadIdx.x & 63) == 0 && in_range != 0)
      atomicAdd(reinterpret_cast<unsigned long long *>(F->oor + hist_idx),
                0ull - static_cast<unsigned long long>(in_range));
  }
}

// One j-tile of a spatially sorted frame for one wave. For every group of 64
// j-points of the tile and every slice r of the wave's i-points, the two
// groups' bounding boxes (fixed-point fractions) decide, axis by axis,
// whether one lattice shift n is the Eq. 5 wrap of all their pairs: the wrap
// of u_j - u_i is the n with u_j - u_i - n 2^32 in [-2^31, 2^31), i.e.
// floor((u_j - u_i + 2^31) / 2^32), in {-1, 0, 1}, and it is shared iff both
// ends of [jlo - ihi, jhi - ilo] give the same n. Lane 3r + k of the wave
// tests axis k of slice r, so one pass of a few instructions and four ballots
// classify all R slices. If every axis is shared, the pairs take the short
// path: the Cartesian difference to the i-point shifted by B n (a table
// entry), with no conversion and no cell matrix per pair (3 subtractions, q,
// root, bin). If exactly one axis K is ambiguous and its two ends differ by
// one, the pairs take the short path with the shift of K's lower end, or
// with one more cell vector B_K when the pair's fractional coordinate along
// K (row K of B^-1 applied to the difference) exceeds 1/2: a compare of the
// j-point's projection with a threshold of the slice and a select of the
// shifted i-point. Otherwise they take the fixed-point path of unsorted
// triclinic frames. The path and the arithmetic of a pair depend only on its
// two groups (species-aligned blocks of 64 points), not on the launch shape
// or on the other slices of the wave, so every launch shape, batch and server
// path gives the same counts.
template <int R, int MODE, bool DIAG, bool CLAMP, typename CountT>
__device__ __forceinline__ void sorted_tile(
    const float4 *__restrict__ tb, const uint32_t *__restrict__ boxes, int jt, int js,
    int jcount, int wbase, int lane, const FrameParams *F, const Geo32 &g,
    const float4 *__restrict__ X, int i0, int i1, const float (&cxi)[R], const float (&cyi)[R],
    const float (&czi)[R], uint32_t ib_lo, uint32_t ib_hi, uint32_t ib_empty, uint32_t hi,
    uint32_t hib, CountT &count_t) {
  const float ax = uni(F->cell32[0]), bx = uni(F->cell32[1]), by = uni(F->cell32[2]);
  const float cx = uni(F->cell32[3]), cy = uni(F->cell32[4]), cz = uni(F->cell32[5]);
  const float s32 = uni(F->s32);
  const float h11 = uni(F->hinv32[0]), h12 = uni(F->hinv32[1]), h13 = uni(F->hinv32[2]);
  const float h22 = uni(F->hinv32[3]), h23 = uni(F->hinv32[4]), h33 = uni(F->hinv32[5]);
  // the lattice shifts B n, read through the scalar cache with a uniform index
  using ConstF = const __attribute__((address_space(4))) float;
  const ConstF *gshift = (const ConstF *)(&F->gshift32[0][0]);
  constexpr uint32_t kAll = (1u << R) - 1u;
  // this lane's axis of the group boxes (lanes 3R and up repeat axis 0)
  const int bk = lane < 3 * R ? lane % 3 : 0;
  const uint32_t keep = ~ib_empty;
  for (int g0 = js & ~63; g0 < jcount; g0 += 64) {
    const int j_begin = max(js, g0), j_end = min(jcount, g0 + 64);
    const uint32_t *gb = boxes + (g0 >> 6) * 8;
    const uint32_t jl = gb[bk], jh = gb[3 + bk];
    // wrap of the lower and upper end of this lane's interval
    const int nl = static_cast<int>(jl - ib_hi >= 0x80000000u) - static_cast<int>(jl < ib_hi);
    const int nh = static_cast<int>(jh - ib_lo >= 0x80000000u) - static_cast<int>(jh < ib_lo);
    // bit 3r + k: axis k of slice r is ambiguous, spans more than two wraps,
    // has lower-end wrap +1, -1 (an empty slice counts nothing: shift 0)
    const uint32_t m_amb = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(nl != nh)) & keep;
    const uint32_t m_wide = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(nh - nl > 1)) & keep;
    const uint32_t m_pos = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(nl > 0)) & keep;
    const uint32_t m_neg = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(nl < 0)) & keep;
    // per slice: bit r of `fast` when all three shifts are shared, of `fix`
    // when exactly one axis is ambiguous by one wrap (`amb`: those axes, over
    // the slices); both get the i-point shifted by the wraps of the lower ends
    uint32_t fast = 0, fix = 0, amb = 0, ambr[R];
    float sx[R], sy[R], sz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t a_r = (m_amb >> (3 * r)) & 7u;
      ambr[r] = a_r;
      if ((a_r & (a_r - 1u)) == 0u && ((m_wide >> (3 * r)) & 7u) == 0u) {
        if (a_r == 0u)
          fast |= 1u << r;
        else
          fix |= 1u << r;
        amb |= a_r;
        const uint32_t q = ((m_pos >> (3 * r)) & 7u) | (((m_neg >> (3 * r)) & 7u) << 3);
        const ConstF *S = gshift + 4 * q;
        sx[r] = cxi[r] + S[0];
        sy[r] = cyi[r] + S[1];
        sz[r] = czi[r] + S[2];
      } else {
        sx[r] = sy[r] = sz[r] = 0.f;
      }
    }
    // Clamp bounds of a pair (see count_t): l = 0 and lb = the guard word
    // below bin 0 for a pair that counts, the lane's discard slot for the
    // lower triangle of a diagonal item. The short paths need nothing else:
    // a lane past the end of the item holds an i-point at infinity, whose q
    // is +inf, which the upper clamp discards. The fixed-point path passes
    // the lane's own bounds (l0, lb0).
    auto mask = [&](int r, int j, uint32_t &l, uint32_t &lb, uint32_t l0 = 0u,
                    uint32_t lb0 = kMagicBits - 1u) {
      l = l0;
      lb = lb0;
      if constexpr (DIAG) {
        const bool up = jt + j > wbase + r * 64 + lane;
        l = up ? l : hi;
        lb = up ? lb : hib;
      }
    };
    auto bin = [&](int r, int j, float dx, float dy, float dz) {
      uint32_t l, lb;
      mask(r, j, l, lb);
      const float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      count_t(__float_as_uint(fmaf(__builtin_amdgcn_sqrtf(q), s32, kMagic32)), l, lb);
    };
    auto fast_pair = [&](int r, const float4 &C, int j) {
      bin(r, j, C.x - sx[r], C.y - sy[r], C.z - sz[r]);
    };
    // row K of B^-1 applied to a point: its fractional coordinate along K
    // (up to the constant of the cell centre)
    auto proj = [&](auto axis_c, float x, float y, float z) {
      constexpr int K = decltype(axis_c)::value;
      if constexpr (K == 0)
        return fmaf(z, h13, fmaf(y, h12, x * h11));
      else if constexpr (K == 1)
        return fmaf(z, h23, y * h22);
      else
        return z * h33;
    };
    // One-axis wrap of slice r along K: the threshold the j-point's
    // projection must exceed (1/2 above the shifted i-point's; +inf for a
    // slice whose shift K is shared, which then takes exactly the short
    // path) and the i-point shifted by one more cell vector B_K.
    struct Wrap {
      float th, x, y, z;
    };
    auto wrap_of = [&](auto axis_c, int r) {
      constexpr int K = decltype(axis_c)::value;
      Wrap w;
      w.th = (fix >> r) & 1u ? proj(axis_c, sx[r], sy[r], sz[r]) + 0.5f : __builtin_inff();
      w.x = sx[r] + (K == 0 ? ax : K == 1 ? bx : cx);
      w.y = K == 0 ? sy[r] : sy[r] + (K == 1 ? by : cy);
      w.z = K == 2 ? sz[r] + cz : sz[r];
      return w;
    };
    auto fix_pair = [&](auto axis_c, int r, const Wrap &w, const float4 &C, float p, int j) {
      constexpr int K = decltype(axis_c)::value;
      const bool up = p > w.th;
      const float ux = up ? w.x : sx[r];
      const float uy = K >= 1 && up ? w.y : sy[r];
      const float uz = K == 2 && up ? w.z : sz[r];
      bin(r, j, C.x - ux, C.y - uy, C.z - uz);
    };
    // The fixed-point path (rare) reloads its i-words: -(b:a) of the
    // i-point of slice r, -(c':c) of slices 2k and 2k+1 (one 64-bit addition
    // to j's (c:c) gives both c differences, the second lowered by one unit
    // when the first borrows), and the lane's clamp bounds.
    struct SlowI {
      uint64_t nab, nzz;
      uint32_t l0, lb0;
    };
    auto slow_i = [&](int r) {
      const int i = wbase + r * 64 + lane, ip = wbase + (r ^ 1) * 64 + lane;
      const float4 P = X[2 * (i < i1 ? i : i0)];
      const float4 Q = X[2 * (ip < i1 ? ip : i0)];
      const float z0 = r % 2 == 0 ? P.z : Q.z, z1 = r % 2 == 0 ? Q.z : P.z;
      SlowI v;
      v.nab = 0ull - ((static_cast<uint64_t>(__float_as_uint(P.y)) << 32) | __float_as_uint(P.x));
      v.nzz = 0ull - ((static_cast<uint64_t>(__float_as_uint(z1)) << 32) | __float_as_uint(z0));
      v.l0 = i < i1 ? 0u : hi;
      v.lb0 = i < i1 ? kMagicBits - 1u : hib;
      return v;
    };
    auto slow_pair = [&](int r, const SlowI &v, uint64_t ab, uint64_t cc, int j) {
      uint32_t l, lb;
      mask(r, j, l, lb, v.l0, v.lb0);
      const uint64_t dcc = cc + v.nzz;
      const float fcd = static_cast<float>(
          static_cast<int32_t>(static_cast<uint32_t>(r % 2 == 0 ? dcc : dcc >> 32)));
      count_t(bits32_packed_c<kBoxTric>(ab, v.nab, fcd, g), l, lb);
    };
    // Every loop reads the next j before the current j's atomics: LDS
    // operations complete in order, so a read issued after the atomics would
    // wait for all of them. At the end of the tile the look-ahead read
    // touches the entry just past it (the next tile or the box area), never
    // used. The entry pointer lives in a VGPR so both reads use immediate
    // offsets (the zero is opaque to the compiler on purpose).
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    auto run_j = [&](auto &&body, int part) {
      // part 1: the Cartesian float4 of each j; part 0: its fixed-point words
      const float4 *cp = tb + 2 * j_begin + part + vzero;
      float4 pa = cp[0];
      int j = j_begin;
      for (; j + 1 < j_end; j += 2, cp += 4) {
        const float4 pb = cp[2];
        __builtin_amdgcn_sched_barrier(0);
        body(pa, j);
        pa = cp[4];
        __builtin_amdgcn_sched_barrier(0);
        body(pb, j + 1);
      }
      if (j < j_end) body(pa, j);
    };
    auto words = [](const float4 &e, uint64_t &ab, uint64_t &cc) {
      ab = (static_cast<uint64_t>(__float_as_uint(e.y)) << 32) | __float_as_uint(e.x);
      cc = (static_cast<uint64_t>(__float_as_uint(e.w)) << 32) | __float_as_uint(e.z);
    };
    auto fix_all = [&](auto axis_c) {
      Wrap w[R];
#pragma unroll
      for (int r = 0; r < R; ++r) w[r] = wrap_of(axis_c, r);
      run_j([&](const float4 &C, int j) {
        const float p = proj(axis_c, C.x, C.y, C.z);
#pragma unroll
        for (int r = 0; r < R; ++r) fix_pair(axis_c, r, w[r], C, p, j);
      }, 1);
    };
    auto fix_one = [&](auto axis_c, int r) {
      const Wrap w = wrap_of(axis_c, r);
      run_j([&](const float4 &C, int j) {
        fix_pair(axis_c, r, w, C, proj(axis_c, C.x, C.y, C.z), j);
      }, 1);
    };
    if (fast == kAll) {
      run_j([&](const float4 &C, int j) {
#pragma unroll
        for (int r = 0; r < R; ++r) fast_pair(r, C, j);
      }, 1);
    } else if ((fast | fix) == kAll && amb == 1u) {
      fix_all(std::integral_constant<int, 0>{});
    } else if ((fast | fix) == kAll && amb == 2u) {
      fix_all(std::integral_constant<int, 1>{});
    } else if ((fast | fix) == kAll && amb == 4u) {
      fix_all(std::integral_constant<int, 2>{});
    } else if ((fast | fix) == 0) {
      SlowI v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = slow_i(r);
      run_j([&](const float4 &A, int j) {
        uint64_t ab, cc;
        words(A, ab, cc);
#pragma unroll
        for (int r = 0; r < R; ++r) slow_pair(r, v[r], ab, cc, j);
      }, 0);
    } else {
      // slices of different kinds: one pass per slice, each slice the path
      // its own ambiguity gives it (so the counts do not depend on which
      // slices share a wave)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (fast & (1u << r)) {
          run_j([&](const float4 &C, int j) { fast_pair(r, C, j); }, 1);
        } else if (fix & (1u << r)) {
          if (ambr[r] == 1u)
            fix_one(std::integral_constant<int, 0>{}, r);
          else if (ambr[r] == 2u)
            fix_one(std::integral_constant<int, 1>{}, r);
          else
            fix_one(std::integral_constant<int, 2>{}, r);
        } else {
          const SlowI v = slow_i(r);
          run_j([&](const float4 &A, int j) {
            uint64_t ab, cc;
            words(A, ab, cc);
            slow_pair(r, v, ab, cc, j);
          }, 0);
        }
      }
    }
  }
}

// Lattice shift along one axis shared by every pair of two groups of a
// binary64 sorted frame. The fractional difference s of a pair (the first
// step of Eq. 5, with its rounding) lies in [jlo - ihi, jhi - ilo] (the
// groups' boxes of B^-1 x) widened by the margin m, which bounds the
// rounding of s, of the boxes and of this test. When both ends of the
// widened interval round to the same n, every s lies strictly inside
// (n - 1/2, n + 1/2), so rint(s) = n for every pair, ties included. False
// when the ends differ or a group is empty (an empty box has lo = +inf,
// hi = -inf) or holds a non-finite value.
__device__ __forceinline__ bool group_shift64(double ilo, double ihi, double jlo, double jhi,
                                              double m, double &n) {
  const double a = floor(((jlo - ihi) - m) + 0.5);
  const double b = floor(((jhi - ilo) + m) + 0.5);
  n = a;
  return a == b;
}

// One j-tile of a spatially sorted binary64 frame for one wave. For every
// group of 64 j-points and every slice r of the wave's i-points, each axis
// whose Eq. 5 shift n is shared by all their pairs (group_shift64) and whose
// terms B n are exact (|n| <= 1) skips that axis's fractional
// coordinate and rounding: each fused step of Eq. 5 with that n, d - B_k n
// rounded once, equals the plain sum d + P_k with the exact term
// P_k = -B_k n. The other axes take Eq. 5's own steps. A pass over the
// group's j serves all R slices with one kind of reduction (the axes that
// need the rounding for any slice take it for all of them: for a shared
// axis it yields the same n), so every reduced vector, q and t is
// bit-identical to the canonical sequence. Sums along an axis whose shared
// shift is zero for every slice are skipped (they would change only the sign
// of a zero component).
//
// Box slot 6 of a group holds the largest |x| + |y| + |z| of its points,
// which bounds the magnitudes, and with them the rounding, that the margin
// of group_shift64 must cover: with u = 2^-53 and h the largest entry of
// B^-1, every rounding error of the fractional difference, of the boxes and
// of the test is below 12 u h (A_i + A_j), well inside 2^-48 h (A_i + A_j).
template <int R, bool DIAG, typename CountT>
__device__ __forceinline__ void sorted_tile64(
    const double4 *__restrict__ tb, const double *__restrict__ boxes, int jt, int js,
    int jcount, int wbase, int lane, const Geo64 &g, bool big_bins, const double (&xi)[R],
    const double (&yi)[R], const double (&zi)[R], double ib_lo, double ib_hi, double ib_mag,
    uint32_t ib_empty, const uint32_t (&lo)[R], uint32_t hi, CountT &count_t) {
  const double hmax = fmax(fmax(fabs(g.h11), fabs(g.h12)),
                           fmax(fmax(fabs(g.h13), fabs(g.h22)), fmax(fabs(g.h23), fabs(g.h33))));
  // lane 3r + k tests axis k of slice r (lanes 3R and up repeat axis 0)
  const int bk = lane < 3 * R ? lane % 3 : 0;
  const uint32_t keep = ~ib_empty;
  for (int g0 = js & ~63; g0 < jcount; g0 += 64) {
    const int j_begin = max(js, g0), j_end = min(jcount, g0 + 64);
    const double *gb = boxes + (g0 >> 6) * 8;
    // this lane's axis: is the shift shared by all pairs of the two groups,
    // and is its term -B_k n exact (|n| <= 1)? Four ballots give, per slice
    // and axis, the rounded axes and the shared shifts +1 and -1 (an empty
    // slice counts nothing: shift 0).
    const double m = fma(hmax * (ib_mag + gb[6]), 0x1p-48, 0x1p-40);
    double n;
    const bool shared = group_shift64(ib_lo, ib_hi, gb[bk], gb[3 + bk], m, n);
    const bool use = shared && fabs(n) <= 1.0;
    const uint32_t m_amb = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(!use)) & keep;
    const uint32_t m_pos =
        static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(use && n == 1.0)) & keep;
    const uint32_t m_neg =
        static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(use && n == -1.0)) & keep;
    // amb: bit k when axis k (a, b, c) needs the rounding for some slice;
    // nz: bit k when some slice has a shared non-zero shift along axis k
    uint32_t amb = 0, nz = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      amb |= (m_amb >> (3 * r)) & 7u;
      nz |= ((m_pos | m_neg) >> (3 * r)) & 7u;
    }
    nz &= ~amb;
    // exact term -B n of slice r along axis k for cell entry b, in the order
    // of the canonical steps (zero where the slice's shift is 0 or the axis
    // takes the rounding); selected from the ballots, so each loop below
    // keeps only the terms it adds
    auto P = [&](int r, int k, double b) {
      const uint32_t bit = 1u << (3 * r + k);
      return (m_pos & bit) ? -b : ((m_neg & bit) ? b : 0.0);
    };

    // The reduced vector, q and short root t of the pairs of all slices with
    // one j, reduced as AMB says (each lane keeps in `gap` how close its t
    // come to an integer, see t_fast64).
    // AMB: the axes that take the rounding; NZ: the axes whose shared shift
    // is non-zero for some slice (the others add nothing: their terms are 0).
    auto reduce = [&](auto amb_c, auto nz_c, const double4 &pj, double *q, double *t,
                      uint32_t &gap) {
      constexpr uint32_t AMB = decltype(amb_c)::value;
      constexpr uint32_t NZ = decltype(nz_c)::value;
      static_assert((AMB & NZ) == 0, "an axis is either rounded or shared");
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double dx = pj.x - xi[r], dy = pj.y - yi[r], dz = pj.z - zi[r];
        // Eq. 5's n of the axes that need it, from the unreduced d
        double na = 0.0, nb = 0.0, nc = 0.0;
        if constexpr (AMB & 1u) na = rint(fma(dz, g.h13, fma(dy, g.h12, dx * g.h11)));
        if constexpr (AMB & 2u) nb = rint(fma(dz, g.h23, dy * g.h22));
        if constexpr (AMB & 4u) nc = rint(dz * g.h33);
        if constexpr (AMB & 4u) dz = fma(-g.cz, nc, dz);
        else if constexpr (NZ & 4u) dz = dz + P(r, 2, g.cz);
        if constexpr (AMB & 2u) dy = fma(-g.by, nb, dy);
        else if constexpr (NZ & 2u) dy = dy + P(r, 1, g.by);
        if constexpr (AMB & 4u) dy = fma(-g.cy, nc, dy);
        else if constexpr (NZ & 4u) dy = dy + P(r, 2, g.cy);
        if constexpr (AMB & 1u) dx = fma(-g.ax, na, dx);
        else if constexpr (NZ & 1u) dx = dx + P(r, 0, g.ax);
        if constexpr (AMB & 2u) dx = fma(-g.bx, nb, dx);
        else if constexpr (NZ & 2u) dx = dx + P(r, 1, g.bx);
        if constexpr (AMB & 4u) dx = fma(-g.cx, nc, dx);
        else if constexpr (NZ & 4u) dx = dx + P(r, 2, g.cx);
        q[r] = fma(dz, dz, fma(dy, dy, dx * dx));
        t[r] = t_fast64(q[r], g.s, gap);
      }
    };
    // The counts of NJ consecutive j from j0: the correctly rounded root for
    // all of them when any lane needs it, then one atomic per pair.
    auto finish = [&](auto nj_c, const double *q, double *t, uint32_t gap, int j0) {
      constexpr int NJ = decltype(nj_c)::value;
      if (__builtin_expect(any_near(gap), 0))
#pragma unroll
        for (int k = 0; k < NJ * R; ++k) t[k] = sqrt_cr(q[k]) * g.s;
#pragma unroll
      for (int k = 0; k < NJ * R; ++k) {
        const int r = k % R;
        uint32_t l = lo[r];
        if constexpr (DIAG) l = jt + j0 + k / R > wbase + r * 64 + lane ? l : hi;
        count_t(t[k], l, 0u);
      }
    };
    // One pass over the group's j, two j per step with one ballot. The next
    // two j are read before the current ones' atomics (see sorted_tile); at
    // the end of the group the look-ahead reads touch at most the two entries
    // after it (the next group, the other tile or the box area), never used.
    auto run_j = [&](auto amb_c, auto nz_c) {
      using Two = std::integral_constant<int, 2>;
      using One = std::integral_constant<int, 1>;
      int vzero;
      asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
      const double4 *cp = tb + j_begin + vzero;
      double4 pa = cp[0], pb = cp[1];
      int j = j_begin;
      for (; j + 1 < j_end; j += 2, cp += 2) {
        double q[2 * R], t[2 * R];
        uint32_t gap = gap_init(big_bins);
        reduce(amb_c, nz_c, pa, q, t, gap);
        reduce(amb_c, nz_c, pb, q + R, t + R, gap);
        pa = cp[2];
        pb = cp[3];
        finish(Two{}, q, t, gap, j);
      }
      if (j < j_end) {
        double q[R], t[R];
        uint32_t gap = gap_init(big_bins);
        reduce(amb_c, nz_c, pa, q, t, gap);
        finish(One{}, q, t, gap, j);
      }
    };
    using M0 = std::integral_constant<uint32_t, 0>;
    using M1 = std::integral_constant<uint32_t, 1>;
    using M2 = std::integral_constant<uint32_t, 2>;
    using M3 = std::integral_constant<uint32_t, 3>;
    using M4 = std::integral_constant<uint32_t, 4>;
    using M5 = std::integral_constant<uint32_t, 5>;
    using M6 = std::integral_constant<uint32_t, 6>;
    using M7 = std::integral_constant<uint32_t, 7>;
    if constexpr (DIAG) {
      // items on the diagonal of a histogram (few pairs): Eq. 5 throughout
      run_j(M7{}, M0{});
    } else {
      // the frequent kinds get their own loop (shared shifts along one axis
      // at most, or one rounded axis with zero shifts along the others);
      // the rest round their ambiguous axes and add the terms of all others
      switch (amb * 8u + nz) {
        case 0: run_j(M0{}, M0{}); break;
        case 1: run_j(M0{}, M1{}); break;
        case 2: run_j(M0{}, M2{}); break;
        case 4: run_j(M0{}, M4{}); break;
        case 8: run_j(M1{}, M0{}); break;
        case 16: run_j(M2{}, M0{}); break;
        case 32: run_j(M4{}, M0{}); break;
        default:
          switch (amb) {
            case 0: run_j(M0{}, M7{}); break;
            case 1: run_j(M1{}, M6{}); break;
            case 2: run_j(M2{}, M5{}); break;
            case 3: run_j(M3{}, M4{}); break;
            case 4: run_j(M4{}, M3{}); break;
            case 5: run_j(M5{}, M2{}); break;
            case 6: run_j(M6{}, M1{}); break;
            default: run_j(M7{}, M0{}); break;
          }
      }
    }
  }
}

// CLAMP = false: the host proved that every t of this frame is below the LDS
// stride and the block has no invalid lanes, so the bin index needs no clamp
// (out-of-range pairs land in slots [n_bins, stride) that are never flushed).
//
// BOX = kBoxTricSearch: the 27-image search only runs for pairs whose reduced
// vector is not provably the nearest image (q0 >= qskip: at least half the
// shortest lattice vector long). Those pairs are queued per wave in LDS and
// searched 64 at a time by the whole wave, so the search never runs for a
// wave with only a few lanes needing it; the others are counted directly.
template <typename T, int R, int BOX, int MODE, bool DIAG, bool CLAMP>
__device__ __forceinline__ void run_item(const PairKernelArgs &a, const WorkItem &w,
                                         const FrameParams *F,
                                         typename V4<T>::type *__restrict__ tile,
                                         uint32_t *__restrict__ my,
                                         typename V4<T>::type *__restrict__ queue,
                                         typename V4<T>::type *__restrict__ sh) {
  using V = typename V4<T>::type;
  using G = typename Geo<T>::type;
  constexpr bool SWEEP = MODE == kModeSweep;
  constexpr bool GLOBAL = MODE == kModeGlobal;
  constexpr bool SEARCH = BOX == kBoxTricSearch;
  // spatially sorted frames: two float4 per point (fixed-point words, then
  // the Cartesian position relative to the cell centre)
  constexpr bool SORTED = BOX == kBoxTricSorted;
  constexpr int EPJ = SORTED && sizeof(T) == 4 ? 2 : 1;
  const V *__restrict__ X = static_cast<const V *>(F->coords);
  const G g = Geo<T>::load(F);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tj = a.tj;
  const int win = uni(F->win);
  const int b_lo = w.sweep * win;
  const int log_copies = a.copies == 4 ? 2 : (a.copies == 2 ? 1 : 0);
  const uint32_t shift_bytes = static_cast<uint32_t>(log_copies + 2);
  char *const my_bytes = reinterpret_cast<char *>(my);
  // binary32 counts address LDS as 32-bit integers: this lane's copy of bin 0,
  // less the offset of the index that is shifted in (the wrap-around is
  // intended): the bin bits for one LDS histogram; for bin windows the slot
  // of the window, where window 0 starts at bin -1 (slot 0 is the guard word)
  using LdsU32 = __attribute__((address_space(3))) uint32_t;
  const uint32_t my_lds =
      static_cast<uint32_t>(reinterpret_cast<uintptr_t>((LdsU32 *)my));
  const uint32_t s0 = w.sweep == 0 ? 1u : 0u;
  uint32_t my_lds_m = SWEEP ? my_lds - (s0 << shift_bytes) : my_lds - (kMagicBits << shift_bytes);
  // opaque, so the compiler keeps (index << shift) + my_lds_m as one
  // v_lshl_add_u32 instead of subtracting the offset from every bin
  asm volatile("" : "+v"(my_lds_m));
  // bin bits of slot 0 of this window
  const uint32_t sweep_base = kMagicBits + static_cast<uint32_t>(b_lo) - s0;
  // largest slot index of binary64 unclamped items
  const double cap64 = static_cast<double>(a.stride - 1);

  // i-particles: wave w holds [wbase, wbase + 64R), lane l the R values
  // wbase + r*64 + l
  const int wbase = w.i0 + wave * 64 * R;
  const bool wave_active = wbase < w.i1;
  T xi[R], yi[R], zi[R];
  const uint32_t hi = static_cast<uint32_t>(win + lane);  // discard slot of this lane
  uint32_t lo[R];
  // sorted frames: Cartesian i-positions, and the fixed-point bounding box of
  // each 64-particle slice r of the wave (its valid lanes), one axis per
  // lane: lane 3r + k holds the lower (ib_lo) and upper (ib_hi) bound along
  // axis k; ib_empty has bits 3r, 3r + 1, 3r + 2 set for a slice without
  // valid lanes
  [[maybe_unused]] float cxi[R], cyi[R], czi[R];
  [[maybe_unused]] uint32_t ib_lo = 0, ib_hi = 0, ib_empty = 0;
  // binary64 sorted frames: boxes of the fractional coordinates B^-1 x, one
  // axis per lane (lane 3r + k: axis k of slice r), the largest
  // |x| + |y| + |z| of slice r in lanes 3r to 3r + 2, and ib64_empty with
  // bits 3r to 3r + 2 set for a slice without valid lanes
  [[maybe_unused]] double ib64_lo = 0.0, ib64_hi = 0.0, ib64_mag = 0.0;
  [[maybe_unused]] uint32_t ib64_empty = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = wbase + r * 64 + lane;
    const bool ok = i < w.i1;
    const V p = X[EPJ * (ok ? i : w.i0)];
    xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
    lo[r] = ok ? 0u : hi;
    if constexpr (SORTED && sizeof(T) == 8) {
      double sg[3];
      frac64(p.x, p.y, p.z, g, sg);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const double bl = wave_min_f64(ok ? sg[ax] : __builtin_inf());
        const double bh = wave_max_f64(ok ? sg[ax] : -__builtin_inf());
        if (lane == 3 * r + ax) {
          ib64_lo = bl;
          ib64_hi = bh;
        }
        if (ax == 0 && !(bl <= bh)) ib64_empty |= 7u << (3 * r);
      }
      const double mag = wave_max_f64(ok ? fabs(p.x) + fabs(p.y) + fabs(p.z) : 0.0);
      if (lane >= 3 * r && lane < 3 * r + 3) ib64_mag = mag;
    }
    if constexpr (SORTED && sizeof(T) == 4) {
      // a lane past the end of the item: an i-point at infinity (every q of
      // its short-path pairs is +inf and lands in its discard slot)
      const V c = X[EPJ * (ok ? i : w.i0) + 1];
      cxi[r] = ok ? c.x : __builtin_inff();
      cyi[r] = ok ? c.y : __builtin_inff();
      czi[r] = ok ? c.z : __builtin_inff();
      const uint32_t u[3] = {__float_as_uint(p.x), __float_as_uint(p.y), __float_as_uint(p.z)};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const uint32_t bl = wave_min_u32(ok ? u[ax] : 0xFFFFFFFFu);
        const uint32_t bh = wave_max_u32(ok ? u[ax] : 0u);
        if (lane == 3 * r + ax) {
          ib_lo = bl;
          ib_hi = bh;
        }
        if (ax == 0 && bl > bh) ib_empty |= 7u << (3 * r);
      }
    }
  }
  // binary32 clamp bounds in bin bits: the guard word below bin 0 for a
  // lane that counts, its discard slot for one that must not
  const uint32_t hib = kMagicBits + hi;
  uint32_t lob[R];
#pragma unroll
  for (int r = 0; r < R; ++r) lob[r] = lo[r] == 0u ? kMagicBits - 1u : hib;
  // -(b:a) of each i-particle for the packed periodic binary32 difference
  uint64_t nab[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (sizeof(T) == 4)
      nab[r] = 0ull - ((static_cast<uint64_t>(__float_as_uint(yi[r])) << 32) |
                       __float_as_uint(xi[r]));
    else
      nab[r] = 0ull;
  }
  // -(c' : c) of i-particles 2k and 2k+1: one 64-bit addition to j's (c : c)
  // gives both c differences, the second lowered by one unit when the first
  // borrows (as for b above)
  static_assert(R % 2 == 0, "i-particles are paired for the c difference");
  uint64_t nzz[R / 2];
#pragma unroll
  for (int k = 0; k < R / 2; ++k) {
    if constexpr (sizeof(T) == 4)
      nzz[k] = 0ull - ((static_cast<uint64_t>(__float_as_uint(zi[2 * k + 1])) << 32) |
                       __float_as_uint(zi[2 * k]));
    else
      nzz[k] = 0ull;
  }
  const int n_bins = uni(F->n_bins);
  // binary64: the correctly rounded root for every pair when t at or above
  // 2^20 can lie near a bin edge (this many bins) or the scale s is so large
  // that a subnormal q could reach bin 1 (see t_fast64)
  [[maybe_unused]] const bool big_bins =
      n_bins >= (1 << 20) - 2 || !(uni(F->s) < 0x1p500);
  // the output is global memory: say so, so the atomics are global_atomic_*
  // (a generic pointer would give flat atomics, which also count as LDS
  // operations in lgkmcnt)
  using GlobalU64 = __attribute__((address_space(1))) unsigned long long;
  GlobalU64 *const gout =
      (GlobalU64 *)(F->out + static_cast<size_t>(w.hist) * static_cast<size_t>(n_bins));

  // Counts one pair: binary64 at scaled distance v = t, binary32 from its bin
  // bits v (bin_bits32). l: 0 for a pair that counts, the lane's discard slot
  // for one that must not (the lower clamp); lb: the same bound in bin bits
  // for the binary32 LDS clamp (guard word or discard slot), passed by the
  // caller so that a diagonal item selects it directly.
  auto count_t = [&](auto v, uint32_t l, uint32_t lb) {
    if constexpr (sizeof(T) == 4) {
      const uint32_t b = v;
      if constexpr (GLOBAL) {
        const uint32_t k = max(b, kMagicBits) - kMagicBits;
        if (l == 0u && k < static_cast<uint32_t>(n_bins))
          __hip_atomic_fetch_add(gout + k, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t m;  // bin + kMagicBits
        if constexpr (!CLAMP) {
          // fixed-point staging bounds every t below the stride; bin -1 is
          // the guard word below the histogram, added to bin 0 on flush
          m = b;
        } else if constexpr (!SWEEP) {
          m = med3_u32(b, lb, kMagicBits + hi);
        } else {
          // slot in the window; bins below it wrap to large values and are
          // discarded with those above (window 0 has no bins below it: bin -1
          // is its slot 0, the guard word)
          const uint32_t hs = hi + s0;
          m = med3_u32(b - sweep_base, l == 0u ? 0u : hs, hs);
        }
        __hip_atomic_fetch_add((LdsU32 *)(uintptr_t)(my_lds_m + (m << shift_bytes)), 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
      const T t = v;
      if constexpr (GLOBAL) {
        // a pair counts iff t < n_bins (in the working precision)
        if (l == 0u && t < static_cast<T>(n_bins))
          __hip_atomic_fetch_add(gout + static_cast<uint32_t>(t), 1ull, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t idx;
        if constexpr (!CLAMP) {
          // binary64 reads raw device coordinates: cap t so that even
          // non-finite or absurd input stays inside the LDS histogram
          idx = static_cast<uint32_t>(min_arith(t, cap64));
        } else {
          // floor(t), saturated; t >= 0 always
          idx = static_cast<uint32_t>(min_arith(t, 4294967295.0));
          if constexpr (SWEEP) idx -= static_cast<uint32_t>(b_lo);
          // the slot clamped to [l, hi] (l is 0 or hi): one v_med3_u32
          idx = med3_u32(idx, l, hi);
        }
        // byte offset with one shift (copies interleaved bin-major), so the
        // address is a single v_lshl_add_u32
        atomicAdd(reinterpret_cast<uint32_t *>(my_bytes + (idx << shift_bytes)), 1u);
      }
    }
  };

  // image-search ring of this wave: qn entries from head (wave-uniform)
  constexpr int cap = queue_cap(R);
  V *const wq = queue + wave * cap;
  int head = 0, qn = 0;
  [[maybe_unused]] uint64_t n_searched = 0;  // pairs this wave searched in this item
  [[maybe_unused]] uint64_t n_images = 0;    // images it evaluated for them
  [[maybe_unused]] T qskip;
  if constexpr (sizeof(T) == 4)
    qskip = uni(F->qskip32);
  else
    qskip = uni(F->qskip64);
  if constexpr (SEARCH) {
    // this frame's shift table; read after the first tile barrier below
    // the search table: the 8 octant rows, then all 27 shift vectors
    for (int k = tid; k < kSearchTable; k += blockDim.x) {
      const int m = k < 8 * kOctCap ? F->oct_shift[k / kOctCap][k % kOctCap] : k - 8 * kOctCap;
      V S;
      if constexpr (sizeof(T) == 4) {
        S.x = F->shift32[m][0]; S.y = F->shift32[m][1]; S.z = F->shift32[m][2];
      } else {
        S.x = F->shift64[m][0]; S.y = F->shift64[m][1]; S.z = F->shift64[m][2];
      }
      S.w = T(0);
      sh[k] = S;
    }
  }
  [[maybe_unused]] uint32_t oct_full = 0;
  [[maybe_unused]] int oct_n = 0;
  if constexpr (SEARCH) {
    oct_full = static_cast<uint32_t>(uni(static_cast<int>(F->oct_full)));
    oct_n = uni(static_cast<int>(F->oct_n));
  }
  // searches and counts the `cnt` (<= 64) oldest queued vectors
  auto drain = [&](int cnt) {
    if constexpr (SEARCH) {
      __builtin_amdgcn_wave_barrier();
      const bool v = lane < cnt;
      int idx = head + (v ? lane : 0);
      if (idx >= cap) idx -= cap;
      const V e = wq[idx];
      T q = fmaT(e.z, e.z, fmaT(e.y, e.y, e.x * e.x));
      // the vector's octant (8: outside the octant boxes), 8 as well when its
      // list is the full one; the wave runs the full list when any of its
      // vectors needs it
      int code;
      if constexpr (sizeof(T) == 4)
        code = __float_as_int(e.w);
      else
        code = octant64(e.x, e.y, e.z, g);
      if ((oct_full >> code) & 1u) code = 8;
      const int n = __builtin_amdgcn_ballot_w64(code == 8) != 0 ? kShifts : oct_n;
      q = search_oct<T>(e.x, e.y, e.z, q, code == 8 ? 8 * kOctCap : code * kOctCap, n, sh);
      n_images += static_cast<uint64_t>(cnt) * static_cast<uint64_t>(n);
      if constexpr (sizeof(T) == 4)
        count_t(bin_bits32(__builtin_amdgcn_sqrtf(q)), v ? 0u : hi, v ? kMagicBits - 1u : hib);
      else
        count_t(t_guarded64(q, g.s, big_bins), v ? 0u : hi, 0u);
      n_searched += cnt;  // wave-uniform; added to the frame's count once per item
      head += cnt;
      if (head >= cap) head -= cap;
      qn -= cnt;
      __builtin_amdgcn_wave_barrier();
    }
  };

  // The i-particles are complete before the tile loop, so the only global
  // load in flight inside it is the next tile's prefetch, which the j-loop
  // never reads.
  __builtin_amdgcn_s_waitcnt(kWaitVm0);

  V pre = {};
  [[maybe_unused]] V preC = {};
  // sorted frames: bounding boxes of the tiles' groups of 64 j-points, after
  // the two tiles (eight words per group)
  [[maybe_unused]] uint32_t *const tboxes = reinterpret_cast<uint32_t *>(tile + 2 * tj * EPJ);
  if (tid < tj && w.j0 + tid < w.j1) {
    pre = X[EPJ * (w.j0 + tid)];
    if constexpr (SORTED && sizeof(T) == 4) preC = X[EPJ * (w.j0 + tid) + 1];
  }
  int buf = 0;
  for (int jt = w.j0; jt < w.j1; jt += tj, buf ^= 1) {
    if (tid < tj) {
      tile[(buf * tj + tid) * EPJ] = pre;
      if constexpr (SORTED && sizeof(T) == 8) {
        // the box of this wave's 64 j in fractional coordinates
        const bool ok = jt + tid < w.j1;
        double sg[3];
        frac64(pre.x, pre.y, pre.z, g, sg);
        double b6[7];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          b6[ax] = wave_min_f64(ok ? sg[ax] : __builtin_inf());
          b6[3 + ax] = wave_max_f64(ok ? sg[ax] : -__builtin_inf());
        }
        b6[6] = wave_max_f64(ok ? fabs(pre.x) + fabs(pre.y) + fabs(pre.z) : 0.0);
        if (lane < 7) {
          double v = b6[0];
#pragma unroll
          for (int q = 1; q < 7; ++q) v = lane == q ? b6[q] : v;
          reinterpret_cast<double *>(tboxes)[(buf * 4 + (tid >> 6)) * 8 + lane] = v;
        }
      }
      if constexpr (SORTED && sizeof(T) == 4) {
        tile[(buf * tj + tid) * EPJ + 1] = preC;
        // the box of this wave's 64 j (tiles start on group boundaries of
        // the species, so the group is the same whatever the launch shape)
        const bool ok = jt + tid < w.j1;
        const uint32_t u[3] = {__float_as_uint(pre.x), __float_as_uint(pre.y),
                               __float_as_uint(pre.z)};
        uint32_t b6[6];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          b6[ax] = wave_min_u32(ok ? u[ax] : 0xFFFFFFFFu);
          b6[3 + ax] = wave_max_u32(ok ? u[ax] : 0u);
        }
        if (lane < 6) {
          uint32_t v = b6[0];
#pragma unroll
          for (int q = 1; q < 6; ++q) v = lane == q ? b6[q] : v;
          tboxes[(buf * 4 + (tid >> 6)) * 8 + lane] = v;
        }
      }
    }
    __syncthreads();
    {
      const int jn = jt + tj + tid;
      if (tid < tj && jn < w.j1) {
        pre = X[EPJ * jn];
        if constexpr (SORTED && sizeof(T) == 4) preC = X[EPJ * jn + 1];
      }
    }
    const int jcount = min(tj, w.j1 - jt);
    int js = 0;
    if constexpr (DIAG) js = max(0, min(jcount, wbase + 1 - jt));
    if constexpr (SORTED && sizeof(T) == 4) {
      if (wave_active && js < jcount)
        sorted_tile<R, MODE, DIAG, CLAMP>(tile + buf * tj * EPJ, tboxes + buf * 32, jt, js,
                                          jcount, wbase, lane, F, g, X, w.i0, w.i1, cxi, cyi,
                                          czi, ib_lo, ib_hi, ib_empty, hi, hib, count_t);
      continue;
    }
    if constexpr (SORTED && sizeof(T) == 8) {
      if (wave_active && js < jcount)
        sorted_tile64<R, DIAG>(tile + buf * tj, reinterpret_cast<const double *>(tboxes) + buf * 32,
                               jt, js, jcount, wbase, lane, g, big_bins, xi, yi, zi, ib64_lo,
                               ib64_hi, ib64_mag, ib64_empty, lo,
                               hi, count_t);
      continue;
    }
    if (wave_active && js < jcount) {
      const V *__restrict__ tb = tile + buf * tj;
      // periodic binary32: j as its packed (b:a) and (c:c) words, one
      // 16-byte read (see t32_packed and the staging)
      constexpr bool kPacked = sizeof(T) == 4 && BOX != kBoxNone;
      struct JPacked {
        uint64_t ab;
        uint64_t cc;
      };
      using J = typename std::conditional<kPacked, JPacked, V>::type;
      const uint64_t *__restrict__ tb64 = reinterpret_cast<const uint64_t *>(tb);
      auto load_j = [&](int k) -> J {
        if constexpr (kPacked)
          return JPacked{tb64[2 * k], tb64[2 * k + 1]};
        else
          return tb[k];
      };
      // R pairs of one j: distance, bin, one atomic each
      auto pairs_of = [&](const J &pj, int j) {
        if constexpr (sizeof(T) == 8 && !SEARCH) {
          // binary64: the short root for all R pairs, one ballot, and the
          // correctly rounded root for all of them when any lane of the wave
          // has a t near an integer (see t_fast64)
          double q[R], t[R];
          uint32_t gap = gap_init(big_bins);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            q[r] = q64<BOX>(xi[r], yi[r], zi[r], pj.x, pj.y, pj.z, g);
            t[r] = t_fast64(q[r], g.s, gap);
          }
          if (__builtin_expect(any_near(gap), 0))
#pragma unroll
            for (int r = 0; r < R; ++r) t[r] = sqrt_cr(q[r]) * g.s;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            uint32_t l = lo[r];
            if constexpr (DIAG) l = j > wbase + r * 64 + lane ? l : hi;
            count_t(t[r], l, 0u);
          }
          return;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          uint32_t l = lo[r], lb = lob[r];
          if constexpr (DIAG) {
            const bool up = j > wbase + r * 64 + lane;
            l = up ? l : hi;
            lb = up ? lb : hib;
          }
          if constexpr (SEARCH) {
            T dx, dy, dz;
            if constexpr (kPacked)
              tric_vec32(pj.ab, nab[r], zi[r], __uint_as_float(static_cast<uint32_t>(pj.cc)),
                         g, dx, dy, dz);
            else
              reduce64<BOX>(xi[r], yi[r], zi[r], pj.x, pj.y, pj.z, g, dx, dy, dz);
            const T q0 = fmaT(dz, dz, fmaT(dy, dy, dx * dx));
            // valid pairs at least half the shortest lattice vector long
            // are searched later; they must not count now
            const bool need = l == 0u && q0 >= qskip;
            if constexpr (sizeof(T) == 4)
              count_t(bin_bits32(__builtin_amdgcn_sqrtf(q0)), need ? hi : l, need ? hib : lb);
            else
              count_t(t_guarded64(q0, g.s, big_bins), need ? hi : l, 0u);
            const uint64_t m = __builtin_amdgcn_ballot_w64(need);
            if (m != 0) {
              const int below = __builtin_amdgcn_mbcnt_hi(
                  static_cast<uint32_t>(m >> 32),
                  __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
              if (need) {
                int pos = head + qn + below;  // < 2 cap: head < cap, qn + below < cap
                if (pos >= cap) pos -= cap;
                // binary32: the octant from the exact signs of the
                // fixed-point differences, as the bits of w; binary64 takes
                // it in the drain from the vector itself
                V e;
                e.x = dx; e.y = dy; e.z = dz;
                if constexpr (kPacked)
                  e.w = __int_as_float(octant32(pj.ab, nab[r], zi[r],
                                                __uint_as_float(static_cast<uint32_t>(pj.cc))));
                else
                  e.w = T(0);
                wq[pos] = e;
              }
              qn += __builtin_popcountll(m);
              if (qn >= 64) drain(64);
            }
          } else if constexpr (kPacked) {
            // c differences of i-particles r and r+1 from one 64-bit add
            const uint64_t dcc = pj.cc + nzz[r / 2];
            const float fc = static_cast<float>(static_cast<int32_t>(
                static_cast<uint32_t>(r % 2 == 0 ? dcc : dcc >> 32)));
            count_t(bits32_packed_c<BOX>(pj.ab, nab[r], fc, g), l, lb);
          } else if constexpr (sizeof(T) == 4) {
            count_t(bin_bits32(pair_t<T, BOX>(xi[r], yi[r], zi[r], pj.x, pj.y, pj.z, g)), l, lb);
          } else {
            count_t(pair_t<T, BOX>(xi[r], yi[r], zi[r], pj.x, pj.y, pj.z, g), l, lb);
          }
        }
      };
      // Ping-pong over two j registers: the read of the next j is issued
      // before the current j's atomics. LDS operations complete in order, so
      // a read issued after the atomics would wait for all of them
      // (bank-conflicted) before the arithmetic could start.
      if constexpr (SEARCH) {
        // one copy of the search code: a plain j loop whose next j is read
        // before the current one's atomics (at the end of the tile the
        // look-ahead reads the entry just past it, never used)
        J pn = load_j(js);
        for (int jj = js; jj < jcount; ++jj) {
          const J pc = pn;
          pn = load_j(jj + 1);
          pairs_of(pc, jt + jj);
        }
      } else {
        // j is read through a pointer kept in a VGPR, so the two reads of an
        // iteration use immediate offsets and one add moves it on (a uniform
        // SGPR address would cost a v_mov per read). The zero is opaque to
        // the compiler on purpose.
        int vzero;
        asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
        const V *cur = tb + js + vzero;
        auto load_at = [&](const V *q) -> J {
          if constexpr (kPacked)
            return JPacked{reinterpret_cast<const uint64_t *>(q)[0],
                           reinterpret_cast<const uint64_t *>(q)[1]};
          else
            return *q;
        };
        J pa = load_at(cur);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        int jj = js;
        for (; jj + 1 < jcount; jj += 2, cur += 2) {
          const J pb = load_at(cur + 1);
          // binary32: pin the read ahead of the atomics (measured faster);
          // binary64 has enough arithmetic per j to hide it unpinned
          if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
          pairs_of(pa, jt + jj);
          // at the end of a tile this reads the entry just past it (the
          // next buffer, the histogram or the allocation's pad): never used
          pa = load_at(cur + 2);
          if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
          pairs_of(pb, jt + jj + 1);
        }
        if (jj < jcount) pairs_of(pa, jt + jj);
      }
    }
  }
  if constexpr (SEARCH) {
    if (qn > 0) drain(qn);
    // one atomic per wave and item for each count (one address each for
    // the whole frame): searched pairs, then the images evaluated for them
    unsigned long long *const searched = F->searched;
    if (searched != nullptr && n_searched != 0 && lane == 0) {
      atomicAdd(searched, static_cast<unsigned long long>(n_searched));
      atomicAdd(searched + 1, static_cast<unsigned long long>(n_images));
    }
  }
}

// Workgroups of up to 1024 threads share one LDS histogram (more waves per
// CU when a wide histogram leaves room for one workgroup only). The image
// search keeps many more live values and is limited to 256 threads.
template <int BOX>
constexpr int max_threads() {
  return BOX == kBoxTricSearch ? 256 : 1024;
}

template <typename T, int R, int BOX, int MODE>
__global__ __launch_bounds__(max_threads<BOX>()) void pairs_kernel(PairKernelArgs a) {
  using V = typename V4<T>::type;
  extern __shared__ __align__(32) unsigned char smem[];
  __shared__ int s_item;
  V *tile = reinterpret_cast<V *>(smem);
  // the histogram follows the two j-tiles and a guard of kGuardBytes: one
  // word per copy for binary32 bin -1 (t < 1/4), added to bin 0 on flush.
  // The host's allocation has one spare coordinate entry there.
  // (sorted frames: two entries per j, then the tiles' group boxes)
  constexpr int EPJ = BOX == kBoxTricSorted && sizeof(T) == 4 ? 2 : 1;
  const size_t tiles_bytes = 2 * static_cast<size_t>(a.tj) * EPJ * sizeof(V) +
                             (BOX == kBoxTricSorted ? kSortedBoxBytes : 0);
  uint32_t *hist = reinterpret_cast<uint32_t *>(smem + tiles_bytes + kGuardBytes);
  const int tid = threadIdx.x;
  // lane-interleaved sub-histogram copies: lanes of one instruction that
  // hit the same bin use different words (and banks) when copies > 1
  uint32_t *my = hist + (tid & 63) % a.copies;
  // image-search queues after the histogram, 32-byte aligned
  const size_t q_off = (2 * static_cast<size_t>(a.tj) * sizeof(V) + kGuardBytes +
                        static_cast<size_t>(a.copies) * a.stride * 4 + 31) / 32 * 32;
  V *queue = reinterpret_cast<V *>(smem + q_off);
  V *shifts = queue + (blockDim.x / 64) * queue_cap(R);

  constexpr bool GLOBAL = MODE == kModeGlobal;
  if constexpr (!GLOBAL)
    for (int k = tid - a.copies; k < a.copies * a.stride; k += blockDim.x) hist[k] = 0u;

  int cur_frame = -1, cur_hist = -1, cur_sweep = -1;
  uint64_t acc = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int it = uni(s_item);
    if (it >= a.n_items) break;
    WorkItem w;
    {
      const WorkItem *p = a.items + it;
      w.frame = uni(p->frame); w.hist = uni(p->hist); w.sweep = uni(p->sweep);
      w.flags = uni(p->flags); w.i0 = uni(p->i0); w.i1 = uni(p->i1);
      w.j0 = uni(p->j0); w.j1 = uni(p->j1);
    }
    if constexpr (!GLOBAL) {
      const uint64_t npairs =
          static_cast<uint64_t>(w.i1 - w.i0) * static_cast<uint64_t>(w.j1 - w.j0);
      if (w.frame != cur_frame || w.hist != cur_hist || w.sweep != cur_sweep ||
          acc + npairs > 0xffffffffull) {
        if (cur_frame >= 0) {
          flush_hist(hist, a, a.frames + cur_frame, cur_hist, cur_sweep);
          __syncthreads();
        }
        cur_frame = w.frame; cur_hist = w.hist; cur_sweep = w.sweep;
        acc = 0;
      }
      acc += npairs;
    }
    const FrameParams *F = a.frames + w.frame;
    if (w.flags & kItemDiag) {
      run_item<T, R, BOX, MODE, true, true>(a, w, F, tile, my, queue, shifts);
    } else {
      // the search needs the clamp to hold back queued pairs
      bool clamp = true;
      if constexpr (MODE == kModeLds && BOX != kBoxTricSearch)
        clamp = !((w.flags & kItemFull) && uni(F->noclamp));
      if (clamp)
        run_item<T, R, BOX, MODE, false, true>(a, w, F, tile, my, queue, shifts);
      else if constexpr (MODE == kModeLds && BOX != kBoxTricSearch)
        run_item<T, R, BOX, kModeLds, false, false>(a, w, F, tile, my, queue, shifts);
    }
  }
  if constexpr (!GLOBAL)
    if (cur_frame >= 0) flush_hist(hist, a, a.frames + cur_frame, cur_hist, cur_sweep);
}

// --------------------------------------------------------------------------
// Small kernels
// --------------------------------------------------------------------------

__global__ void zero_kernel(uint64_t *__restrict__ out, int64_t n, int32_t *counters,
                            int32_t n_counters, uint64_t *oor, const uint64_t *pairs,
                            int32_t n_hist) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t i0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (int64_t i = i0; i < n_counters; i += step) counters[i] = 0;
  if (oor)
    for (int64_t i = i0; i < n_hist; i += step) oor[i] = pairs[i];
  for (int64_t i = i0; i < n; i += step) out[i] = 0ull;
}

__global__ void oor_kernel(const uint64_t *__restrict__ hist, int32_t n_bins,
                           const uint64_t *__restrict__ pairs, uint64_t *__restrict__ oor) {
  __shared__ unsigned long long part[256];
  const int h = blockIdx.x;
  unsigned long long v = 0;
  for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
    v += hist[static_cast<size_t>(h) * n_bins + b];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) oor[h] = pairs[h] - part[0];
}

template <typename T, int BOX>
__global__ void pair_t_kernel(const FrameParams *F, const int32_t *__restrict__ pi,
                              const int32_t *__restrict__ pj, int64_t n_pairs, int32_t n,
                              double *__restrict__ out) {
  using V = typename V4<T>::type;
  const V *X = static_cast<const V *>(F->coords);
  const typename Geo<T>::type g = Geo<T>::load(F);
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n_pairs;
       k += step) {
    const int i = min(max(pi[k], 0), n - 1), j = min(max(pj[k], 0), n - 1);
    const V a = X[i], b = X[j];
    out[k] = static_cast<double>(pair_t<T, BOX>(a.x, a.y, a.z, b.x, b.y, b.z, g));
  }
}

using PairFn = void (*)(PairKernelArgs);

template <typename T, int R, int SW>
PairFn pick_box(int box) {
  switch (box) {
    case kBoxNone: return pairs_kernel<T, R, kBoxNone, SW>;
    case kBoxOrtho: return pairs_kernel<T, R, kBoxOrtho, SW>;
    case kBoxTric: return pairs_kernel<T, R, kBoxTric, SW>;
    case kBoxCube:
      if constexpr (sizeof(T) == 4) return pairs_kernel<T, R, kBoxCube, SW>;
      return pairs_kernel<T, R, kBoxOrtho, SW>;
    case kBoxTricSorted: return pairs_kernel<T, R, kBoxTricSorted, SW>;
    default: return pairs_kernel<T, R, kBoxTricSearch, SW>;
  }
}

template <typename T, int R>
PairFn pick_mode(int box, int mode) {
  switch (mode) {
    case kModeSweep: return pick_box<T, R, kModeSweep>(box);
    case kModeGlobal: return pick_box<T, R, kModeGlobal>(box);
    default: return pick_box<T, R, kModeLds>(box);
  }
}

template <typename T>
PairFn pick_r(int r, int box, int mode) {
  return r == 8 ? pick_mode<T, 8>(box, mode) : pick_mode<T, 4>(box, mode);
}

PairFn pick(int precision, int r, int box, int mode) {
  return precision == 1 ? pick_r<double>(r, box, mode) : pick_r<float>(r, box, mode);
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

}  // namespace

hipError_t launch_stage_sorted(int precision, const double *in, void *out, int64_t n,
                               const int64_t *offsets, int32_t n_species, const FrameParams &fp,
                               uint64_t *keys, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n_species < 1 || n_species > kMaxSpeciesStage || n > 0x7FFFFFFFll)
    return hipErrorInvalidValue;
  const int64_t npad = sort_keys_count(n);
  SpeciesOffsets off;
  for (int s = 0; s <= kMaxSpeciesStage; ++s) off.v[s] = offsets[s < n_species ? s : n_species];
  const int threads = 256;
  sort_keys_kernel<<<grid_for(npad, threads), threads, 0, st>>>(in, n, npad, off, n_species, fp,
                                                                keys);
  const int blocks = static_cast<int>(npad / kBitonicBlock);
  bitonic_local_kernel<<<blocks, 1024, 0, st>>>(keys, 0, 1);
  for (int64_t kk = 2 * kBitonicBlock; kk <= npad; kk <<= 1) {
    for (int64_t j = kk / 2; j >= kBitonicBlock; j >>= 1)
      bitonic_global_kernel<<<grid_for(npad / 2, threads), threads, 0, st>>>(keys, npad, j, kk);
    bitonic_local_kernel<<<blocks, 1024, 0, st>>>(keys, kk, 0);
  }
  if (precision == 1)
    stage_sorted64_kernel<<<grid_for(n, threads), threads, 0, st>>>(in, keys, n,
                                                                    static_cast<double4 *>(out));
  else
    stage_sorted_kernel<<<grid_for(n, threads), threads, 0, st>>>(in, keys, n, fp,
                                                                  static_cast<float4 *>(out));
  return hipGetLastError();
}

hipError_t launch_stage(int precision, int box_kind, const double *in, void *out, int64_t n,
                        const FrameParams &fp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int threads = 256;
  const int grid = grid_for(n, threads);
  if (box_kind == kBoxTricSorted) return hipErrorInvalidValue;  // launch_stage_sorted
  if (precision == 1) {
    stage64_kernel<<<grid, threads, 0, st>>>(in, static_cast<double4 *>(out), n);
  } else {
    float4 *o = static_cast<float4 *>(out);
    switch (box_kind) {
      case kBoxNone: stage32_kernel<kBoxNone><<<grid, threads, 0, st>>>(in, o, n, fp); break;
      case kBoxOrtho:
      case kBoxCube: stage32_kernel<kBoxOrtho><<<grid, threads, 0, st>>>(in, o, n, fp); break;
      case kBoxTricSorted: return hipErrorInvalidValue;  // launch_stage_sorted stages these
      default: stage32_kernel<kBoxTric><<<grid, threads, 0, st>>>(in, o, n, fp); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_zero(uint64_t *out, int64_t n_words, int32_t *counters, int32_t n_counters,
                       uint64_t *oor, const uint64_t *pairs, int32_t n_hist, hipStream_t st) {
  const int threads = 256;
  const int64_t n = std::max<int64_t>({n_words, n_counters, oor ? n_hist : 0, 1});
  zero_kernel<<<grid_for(n, threads), threads, 0, st>>>(out, n_words, counters, n_counters, oor,
                                                        pairs, n_hist);
  return hipGetLastError();
}

// Allows a pair kernel the whole LDS of a CU. Every caller sets the same
// value, so contexts launching from several host threads cannot lower the
// limit between another thread's check and launch.
static void allow_full_lds(PairFn fn) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
}

hipError_t launch_pairs(int precision, int box_kind, int mode, const KernelConfig &cfg,
                        const PairKernelArgs &args, int grid, size_t lds_bytes, hipStream_t st) {
  PairFn fn = pick(precision, cfg.r, box_kind, mode);
  allow_full_lds(fn);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.threads), lds_bytes, st, args);
  return hipGetLastError();
}

int pairs_occupancy(int precision, int box_kind, int mode, const KernelConfig &cfg,
                    size_t lds_bytes) {
  PairFn fn = pick(precision, cfg.r, box_kind, mode);
  allow_full_lds(fn);
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, cfg.threads, lds_bytes) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return blocks > 0 ? blocks : 1;
}

hipError_t launch_oor(const uint64_t *hist, int32_t n_hist, int32_t n_bins, const uint64_t *pairs,
                      uint64_t *oor, hipStream_t st) {
  if (n_hist <= 0) return hipSuccess;
  oor_kernel<<<n_hist, 256, 0, st>>>(hist, n_bins, pairs, oor);
  return hipGetLastError();
}

hipError_t launch_stage_batch(int precision, const FrameParams *d_frames, int32_t n_frames,
                              int64_t max_points, hipStream_t st) {
  if (n_frames <= 0 || max_points <= 0) return hipSuccess;
  const int threads = 256;
  int gx = static_cast<int>(std::min<int64_t>((max_points + threads - 1) / threads, 64));
  dim3 grid(gx, n_frames);
  if (precision == 1)
    stage_batch_kernel<1><<<grid, threads, 0, st>>>(d_frames);
  else
    stage_batch_kernel<0><<<grid, threads, 0, st>>>(d_frames);
  return hipGetLastError();
}

hipError_t launch_zero_batch(const FrameParams *d_frames, int32_t n_frames, int64_t max_words,
                             int32_t *counters, int32_t n_counters, hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  const int threads = 256;
  int64_t need = std::max<int64_t>(max_words, n_counters);
  int gx = static_cast<int>(std::min<int64_t>(std::max<int64_t>((need + threads - 1) / threads, 1), 64));
  zero_batch_kernel<<<dim3(gx, n_frames), threads, 0, st>>>(d_frames, counters, n_counters);
  return hipGetLastError();
}

hipError_t launch_oor_batch(const FrameParams *d_frames, int32_t n_frames, int32_t max_hist,
                            hipStream_t st) {
  if (n_frames <= 0 || max_hist <= 0) return hipSuccess;
  oor_batch_kernel<<<dim3(max_hist, n_frames), 256, 0, st>>>(d_frames);
  return hipGetLastError();
}

hipError_t launch_pair_t(int precision, int box_kind, const FrameParams *d_fp, const int32_t *pi,
                         const int32_t *pj, int64_t n_pairs, int32_t n, double *t,
                         hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  const int threads = 256;
  const int grid = grid_for(n_pairs, threads);
  if (precision == 1) {
    switch (box_kind) {
      case kBoxNone: pair_t_kernel<double, kBoxNone><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      case kBoxOrtho:
      case kBoxCube: pair_t_kernel<double, kBoxOrtho><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      case kBoxTric: pair_t_kernel<double, kBoxTric><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      default: pair_t_kernel<double, kBoxTricSearch><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
    }
  } else {
    switch (box_kind) {
      case kBoxNone: pair_t_kernel<float, kBoxNone><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      case kBoxOrtho: pair_t_kernel<float, kBoxOrtho><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      case kBoxCube: pair_t_kernel<float, kBoxCube><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      case kBoxTric: pair_t_kernel<float, kBoxTric><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
      default: pair_t_kernel<float, kBoxTricSearch><<<grid, threads, 0, st>>>(d_fp, pi, pj, n_pairs, n, t); break;
    }
  }
  return hipGetLastError();
}

}  // namespace dh
