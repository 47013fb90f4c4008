// Device building blocks of the SRD step: Philox4x32-10, the word -> uniform
// map, exact fixed-point accumulation, periodic wrap and binning in both
// storage forms, the per-cell draws (axis, Maxwell-Boltzmann factor) and the
// rotation about the cell axis (Rodrigues' formula). Everything here is compiled with -ffp-contract=off so each
// floating-point operation rounds once, in the order written.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mpcd {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): the counter-based,
// stateless generator family the paper's per-cell streams rely on (sec. 3.6).
// Counter layout used by the library: (cell, step, purpose, attempt),
// key = (seed low word, seed high word).
struct U4 {
  uint32_t x, y, z, w;
};

constexpr uint32_t TAG_AXIS = 0;
constexpr uint32_t TAG_THERMO = 1;
constexpr uint32_t TAG_SHIFT = 2;
constexpr uint32_t TAG_AT = 3;
constexpr int GAMMA_MAX_ATTEMPTS = 64;

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// u = (w + 1/2) 2^-32: exact in FP64, strictly inside (0, 1).
__host__ __device__ inline double u01(uint32_t w) {
  return ((double)w + 0.5) * 0x1p-32;
}

// Grid shift of step n (sec. 2): each component uniform on (-a/2, a/2).
__host__ __device__ inline void grid_shift(uint32_t k0, uint32_t k1, uint32_t n,
                                           double a, double s[3]) {
  const U4 w = philox4x32_10(U4{0u, n, TAG_SHIFT, 0u}, k0, k1);
  s[0] = (u01(w.x) - 0.5) * a;
  s[1] = (u01(w.y) - 0.5) * a;
  s[2] = (u01(w.z) - 0.5) * a;
}

// ------------------------------------------------------------ fixed point
// A value x is split into two int64 limbs, hi = round(x 2^20) and
// lo = round((x - hi 2^-20) 2^72); the remainder x - hi 2^-20 is exact
// (|x - hi 2^-20| <= 2^-21 and the operands are within a factor two, or hi is
// 0). Sums of limbs are exact integer sums, so a cell total does not depend on
// the order its particles are visited in: results are deterministic although
// the scatter into the slabs leaves a cell's particles in a run-dependent order. The
// resolution is 2^-72 and the range |x| < 2^30 per term.
struct Fx {
  long long hi, lo;
};

__device__ inline void fx_split(double x, long long& hi, long long& lo, bool& bad) {
  const double C = 6755399441055744.0;  // 1.5 * 2^52: rounds to an integer
  const long long CB = 0x4338000000000000LL;
  bad |= !(fabs(x) < 0x1p30);
  const double t = x * 0x1p20 + C;
  const double hd = t - C;  // exact
  const double r = x - hd * 0x1p-20;  // exact
  const double t2 = r * 0x1p72 + C;
  hi = __double_as_longlong(t) - CB;
  lo = __double_as_longlong(t2) - CB;
}

__device__ inline void fx_add(Fx& acc, double x, bool& bad) {
  long long hi, lo;
  fx_split(x, hi, lo, bad);
  acc.hi += hi;
  acc.lo += lo;
}

__device__ inline double fx_value(const Fx& a) {
  return (double)a.hi * 0x1p-20 + (double)a.lo * 0x1p-72;
}

// One-limb variant used by the FP32 storage form: round(x 2^40) in one int64,
// range |x| < 2^11, resolution 2^-40. A term's rounding error (<= 2^-41) is
// far below the FP32 precision of the stored velocities; sums stay exact
// integer sums, so they remain independent of the order of the terms.
__device__ inline long long fx1_split(double x, bool& bad) {
  const double C = 6755399441055744.0;  // 1.5 * 2^52
  bad |= !(fabs(x) < 0x1p11);
  const double t = x * 0x1p40 + C;  // x 2^40 is exact: one rounding
  return __double_as_longlong(t) - 0x4338000000000000LL;
}

__device__ inline double fx1_value(long long a) { return (double)a * 0x1p-40; }

// ------------------------------------------------------ wrap and binning
// w in (-L, 2L) -> [0, L); the subtraction is exact (Sterbenz), an addition
// that rounds up to L gives 0.
__device__ inline double wrap_box(double w, double L) {
  if (w >= L) {
    w -= L;
  } else if (w < 0.0) {
    w += L;
    if (w >= L) w = 0.0;
  }
  return w;
}

__device__ inline int bin_axis64(double x, double s, double L, double inv_a,
                                 int n) {
  const double w = wrap_box(x + s, L);
  const int i = (int)floor(w * inv_a);
  // w is in [0, L) for any position the stream produced, so only the top
  // clamp can act; the bottom one keeps a corrupt position inside the grid.
  return min(max(i, 0), n - 1);
}

// FP32 cell-relative form: position = home cell h (per axis) + offset o in
// [0, a), all single-precision operations rounded once, no contraction.
__device__ inline int wrap_index(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// i in [-n, 2n) -> i mod n, by two unsigned minima (a negative i is a large
// unsigned value, and i - n wraps round for i < n); any other i is returned
// as an unsigned value >= n.
__device__ inline uint32_t wrap_once(int i, int n) {
  uint32_t u = (uint32_t)i;
  u = min(u, u + (uint32_t)n);
  return min(u, u - (uint32_t)n);
}

__device__ inline void stream_axis32(float& o, int& h, float v, float dt32,
                                     float a32, float inv_a32, int n) {
  const float t = v * dt32;
  const float o1 = o + t;
  float kf = floorf(o1 * inv_a32);
  kf = fminf(fmaxf(kf, -1.0e9f), 1.0e9f);
  float o2 = o1 - kf * a32;
  int k = (int)kf;
  if (o2 >= a32) {
    o2 = 0.0f;
    k += 1;
  }
  if (o2 < 0.0f) o2 = 0.0f;
  o = o2;
  // periodic home cell; a move of a whole box or more (never for
  // |v dt| < L) takes the general modulo
  const uint32_t hn = wrap_once(h + k, n);
  h = hn < (uint32_t)n ? (int)hn : wrap_index(h + k, n);
}

// min(max(floor(x), -1), 1) as an integer: floor and conversion in one
// instruction (out-of-range values saturate and NaN gives 0, as the separate
// floor and conversion do), then the clamp as a median of three.
__device__ inline int floor_unit(float x) {
  int j;
  asm("v_cvt_flr_i32_f32 %0, %1\n\tv_med3_i32 %0, %0, -1, 1" : "=v"(j) : "v"(x));
  return j;
}

__device__ inline int bin_axis32(float o, int h, float s32, float inv_a32,
                                 int n) {
  const float q = o + s32;
  return (int)wrap_once(h + floor_unit(q * inv_a32), n);
}

__device__ inline uint32_t pack_home(int hx, int hy, int hz) {
  return (uint32_t)hx | ((uint32_t)hy << 10) | ((uint32_t)hz << 20);
}
__device__ inline void unpack_home(uint32_t h, int& hx, int& hy, int& hz) {
  hx = (int)(h & 1023u);
  hy = (int)((h >> 10) & 1023u);
  hz = (int)(h >> 20);
}

// ------------------------------------------------------- per-cell draws
// Rotation axis by the cylindrical projection (sec. 3.6): z = 2 u1 - 1,
// phi = 2 pi u2, n = (r cos phi, r sin phi, z), r = sqrt(1 - z^2). The
// angle functions are evaluated as sincospi(2 u2), which needs no argument
// reduction.
__device__ inline void cell_axis(uint32_t cell, uint32_t step, uint32_t k0,
                                 uint32_t k1, double n[3]) {
  const U4 w = philox4x32_10(U4{cell, step, TAG_AXIS, 0u}, k0, k1);
  const double z = 2.0 * u01(w.x) - 1.0;
  const double r = sqrt(fmax(0.0, 1.0 - z * z));
  double sp, cp;
  sincospi(2.0 * u01(w.y), &sp, &cp);
  n[0] = r * cp;
  n[1] = r * sp;
  n[2] = z;
}

// Attempt j of Marsaglia and Tsang's Gamma(k, theta) sampler (k >= 1;
// d = k - 1/3, c = 1/sqrt(9 d)), drawn from counter (cell, step,
// TAG_THERMO, j): words 0, 1 give a Box-Muller normal g (cos branch), word 2
// the uniform U. With t = 1 + c g > 0 and V = t^3, accept if
// U < 1 - 0.0331 g^4 (squeeze) or log U < g^2/2 + d - d V + d log V.
// Returns d V theta, or -1 when the attempt is rejected.
// The attempt in two parts. gamma_quick draws the attempt's numbers and
// decides what needs no logarithm of U: returns GQ_ACCEPT (squeeze),
// GQ_REJECT (t <= 0), or GQ_FULL with g, V, U kept for gamma_full, the full
// test. Splitting lets a kernel run the full test only for the few attempts
// that reach it.
enum { GQ_ACCEPT = 0, GQ_REJECT = 1, GQ_FULL = 2 };

// The numbers of attempt j: the Box-Muller normal g and the uniform U. They
// depend on (cell, step, j) only, not on N_c.
__device__ inline void gamma_numbers(uint32_t cell, uint32_t step, uint32_t j, uint32_t k0,
                                     uint32_t k1, double& g, double& u2) {
  const U4 w = philox4x32_10(U4{cell, step, TAG_THERMO, j}, k0, k1);
  const double u0 = u01(w.x), u1 = u01(w.y);
  u2 = u01(w.z);
  g = sqrt(-2.0 * log(u0)) * cospi(2.0 * u1);
}

// The squeeze U < 1 - 0.0331 g^4. It does not depend on k (so not on N_c).
__device__ inline bool gamma_squeeze(double g, double u2) {
  const double sq = g * g;
  return u2 < 1.0 - 0.0331 * (sq * sq);
}

// The decision that needs no logarithm of U, from the attempt's numbers.
__device__ inline int gamma_decide(double g, double u2, double c, double& V) {
  const double t = 1.0 + c * g;
  V = t * t * t;
  if (t <= 0.0) return GQ_REJECT;
  return gamma_squeeze(g, u2) ? GQ_ACCEPT : GQ_FULL;
}

__device__ inline int gamma_quick(uint32_t cell, uint32_t step, uint32_t j, double c,
                                  uint32_t k0, uint32_t k1, double& g, double& V,
                                  double& u2) {
  gamma_numbers(cell, step, j, k0, k1, g, u2);
  return gamma_decide(g, u2, c, V);
}

// The full test with log U given (lu).
__device__ inline bool gamma_full_log(double g, double V, double lu, double d) {
  return lu < 0.5 * g * g + d - d * V + d * log(V);
}

__device__ inline bool gamma_full(double g, double V, double u2, double d) {
  return gamma_full_log(g, V, log(u2), d);
}

__device__ inline double gamma_attempt(uint32_t cell, uint32_t step, uint32_t j,
                                       double d, double c, double theta,
                                       uint32_t k0, uint32_t k1) {
  double g, V, u2;
  const int q = gamma_quick(cell, step, j, c, k0, k1, g, V, u2);
  if (q == GQ_ACCEPT || (q == GQ_FULL && gamma_full(g, V, u2, d))) return d * V * theta;
  return -1.0;
}

// The sampler run attempt after attempt from attempt j0 on; cap_hit is set
// if GAMMA_MAX_ATTEMPTS attempts are all rejected.
__device__ inline double gamma_mt(double k, uint32_t cell, uint32_t step,
                                  uint32_t k0, uint32_t k1, double theta,
                                  bool& cap_hit, uint32_t j0 = 0u) {
  const double d = k - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  // attempts one at a time: an unrolled loop would only hold more registers
#pragma nounroll
  for (uint32_t j = j0; j < (uint32_t)GAMMA_MAX_ATTEMPTS; ++j) {
    const double e = gamma_attempt(cell, step, j, d, c, theta, k0, k1);
    if (e >= 0.0) return e;
  }
  cap_hit = true;
  return k * theta;
}

// Random velocity of one particle under the Andersen-thermostat rule (eq. 4,
// sec. 3.7): counter (tag, step, TAG_AT, 0); Box-Muller on words 0, 1 gives
// two components (cos and sin branches, via sincospi(2 u)), words 2, 3 the
// third (cos branch); scaled by `scale` = sqrt(kT / m).
__device__ inline void at_kick(uint32_t tag, uint32_t step, uint32_t k0, uint32_t k1,
                               double scale, double dv[3]) {
  const U4 w = philox4x32_10(U4{tag, step, TAG_AT, 0u}, k0, k1);
  const double r0 = sqrt(-2.0 * log(u01(w.x)));
  const double r2 = sqrt(-2.0 * log(u01(w.z)));
  double s1, c1;
  sincospi(2.0 * u01(w.y), &s1, &c1);
  dv[0] = scale * (r0 * c1);
  dv[1] = scale * (r0 * s1);
  dv[2] = scale * (r2 * cospi(2.0 * u01(w.w)));
}

// The FP32 storage form draws the AT kicks in single precision (sec. 4.1: the
// mixed-precision model uses single precision wherever the method does not
// need double, which it names for the cell sums and the rotation only):
// uniforms from the top 23 bits of each word, u = (w / 2^9 + 1/2) 2^-23
// (exact in FP32, strictly inside (0, 1)); the same Box-Muller pairing as
// at_kick with single-precision logf, sqrtf, sincospif and cospif, and the
// scale sqrt(kT / m) rounded once to FP32. The FP32 kick is exact in FP64.
__device__ inline float u01f(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

__device__ inline void at_kick32(uint32_t tag, uint32_t step, uint32_t k0, uint32_t k1,
                                 float scale, float dv[3]) {
  const U4 w = philox4x32_10(U4{tag, step, TAG_AT, 0u}, k0, k1);
  const float r0 = sqrtf(-2.0f * logf(u01f(w.x)));
  const float r2 = sqrtf(-2.0f * logf(u01f(w.z)));
  float s1, c1;
  sincospif(2.0f * u01f(w.y), &s1, &c1);
  dv[0] = scale * (r0 * c1);
  dv[1] = scale * (r0 * s1);
  dv[2] = scale * (r2 * cospif(2.0f * u01f(w.w)));
}

// Right-handed rotation of d by the angle a (cos a, sin a, 1 - cos a given)
// about the unit axis n, by Rodrigues' formula evaluated in this order:
// (d cos a + (n x d) sin a) + n ((n . d)(1 - cos a)).
__device__ inline void rodrigues(const double n[3], double ca, double sa, double omc,
                                 const double d[3], double r[3]) {
  const double nd = (n[0] * d[0] + n[1] * d[1]) + n[2] * d[2];
  const double c[3] = {n[1] * d[2] - n[2] * d[1], n[2] * d[0] - n[0] * d[2], n[0] * d[1] - n[1] * d[0]};
  const double q = nd * omc;
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k] = (d[k] * ca + c[k] * sa) + n[k] * q;
}
}  // namespace mpcd
