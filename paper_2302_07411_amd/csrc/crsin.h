// Correctly rounded binary64 sine on [0, RN(pi)] for the 2DLASM generator
// (Sec. 3, Eq. (6)), whose sine arguments pi*mu*(y+3)*x*(1-x) always lie in
// that range.  Both ends of the cipher must compute the same bits, so the
// sine is the exactly rounded one: RN(sin(t)).
//
// Stage 1 (every call): u = t or pi - t as above, split u = j/256 + h with
// |h| <= 2^-9 and a table of sin, cos at j/256 as double-double.  Only
// cos(j/256)*h is formed exactly (one FMA); the h^2 ... h^7 terms, each at
// most 2^-19 of the result, are plain doubles.  The evaluation error is
// below 2^-70 relative (every dropped or rounded term bounded in sin_quick),
// and a rounding test at 2^-68 accepts the result; otherwise (about one call
// in 2^15) the fast path decides.  Stage 1 has about a third of the fast
// path's dependent operations, which set the speed of a 2DLASM chain.
//
// Fast path: reduce t to u = t or pi - t in [0, pi/2 + 2^-53]
// (pi as three doubles, so u is exact to 2^-160), split u = j/64 + h with
// |h| <= 1/128, and evaluate sin(j/64)cos(h) + cos(j/64)sin(h) in
// double-double arithmetic (tables of sin, cos at j/64 as double-double,
// Taylor series in h).  The evaluation error stays below 2^-100 relative; a
// rounding test at 2^-95 accepts the result when both ends of that interval
// round to the same double (Ziv's strategy).
//
// Exact path (when the test fails, about once in 2^41 calls): the same
// decomposition in 256-bit two's-complement fixed point (scale 2^252),
// error below 2^-240 absolute, rounded to nearest-even by inspecting the
// bits; a value within 2^-242 of a rounding boundary (none is expected: the
// hardest binary64 cases of sin sit far above that) raises `undecided`.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sin_tables.h"

// Host and device: the library's host code uses the same functions for the
// key schedule of 2DLASM master keys.
#define CRSIN_HD __host__ __device__ __forceinline__

namespace cv {
namespace crsin {

struct DD {
  double hi, lo;
};

CRSIN_HD DD two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
CRSIN_HD DD fast_two_sum(double a, double b) {  // |a| >= |b| or a == 0
  const double s = a + b;
  return {s, b - (s - a)};
}
CRSIN_HD DD two_prod(double a, double b) {
  const double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}
CRSIN_HD DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  const DD t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
CRSIN_HD DD dd_add_d(DD a, double b) {
  DD s = two_sum(a.hi, b);
  s.lo += a.lo;
  return fast_two_sum(s.hi, s.lo);
}
CRSIN_HD DD dd_mul(DD a, DD b) {
  DD p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}

constexpr double kHalfPi = 0x1.921fb54442d18p+0;  // RN(pi)/2, exactly half of kPiHi

// u = t, or pi - t for t above pi/2, as a normalised double-double.
CRSIN_HD DD reduce(double t) {
  if (t <= kHalfPi) return {t, 0.0};
  const double d = kPiHi - t;  // exact (Sterbenz: t in [kPiHi/2, kPiHi])
  DD s = two_sum(d, kPiMid);
  s.lo += kPiLo;
  return fast_two_sum(s.hi, s.lo);
}

// The tables per point j: {sin hi, sin lo, cos hi, cos lo}, v1 for stage 1
// (j/256) and v for the fast path (j/64).  Kernels stage them in LDS (a
// sine's table read is on the critical path of a generator step and must not
// wait for global memory); host code fills one copy.
struct LdsTable {
  double v1[kTab1][4];
  double v[kTab][4];
};

CRSIN_HD void fill_entry(LdsTable* t, uint32_t i) {
  if (i < (uint32_t)kTab1) {
    t->v1[i][0] = kSin1DD[i][0];
    t->v1[i][1] = kSin1DD[i][1];
    t->v1[i][2] = kCos1DD[i][0];
    t->v1[i][3] = kCos1DD[i][1];
  }
  if (i < (uint32_t)kTab) {
    t->v[i][0] = kSinDD[i][0];
    t->v[i][1] = kSinDD[i][1];
    t->v[i][2] = kCosDD[i][0];
    t->v[i][3] = kCosDD[i][1];
  }
}
constexpr uint32_t kTabEntries = kTab1 > kTab ? kTab1 : kTab;  // fill_entry indices

// Copy the tables into LDS (all threads of the workgroup take part; the
// caller synchronises before use).
__device__ __forceinline__ void stage_table(LdsTable* t) {
  for (uint32_t i = threadIdx.x; i < kTabEntries; i += blockDim.x) fill_entry(t, i);
}

CRSIN_HD uint64_t bits_of(double x) { return __builtin_bit_cast(uint64_t, x); }

// High 64 bits of a 64x64-bit product.
CRSIN_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// Stage 1; *hi + *lo is the sine's approximation (relative error below
// 2^-70), *hi its rounding to double.  Returns false when the rounding test
// at 2^-68 cannot decide RN(sin t).
//
// With u = c + h (c = j/256 with j = rint(256 u.hi), h = a + b: a = u.hi - c
// exact by Sterbenz' lemma, b = u.lo, |a| <= 2^-9, |b| <= 2^-53 u), and
// S + s = sin c, C + k = cos c from the table:
//   sin u = S + C a + [-S a^2/2] + [s + C b + k a - S a b - C a^2 b/2]
//           + C a^3 (-1/6 + a^2/120 - a^4/5040) + S a^4 (1/24 - a^2/720) + e
// where e (the h^8 and h^9 terms, the other products with b, table
// errors) is below 2^-84 of the result R.  On [0, pi/2 + 2^-53],
// |S| <= 2R and |C a| <= R (1 + 2^-8); C a is formed exactly (P1 + P2), so
//   -S a^2/2 (at most 2^-18 R, two roundings) errs by at most 2^-70 R;
//   C a^3/6 (at most 2^-20.5 R, about five roundings) by at most 2^-71.1 R;
//   the bracket (each term at most 2^-52 R), the a^4 terms (at most
//   2^-39 R) and the additions of the tail (at most 2^-20.4 R) by at most
//   2^-72.4 R together.
// The total, below 2^-69.2 R, is covered by the test bound 2^-68.
CRSIN_HD bool sin_quick(double t, const LdsTable* tab, double* hi, double* lo) {
  double uh, ul;
  if (t <= kHalfPi) {
    uh = t;
    ul = 0.0;
  } else {
    // kPiHi - t is exact (Sterbenz) and a multiple of 2^-52, so it is 0 or
    // above kPiMid (about 1.2e-16): the three-operation exact sum applies
    const DD s = fast_two_sum(kPiHi - t, kPiMid);
    uh = s.hi;
    ul = s.lo + kPiLo;
  }
  const double jd = rint(uh * 256.0);  // no rounding error: |uh*256 - jd| <= 1/2
  const int j = (int)jd;
  const double c = jd * 0x1p-8;
  const double a = uh - c;  // exact (Sterbenz for j >= 1)
  const double b = ul;
  const double S = tab->v1[j][0], s = tab->v1[j][1], C = tab->v1[j][2], k = tab->v1[j][3];
  const double q = a * a;
  const double P1 = C * a, P2 = __builtin_fma(C, a, -P1);  // C a = P1 + P2 exactly
  const double T2 = -0.5 * (S * q);
  const double pc = C * (a * q) * (-kInv6Hi + q * (kInv120Hi - q * kInv5040));
  const double ps = S * (q * q) * (kInv24Hi - q * kInv720Hi);
  const double small = ((s + C * b) + (k * a - S * (a * b) - 0.5 * (C * (q * b)))) + (ps + pc);
  // Both sums have their larger term first (|S| >= sin(1/256) > 2^-9 >= |P1|
  // for j >= 1, and |T2| <= 2^-19 S below s1.hi; for j = 0, S = T2 = 0), so
  // the three-operation exact sum gives the same pair as the six-operation
  // one: fewer FP64 instructions on a 2DLASM chain, identical results.
  const DD s1 = fast_two_sum(S, P1);
  const DD s2 = fast_two_sum(s1.hi, T2);
  const double tail = ((s1.lo + s2.lo) + P2) + small;
  const DD r = fast_two_sum(s2.hi, tail);
  const double e = fabs(r.hi) * 0x1p-68;
  *hi = r.hi;
  *lo = r.lo;
  return r.hi + (r.lo + e) == r.hi + (r.lo - e);
}

// Fast path; returns false when the rounding cannot be decided.
CRSIN_HD bool sin_fast(double t, const LdsTable* tab, double* out) {
  const DD u = reduce(t);
  int j = (int)(u.hi * 64.0 + 0.5);
  j = j > kTab - 1 ? kTab - 1 : j;
  const double c = (double)j * 0.015625;
  const DD h = two_sum(u.hi - c, u.lo);  // u.hi - c is exact
  const DD z = dd_mul(h, h);
  const double zh = z.hi;
  // cos(h) - 1 = z*(-1/2 + z*(1/24 + z*(-1/720 + z*(1/8! - z/10! + z^2/12!))))
  const double p8 = kC8 + zh * (kC10 + zh * kC12);
  DD w = dd_add_d(DD{-kInv720Hi, -kInv720Lo}, zh * p8);
  w = dd_add(DD{kInv24Hi, kInv24Lo}, dd_mul(z, w));
  w = dd_add_d(dd_mul(z, w), -0.5);
  const DD cm1 = dd_mul(z, w);
  // sin(h) = h*(1 + z*(-1/6 + z*(1/120 + z*(-1/7! + z/9! - z^2/11! + z^3/13!))))
  const double q7 = kS7 + zh * (kS9 + zh * (kS11 + zh * kS13));
  DD v = dd_add_d(DD{kInv120Hi, kInv120Lo}, zh * q7);
  v = dd_add(DD{-kInv6Hi, -kInv6Lo}, dd_mul(z, v));
  v = dd_add_d(dd_mul(z, v), 1.0);
  const DD sh = dd_mul(h, v);
  const DD S{tab->v[j][0], tab->v[j][1]}, C{tab->v[j][2], tab->v[j][3]};
  const DD r = dd_add(S, dd_add(dd_mul(S, cm1), dd_mul(C, sh)));
  // Ziv's rounding test with a 2^-95 relative error bound
  const double e = fabs(r.hi) * 0x1p-95;
  const double a = r.hi + (r.lo + e), b = r.hi + (r.lo - e);
  *out = a;
  return a == b;
}

// ------------------------------------------------------ exact path ---
// 256-bit two's complement, value = int / 2^252, w[0] least significant.
struct F256 {
  uint64_t w[4];
};

CRSIN_HD F256 fx_load(const uint64_t* p) { return {{p[0], p[1], p[2], p[3]}}; }

CRSIN_HD F256 fx_add(const F256& a, const F256& b) {
  F256 r;
  uint64_t carry = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint64_t s = a.w[k] + b.w[k];
    const uint64_t c1 = s < a.w[k];
    r.w[k] = s + carry;
    carry = c1 | (r.w[k] < s);
  }
  return r;
}
CRSIN_HD F256 fx_neg(const F256& a) {
  F256 r;
  uint64_t carry = 1;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    r.w[k] = ~a.w[k] + carry;
    carry = carry && r.w[k] == 0;
  }
  return r;
}
CRSIN_HD F256 fx_sub(const F256& a, const F256& b) { return fx_add(a, fx_neg(b)); }
CRSIN_HD bool fx_neg_p(const F256& a) { return (a.w[3] >> 63) != 0; }

// Signed product, truncated to the 2^-252 grid.
CRSIN_HD F256 fx_mul(F256 a, F256 b) {
  const bool na = fx_neg_p(a), nb = fx_neg_p(b);
  if (na) a = fx_neg(a);
  if (nb) b = fx_neg(b);
  uint64_t P[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 4; i++) {
    uint64_t carry = 0;
    for (int k = 0; k < 4; k++) {
      const uint64_t lo = a.w[i] * b.w[k], hi = mulhi64(a.w[i], b.w[k]);
      uint64_t s = P[i + k] + lo;
      uint64_t c = s < lo;
      s += carry;
      c += s < carry;
      P[i + k] = s;
      carry = hi + c;  // hi <= 2^64-2, so no overflow
    }
    P[i + 4] += carry;
  }
  F256 r;
#pragma unroll
  for (int k = 0; k < 4; k++) r.w[k] = (P[k + 3] >> 60) | (P[k + 4] << 4);
  return (na != nb) ? fx_neg(r) : r;
}

// Exact conversion of a double in [2^-200, 8) to fixed point.
CRSIN_HD F256 fx_from_double(double t) {
  const uint64_t bits = bits_of(t);
  const int e = (int)((bits >> 52) & 0x7FF) - 1023;
  const uint64_t m = (bits & ((1ull << 52) - 1)) | (1ull << 52);
  const int sh = e - 52 + 252;  // position of the mantissa's lowest bit
  F256 r{{0, 0, 0, 0}};
  const int q = sh >> 6, s = sh & 63;
  r.w[q] = m << s;
  if (s && q + 1 < 4) r.w[q + 1] = m >> (64 - s);
  return r;
}

CRSIN_HD int fx_bit(const F256& a, int i) { return (int)((a.w[i >> 6] >> (i & 63)) & 1u); }

// Round a positive fixed-point value to binary64, nearest-even; `undecided`
// when it lies within 2^10 units of a rounding boundary.
CRSIN_HD double fx_to_double(const F256& R, bool* undecided) {
  int p = 255;
  while (p >= 0 && !fx_bit(R, p)) p--;
  if (p < 53) {  // not reached for the arguments of the exact path
    *undecided = true;
    return 0.0;
  }
  const int low = p - 52;  // lowest mantissa bit
  uint64_t m = 0;
  for (int i = p; i >= low; i--) m = (m << 1) | (uint64_t)fx_bit(R, i);
  // remainder below the mantissa against the half unit 2^(low-1)
  const bool half_bit = fx_bit(R, low - 1);
  bool below_all_zero = true, below_all_one = true;  // bits low-2 .. 11
  for (int i = low - 2; i >= 11; i--) {
    const int b = fx_bit(R, i);
    below_all_zero = below_all_zero && !b;
    below_all_one = below_all_one && b;
  }
  if ((half_bit && below_all_zero) || (!half_bit && below_all_one)) *undecided = true;
  if (half_bit) m += 1;  // above the midpoint (ties are undecided above)
  return ldexp((double)m, low - 252);  // m may be 2^53: still exact
}

CRSIN_HD double sin_exact(double t, bool* undecided) {
  const F256 tf = fx_from_double(t);
  const F256 u = t <= kHalfPi ? tf : fx_sub(fx_load(kPiFX), tf);
  // j = round(u * 64); 1/64 is 2^246 in fixed point
  F256 half{{0, 0, 0, 0}};
  half.w[245 >> 6] = 1ull << (245 & 63);
  const F256 uj = fx_add(u, half);
  const int j = (int)((uj.w[3] >> 54) & 0xFFu);  // bits 246..253 (j <= 101)
  F256 c{{0, 0, 0, 0}};
  c.w[246 >> 6] = (uint64_t)j << (246 & 63);
  const F256 h = fx_sub(u, c);
  // Taylor series of sin(h) and cos(h) to h^21 (|h| <= 2^-7: remainder < 2^-210)
  F256 sn = h, cs = fx_load(kInvFactFX[0]);
  F256 pw = h;  // h^k
  for (int k = 2; k <= 21; k++) {
    pw = fx_mul(pw, h);
    const F256 term = fx_mul(pw, fx_load(kInvFactFX[k]));
    const bool neg = ((k / 2) & 1) != 0;  // signs of h^k/k!: + - - + + - - ...
    if (k & 1)
      sn = neg ? fx_sub(sn, term) : fx_add(sn, term);
    else
      cs = neg ? fx_sub(cs, term) : fx_add(cs, term);
  }
  const F256 r = fx_add(fx_mul(fx_load(kSinFX[j]), cs), fx_mul(fx_load(kCosFX[j]), sn));
  return fx_to_double(r, undecided);
}

// RN(sin(t)) for t in [0, RN(pi)].  `force_exact` sends every argument at
// least 2^-30 to the exact path (for testing it); smaller arguments are
// always decided by the fast path.
CRSIN_HD double cr_sin(double t, const LdsTable* tab, bool force_exact,
                                         bool* undecided) {
  double r, rl;
  if (!force_exact && sin_quick(t, tab, &r, &rl)) return r;
  const bool ok = sin_fast(t, tab, &r);
  if (ok && !(force_exact && t >= 0x1p-30)) return r;
  if (t < 0x1p-30) {  // the fast path cannot fail here; keep its result but report
    *undecided = true;
    return r;
  }
  return sin_exact(t, undecided);
}

}  // namespace crsin
}  // namespace cv
