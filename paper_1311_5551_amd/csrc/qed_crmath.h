// Correctly rounded exp, log, sin and cos for the FP64 kernels.
//
// Each function evaluates its result in double-double arithmetic (Dekker's exact
// two-sum / two-product splits, relative error ~2^-100) and rounds once to double.  The
// rounded value is then the correctly rounded one except when the exact result lies
// within ~2^-100 of a rounding midpoint (probability ~2^-47 per call).  Correct rounding
// makes the FP64 step independent of the math library's last-bit choices, so two correct
// implementations of the method agree bit for bit.
//
//   exp: x = k ln2 + r, |r| <= ln2/2 (ln2 in three parts, the first with 42 bits so k*L1
//        is exact), e^r by a degree-25 Taylor polynomial in Horner form, times 2^k.
//   log: x = m 2^e, m in [1/sqrt2, sqrt2); one Newton step y1 = y0 + m e^{-y0} - 1 from the
//        library value y0 = log(m), with e^{-y0} in double-double; plus e ln2.
//   sin/cos: x = k pi/2 + r, |r| <= pi/4 (pi/2 in three parts, the first with 33 bits),
//        Taylor polynomials in r^2 to degree 29, quadrant from k mod 4.
// These full double-double evaluations (*_dd) are the slow paths.  The entry points cr_exp,
// cr_log, cr_sin, cr_cos and cr_sincos first evaluate a shorter series whose unrounded error is
// below 2^-68 and return its rounding when an interval of 2^-66 around it rounds to a single
// double (Ziv's test), which is then the correctly rounded result; about one call in 5000 falls
// through to the slow path.  Same results, a tenth of the work and of the dependent latency.
#pragma once

#include <hip/hip_runtime.h>

namespace qedk {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd dd_two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ dd dd_fast_two_sum(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ dd dd_two_prod(double a, double b) {
  const double p = a * b;
  return {p, fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = dd_two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return dd_fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = dd_two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = dd_two_prod(a.hi, b);
  p.lo += a.lo * b;
  return dd_fast_two_sum(p.hi, p.lo);
}

// 1/n!, n = 0..29, as double-double; filled by the host (init_crmath in qed_step.hip, the
// translation unit whose kernels use it)
static __constant__ dd c_inv_fact[30];

constexpr double kLn2A = 0x1.62e42fefa3800p-1;   // ln 2 = A + B + C, A with 42 significant bits
constexpr double kLn2B = 0x1.ef35793c76730p-45;
constexpr double kLn2C = 0x1.f97b57a079a19p-103;
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;  // ln 2 as a double-double
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kPio2A = 0x1.921fb54400000p+0;  // pi/2 = A + B + C, A with 33 significant bits
constexpr double kPio2B = 0x1.0b4611a626331p-34;
constexpr double kPio2C = 0x1.1701b839a2520p-88;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;

// e^x as a double-double, for -740 < x < 709
__device__ inline dd exp_dd(double x) {
  const double k = rint(x * kInvLn2);
  // r = x - k ln2: k*A and x - k*A are exact (Sterbenz), k*B is split exactly, k*C is below
  // the working precision's last bit
  dd r = dd_add(dd{x - k * kLn2A, 0.0}, dd_two_prod(-k, kLn2B));
  r = dd_fast_two_sum(r.hi, r.lo - k * kLn2C);
  dd p = c_inv_fact[25];
#pragma unroll
  for (int n = 24; n >= 0; --n) p = dd_add(dd_mul(p, r), c_inv_fact[n]);
  const int ki = (int)k;
  return {ldexp(p.hi, ki), ldexp(p.lo, ki)};
}

__device__ __noinline__ double cr_exp_dd(double x) {
  if (!(x < 709.0)) return x != x ? x : (x > 709.782712893384 ? INFINITY : exp(x));
  if (!(x > -700.0)) return exp(x);  // results near the subnormal range are left to the library
  const dd e = exp_dd(x);
  return e.hi + e.lo;
}

__device__ __noinline__ double cr_log_dd(double x) {
  if (!(x > 0.0) || !(x < INFINITY)) return log(x);
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double y0 = log(m);
  // Newton step on e^y = m: y1 = y0 + m e^{-y0} - 1
  const dd t = dd_add(dd_mul_d(exp_dd(-y0), m), dd{-1.0, 0.0});
  const dd y = dd_add(dd{y0, 0.0}, t);
  const double ed = (double)e;
  dd l = dd_two_prod(ed, kLn2Hi);
  l.lo += ed * kLn2Lo;
  l = dd_fast_two_sum(l.hi, l.lo);
  const dd s = dd_add(l, y);
  return s.hi + s.lo;
}

// sin and cos of x (|x| < 2^20) in one reduction.  The entry points are out of line so that
// the double-double temporaries do not raise the register budget of the calling kernels.
__device__ __noinline__ void cr_sincos_dd(double x, double* sn, double* cs) {
  if (!(fabs(x) < 1048576.0)) {
    *sn = sin(x);
    *cs = cos(x);
    return;
  }
  const double k = rint(x * kTwoOverPi);
  dd r = dd_add(dd{x - k * kPio2A, 0.0}, dd_two_prod(-k, kPio2B));
  r = dd_fast_two_sum(r.hi, r.lo - k * kPio2C);
  const dd r2 = dd_mul(r, r);
  const dd mr2 = {-r2.hi, -r2.lo};
  // cos r = sum (-1)^n r^2n / (2n)!, sin r = r sum (-1)^n r^2n / (2n+1)!
  dd pc = c_inv_fact[28], ps = c_inv_fact[29];
#pragma unroll
  for (int n = 13; n >= 0; --n) {
    pc = dd_add(dd_mul(pc, mr2), c_inv_fact[2 * n]);
    ps = dd_add(dd_mul(ps, mr2), c_inv_fact[2 * n + 1]);
  }
  const dd s = dd_mul(ps, r);
  const double sv = s.hi + s.lo, cv = pc.hi + pc.lo;
  const int q = ((int)fmod(k, 4.0) + 4) & 3;
  *sn = q == 0 ? sv : q == 1 ? cv : q == 2 ? -sv : -cv;
  *cs = q == 0 ? cv : q == 1 ? -sv : q == 2 ? -cv : sv;
}

// sin(x + qs pi/2) alone: the same reduction and the same double-double polynomial as the
// matching output of cr_sincos (so the same bits), with only the polynomial the quadrant needs
// evaluated.  qs = 0: sin, qs = 1: cos.
__device__ __noinline__ double cr_sinq_dd(double x, int qs) {
  if (!(fabs(x) < 1048576.0)) return qs ? cos(x) : sin(x);
  const double k = rint(x * kTwoOverPi);
  dd r = dd_add(dd{x - k * kPio2A, 0.0}, dd_two_prod(-k, kPio2B));
  r = dd_fast_two_sum(r.hi, r.lo - k * kPio2C);
  const dd r2 = dd_mul(r, r);
  const dd mr2 = {-r2.hi, -r2.lo};
  const int q = (((int)fmod(k, 4.0) + 4) + qs) & 3;
  const bool odd = (q & 1) == 0;  // true: sin r series (odd factorials), false: cos r series
  dd p = odd ? c_inv_fact[29] : c_inv_fact[28];
#pragma unroll
  for (int n = 13; n >= 0; --n) p = dd_add(dd_mul(p, mr2), odd ? c_inv_fact[2 * n + 1] : c_inv_fact[2 * n]);
  if (odd) p = dd_mul(p, r);
  const double v = p.hi + p.lo;
  return (q & 2) ? -v : v;
}

// ---------------------------------------------------------------------------
// Fast path of the same correctly rounded sin and cos (Ziv's rounding test).  The reduced
// argument r = rh + rl is a double-double as above; sin rh and cos rh come from their Taylor
// series with the terms up to r^7 (sin) and r^6 (cos) in double-double and the rest, a tail
// below 3e-6 of the result, in double, truncated past r^19 and r^20 (remainders below 2^-72).
// rl enters through rl cos rh and -rl sin rh (second order below 2^-100).  The unrounded
// result is thus within 2^-68 of the exact value (relative).  It is returned when every value
// within kZivEps of it rounds to the same double, i.e. when that double is the correctly rounded
// result; otherwise (probability ~2^-12 per call) the full double-double series above decides.
// ---------------------------------------------------------------------------
constexpr double kZivEps = 0x1p-66;

// 1/n! rounded to double, for the double tails
namespace crc {
constexpr double i8 = 1.0 / 40320.0, i9 = 1.0 / 362880.0, i10 = 1.0 / 3628800.0, i11 = 1.0 / 39916800.0,
                 i12 = 1.0 / 479001600.0, i13 = 1.0 / 6227020800.0, i14 = 1.0 / 87178291200.0,
                 i15 = 1.0 / 1307674368000.0, i16 = 1.0 / 20922789888000.0, i17 = 1.0 / 355687428096000.0,
                 i18 = 1.0 / 6402373705728000.0, i19 = 1.0 / 121645100408832000.0,
                 i20 = 1.0 / 2432902008176640000.0;
}  // namespace crc

__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

// sin rh as a double-double (z = rh^2 exact)
__device__ __forceinline__ dd sin_series_dd(double rh, dd z) {
  using namespace crc;
  const double zh = z.hi;
  double t = -i19;
  t = t * zh + i17;
  t = t * zh - i15;
  t = t * zh + i13;
  t = t * zh - i11;
  t = t * zh + i9;                                          // r^9 on: 1/9! - z/11! + ...
  dd m = dd_add(dd_neg(c_inv_fact[7]), dd_two_prod(zh, t));  // -1/7! + z T
  m = dd_add(dd_mul(z, m), c_inv_fact[5]);
  m = dd_add(dd_mul(z, m), dd_neg(c_inv_fact[3]));          // S(z) = -1/3! + z/5! - ...
  const dd q = dd_mul(z, m);                                // sin rh = rh (1 + z S)
  return dd_add(dd{rh, 0.0}, dd_mul_d(q, rh));
}

// cos rh as a double-double
__device__ __forceinline__ dd cos_series_dd(dd z) {
  using namespace crc;
  const double zh = z.hi;
  double u = i20;
  u = u * zh - i18;
  u = u * zh + i16;
  u = u * zh - i14;
  u = u * zh + i12;
  u = u * zh - i10;
  u = u * zh + i8;                                          // r^8 on: 1/8! - z/10! + ...
  dd m = dd_add(dd_neg(c_inv_fact[6]), dd_two_prod(zh, u));  // -1/6! + z U
  m = dd_add(dd_mul(z, m), c_inv_fact[4]);
  m = dd_add(dd_mul(z, m), dd{-0.5, 0.0});
  return dd_add(dd{1.0, 0.0}, dd_mul(z, m));               // 1 - z/2 + z^2/4! - ...
}

// sin rh and cos rh in double only (for the rl terms)
__device__ __forceinline__ double sin_series_d(double rh, double zh) {
  using namespace crc;
  double t = -i19;
  t = t * zh + i17;
  t = t * zh - i15;
  t = t * zh + i13;
  t = t * zh - i11;
  t = t * zh + i9;
  t = t * zh - 1.0 / 5040.0;
  t = t * zh + 1.0 / 120.0;
  t = t * zh - 1.0 / 6.0;
  return rh + rh * (zh * t);
}
__device__ __forceinline__ double cos_series_d(double zh) {
  using namespace crc;
  double u = i20;
  u = u * zh - i18;
  u = u * zh + i16;
  u = u * zh - i14;
  u = u * zh + i12;
  u = u * zh - i10;
  u = u * zh + i8;
  u = u * zh - 1.0 / 720.0;
  u = u * zh + 1.0 / 24.0;
  u = u * zh - 0.5;
  return 1.0 + zh * u;
}

// x = k pi/2 + r with r as a double-double (the reduction of cr_sincos_dd)
__device__ __forceinline__ dd reduce_pio2(double x, double* k) {
  *k = rint(x * kTwoOverPi);
  dd r = dd_add(dd{x - *k * kPio2A, 0.0}, dd_two_prod(-*k, kPio2B));
  return dd_fast_two_sum(r.hi, r.lo - *k * kPio2C);
}

// the double nearest to v when every value within kZivEps |v| of it rounds to it
__device__ __forceinline__ bool ziv_round(dd v, double* out) {
  const double e = kZivEps * fabs(v.hi);
  const double a = v.hi + (v.lo + e), b = v.hi + (v.lo - e);
  *out = a;
  return a == b;
}

__device__ inline void cr_sincos(double x, double* sn, double* cs) {
  if (fabs(x) < 1048576.0) {
    double k;
    const dd r = reduce_pio2(x, &k);
    const dd z = dd_two_prod(r.hi, r.hi);
    const dd s0 = sin_series_dd(r.hi, z), c0 = cos_series_dd(z);
    const dd s = dd_add(s0, dd{r.lo * c0.hi, 0.0});
    const dd c = dd_add(c0, dd{-r.lo * s0.hi, 0.0});
    double sv, cv;
    if (ziv_round(s, &sv) && ziv_round(c, &cv)) {
      const int q = (int)k & 3;
      *sn = q == 0 ? sv : q == 1 ? cv : q == 2 ? -sv : -cv;
      *cs = q == 0 ? cv : q == 1 ? -sv : q == 2 ? -cv : sv;
      return;
    }
  }
  cr_sincos_dd(x, sn, cs);
}

// sin(x + qs pi/2): qs = 0 sin, qs = 1 cos
__device__ inline double cr_sinq(double x, int qs) {
  if (fabs(x) < 1048576.0) {
    double k;
    const dd r = reduce_pio2(x, &k);
    const dd z = dd_two_prod(r.hi, r.hi);
    const int q = ((int)k + qs) & 3;
    dd v;
    if (q & 1) v = dd_add(cos_series_dd(z), dd{-r.lo * sin_series_d(r.hi, z.hi), 0.0});  // +-cos r
    else v = dd_add(sin_series_dd(r.hi, z), dd{r.lo * cos_series_d(z.hi), 0.0});        // +-sin r
    double out;
    if (ziv_round(v, &out)) return (q & 2) ? -out : out;
  }
  return cr_sinq_dd(x, qs);
}

__device__ inline double cr_sin(double x) { return cr_sinq(x, 0); }
__device__ inline double cr_cos(double x) { return cr_sinq(x, 1); }

// Fast paths of the correctly rounded exp and log (the same Ziv test).
//   exp: x = k ln2 + r (double-double, |r| <= 0.347); e^r by its Taylor series with the terms up
//        to r^5 in double-double and r^6 .. r^17 in double (tail below 1.7e-3 of the result,
//        truncation below 1e-24): the unrounded e^r is within 2^-68 of the exact value; times 2^k.
//   log: x = m 2^e, m in [1/sqrt2, sqrt2); log m = 2 atanh(s), s = (m - 1)/(m + 1) as a
//        double-double (|s| <= 0.172), the series 2 (s + s^3/3 + s^5/5) in double-double and
//        s^7/7 .. s^27/27 in double (tail below 4e-6 of the result, truncation below 1e-21);
//        plus e ln2.  Relative error below 2^-68 of the result.
constexpr double kThirdHi = 0x1.5555555555555p-2, kThirdLo = 0x1.5555555555555p-56;  // 1/3
constexpr double kFifthHi = 0x1.999999999999ap-3, kFifthLo = -0x1.999999999999ap-57;  // 1/5

__device__ inline double cr_exp(double x) {
  if (x > -700.0 && x < 709.0) {
    using namespace crc;
    const double k = rint(x * kInvLn2);
    dd r = dd_add(dd{x - k * kLn2A, 0.0}, dd_two_prod(-k, kLn2B));
    r = dd_fast_two_sum(r.hi, r.lo - k * kLn2C);
    const double rh = r.hi;
    double t = i17;
    t = t * rh + i16;
    t = t * rh + i15;
    t = t * rh + i14;
    t = t * rh + i13;
    t = t * rh + i12;
    t = t * rh + i11;
    t = t * rh + i10;
    t = t * rh + i9;
    t = t * rh + i8;
    t = t * rh + 1.0 / 5040.0;
    t = t * rh + 1.0 / 720.0;                          // 1/6! + r/7! + ...
    dd p = dd_add(c_inv_fact[5], dd_two_prod(rh, t));  // 1/5! + r (1/6! + ...)
    p = dd_add(dd_mul(r, p), c_inv_fact[4]);
    p = dd_add(dd_mul(r, p), c_inv_fact[3]);
    p = dd_add(dd_mul(r, p), c_inv_fact[2]);
    p = dd_add(dd_mul(r, p), c_inv_fact[1]);
    p = dd_add(dd_mul(r, p), c_inv_fact[0]);
    double out;
    if (ziv_round(p, &out)) return ldexp(out, (int)k);
  }
  return cr_exp_dd(x);
}

__device__ inline double cr_log(double x) {
  if (x >= 0x1p-1021 && x < INFINITY) {
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752) {
      m *= 2.0;
      e -= 1;
    }
    const double num = m - 1.0;              // exact
    const dd den = dd_two_sum(m, 1.0);       // m + 1 exactly
    const double q1 = num / den.hi;
    const dd pq = dd_two_prod(q1, den.hi);
    const double q2 = (((num - pq.hi) - pq.lo) - q1 * den.lo) / den.hi;
    const dd s = dd_fast_two_sum(q1, q2);    // (m - 1)/(m + 1)
    const dd s2 = dd_mul(s, s);
    const double z = s2.hi;
    double t = 1.0 / 27.0;
    t = t * z + 1.0 / 25.0;
    t = t * z + 1.0 / 23.0;
    t = t * z + 1.0 / 21.0;
    t = t * z + 1.0 / 19.0;
    t = t * z + 1.0 / 17.0;
    t = t * z + 1.0 / 15.0;
    t = t * z + 1.0 / 13.0;
    t = t * z + 1.0 / 11.0;
    t = t * z + 1.0 / 9.0;
    t = t * z + 1.0 / 7.0;                                       // 1/7 + z/9 + ...
    dd p = dd_add(dd{kFifthHi, kFifthLo}, dd_two_prod(z, t));    // 1/5 + z (1/7 + ...)
    p = dd_add(dd_mul(s2, p), dd{kThirdHi, kThirdLo});
    p = dd_add(dd_mul(s2, p), dd{1.0, 0.0});
    const dd lm = dd_mul(p, s);                                  // atanh(s)
    const double ed = (double)e;
    dd l = dd_two_prod(ed, kLn2Hi);
    l.lo += ed * kLn2Lo;
    l = dd_fast_two_sum(l.hi, l.lo);
    const dd y = dd_add(l, dd{2.0 * lm.hi, 2.0 * lm.lo});
    double out;
    if (ziv_round(y, &out)) return out;
  }
  return cr_log_dd(x);
}

}  // namespace qedk
