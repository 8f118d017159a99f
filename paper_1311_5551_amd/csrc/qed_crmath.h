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

__device__ __noinline__ double cr_exp(double x) {
  if (!(x < 709.0)) return x != x ? x : (x > 709.782712893384 ? INFINITY : exp(x));
  if (!(x > -700.0)) return exp(x);  // results near the subnormal range are left to the library
  const dd e = exp_dd(x);
  return e.hi + e.lo;
}

__device__ __noinline__ double cr_log(double x) {
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
__device__ __noinline__ void cr_sincos(double x, double* sn, double* cs) {
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
__device__ __noinline__ double cr_sinq(double x, int qs) {
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

__device__ inline double cr_sin(double x) { return cr_sinq(x, 0); }
__device__ inline double cr_cos(double x) { return cr_sinq(x, 1); }

}  // namespace qedk
