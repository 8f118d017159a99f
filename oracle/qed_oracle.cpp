// Oracle for the QED Monte-Carlo emission step of Ridgers et al., "Modelling
// gamma-ray photon emission and pair production in high-intensity laser-matter
// interactions" (arXiv:1311.5551).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, FP64 CPU statement of
// what the GPU path computes.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the product library never
// links, calls or reads anything here, and nothing here is taken from the
// product library.  Compiled with -O2 -ffp-contract=off, no fast-math.
//
// Structure (paper order):
//   1. quantum synchrotron function F(eta, chi)           -- Appendix A
//   2. h(eta), g(eta), the 1e-9 energy cut-off, P_chi     -- Appendix A, Sec. 3
//   3. T_pm(chi), p_f(f, chi), k(chi), P_f                -- Appendix B, Sec. 3
//   4. Philox4x64-10 counter-based generator (Salmon et al., SC'11)
//   5. fields, Boris push, optical-depth Monte-Carlo step -- Sec. 3, Sec. 3.2
//   6. energy ledger                                      -- Sec. 3.1, Table 2
//
// Code units (a reading, shared by both sides of the parity contract):
//   t' = w t with w = 2 pi c / lambda_L;  x' = w x / c;  u = p/(m c);
//   E' = E/E_s;  B' = cB/E_s;  photon momentum k = p_gamma/(m c), energy |k|.
//   kappa = m c^2/(hbar w) = lambda_L/lambda_c with lambda_c = h/(m c).
//   Lorentz force  du/dt' = q kappa (E' + u/gamma x B').
//   Photon rate (eq. 2)  lambda'_gamma = (sqrt(3) alpha kappa / 2 pi) (eta/gamma) h(eta).
//   Pair rate   (eq. 3)  lambda'_pm    = alpha kappa chi T(chi) / |k|.
//
// Parity unpinned: nothing.  Every function below is pinned by a test in
// tests/test_oracle_*.py against closed forms, the paper's printed numbers,
// an independent library, or brute force.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ----------------------------------------------------------------------------
// physical constants (CODATA 2018)
// ----------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double kAlpha = 7.2973525693e-3;          // fine-structure constant
constexpr double kLambdaCompton = 2.42631023867e-12; // h/(m_e c), metres

// ----------------------------------------------------------------------------
// quadrature: Gauss-Legendre nodes by Newton iteration on P_n, and adaptive
// bisection that accepts a panel when the n-point rule on the panel and the sum
// over its two halves agree within tolerance.
// ----------------------------------------------------------------------------
struct GaussLegendre {
  int n;
  double x[24];
  double w[24];
};

GaussLegendre make_gauss_legendre(int n) {
  GaussLegendre r;
  r.n = n;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 200; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // derivative at the converged node
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= n; ++k) {
      double p2 = p1;
      p1 = p0;
      p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    dp = n * (z * p0 - p1) / (z * z - 1.0);
    r.x[i] = -z;
    r.x[n - 1 - i] = z;
    r.w[i] = r.w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return r;
}

const GaussLegendre& gl10() {
  static const GaussLegendre r = make_gauss_legendre(10);
  return r;
}

template <class Fn>
double gl_panel(const Fn& f, double a, double b) {
  const GaussLegendre& r = gl10();
  const double c = 0.5 * (a + b), hw = 0.5 * (b - a);
  double s = 0.0;
  for (int i = 0; i < r.n; ++i) s += r.w[i] * f(c + hw * r.x[i]);
  return s * hw;
}

// Accept a panel when the two estimates agree to within the panel's share of the
// tolerance, or to within rounding noise of the panel's value (the floor keeps the
// bisection finite when the requested tolerance is below what FP64 can resolve).
template <class Fn>
double adapt(const Fn& f, double a, double b, double whole, double tol_per_width, int depth) {
  const double m = 0.5 * (a + b);
  const double l = gl_panel(f, a, m), r = gl_panel(f, m, b);
  const double diff = std::fabs(l + r - whole);
  const double floor_ = 32.0 * 2.220446049250313e-16 * (std::fabs(l) + std::fabs(r));
  if (depth <= 0 || diff <= tol_per_width * (b - a) || diff <= floor_) return l + r;
  return adapt(f, a, m, l, tol_per_width, depth - 1) + adapt(f, m, b, r, tol_per_width, depth - 1);
}

// integral of f over [a, b] to relative tolerance rel (of the whole integral) plus an
// absolute tolerance abs_tol (needed where the integral is a small piece of a larger
// total, e.g. one segment of a cumulative table near the cut-off of the spectrum)
template <class Fn>
double integrate(const Fn& f, double a, double b, double rel, int n0 = 8, double abs_tol = 0.0) {
  if (!(b > a)) return 0.0;
  std::vector<double> part(n0);
  double est = 0.0;
  const double w = (b - a) / n0;
  for (int i = 0; i < n0; ++i) {
    part[i] = gl_panel(f, a + i * w, a + (i + 1) * w);
    est += std::fabs(part[i]);
  }
  const double tol_per_width = (rel * est + abs_tol) / (b - a) + 1e-300;
  double s = 0.0;
  for (int i = 0; i < n0; ++i) s += adapt(f, a + i * w, a + (i + 1) * w, part[i], tol_per_width, 40);
  return s;
}

// ----------------------------------------------------------------------------
// 1. Bessel functions and the quantum synchrotron function F(eta, chi)
// ----------------------------------------------------------------------------

// K_nu(y): modified Bessel function of the second kind (library primitive).
double bessel_k(double nu, double y) {
  if (y > 700.0) return 0.0;
  return std::cyl_bessel_k(nu, y);
}

// int_y^inf K_nu(t) dt, from K_nu(t) = int_0^inf exp(-t cosh s) cosh(nu s) ds
// integrated over t under the integral sign:
//   int_y^inf K_nu = exp(-y) int_0^inf exp(-2 y sinh^2(s/2)) cosh(nu s) / cosh(s) ds,
// (cosh s - 1 = 2 sinh^2(s/2)), truncated where the exponent passes -750.
double bessel_k_tail(double nu, double y) {
  if (y > 700.0) return 0.0;
  const double smax = std::acosh(1.0 + 750.0 / y);
  auto f = [&](double s) {
    const double sh = std::sinh(0.5 * s);
    return std::exp(-2.0 * y * sh * sh) * std::cosh(nu * s) / std::cosh(s);
  };
  return std::exp(-y) * integrate(f, 0.0, smax, 1e-15, 4);
}

// Appendix A: F(eta, chi) = (4 chi^2/eta^2) y K_{2/3}(y) + (1 - 2chi/eta) y int_y^inf K_{5/3},
// y = 4 chi / [3 eta (eta - 2 chi)], and F = 0 for chi >= eta/2.
// Written in xi = 2 chi/eta and 1 - xi (passed separately so that callers near the
// top of the spectrum can supply 1 - xi without cancellation): y = 2 xi / [3 eta (1 - xi)].
double synch_F_xi(double eta, double xi, double omxi) {
  if (!(xi > 0.0) || !(omxi > 0.0)) return 0.0;
  const double y = 2.0 * xi / (3.0 * eta * omxi);
  if (y > 700.0) return 0.0;
  return xi * xi * y * bessel_k(2.0 / 3.0, y) + omxi * y * bessel_k_tail(5.0 / 3.0, y);
}

double synch_F(double eta, double chi) {
  if (!(chi > 0.0) || !(chi < 0.5 * eta)) return 0.0;
  return synch_F_xi(eta, 2.0 * chi / eta, (eta - 2.0 * chi) / eta);
}

// F at s = ln chi, with d = s - ln(eta/2) <= 0: xi = e^d and 1 - xi = -expm1(d)
double synch_F_s(double eta, double s, double stop) {
  const double d = s - stop;
  if (!(d < 0.0)) return 0.0;
  return synch_F_xi(eta, std::exp(d), -std::expm1(d));
}

// The integrals below run over s = ln chi from s0 = ln(eta/2) - kTailSpan up to
// ln(eta/2).  Below s0 the spectrum follows its small-chi power law F ~ chi^{1/3}
// (Appendix A, classical limit), so
//   int_0^{chi0} F/chi dchi = 3 F(chi0)    and    int_0^{chi0} F dchi = (3/4) chi0 F(chi0),
// with relative error O(y0^{2/3}) < 1e-20 at this span.
constexpr double kTailSpan = 80.0;

// number integral int_{chi_a}^{chi_b} F/chi dchi over s in [sa, sb]
double number_integral(double eta, double sa, double sb, double abs_tol = 0.0) {
  const double stop = std::log(0.5 * eta);
  auto f = [&](double s) { return synch_F_s(eta, s, stop); };
  return integrate(f, sa, sb, 1e-13, 2, abs_tol);
}

// energy integral int F dchi over s in [sa, sb]
double energy_integral(double eta, double sa, double sb) {
  const double stop = std::log(0.5 * eta);
  auto f = [&](double s) { return synch_F_s(eta, s, stop) * std::exp(s); };
  return integrate(f, sa, sb, 1e-13, 8);
}

// Appendix A: h(eta) = int_0^{eta/2} F/chi dchi
double synch_h(double eta) {
  const double stop = std::log(0.5 * eta), s0 = stop - kTailSpan;
  return 3.0 * synch_F_s(eta, s0, stop) + number_integral(eta, s0, stop);
}

// int_0^{chi} F dchi' with chi = exp(s)
double energy_below(double eta, double s) {
  const double stop = std::log(0.5 * eta), s0 = stop - kTailSpan;
  return 0.75 * std::exp(s0) * synch_F_s(eta, s0, stop) + energy_integral(eta, s0, std::min(s, stop));
}

// Appendix A: g(eta) = (3 sqrt3 / 2 pi eta^2) int_0^{eta/2} F dchi
double synch_g(double eta) {
  return 3.0 * std::sqrt(3.0) / (2.0 * kPi * eta * eta) * energy_below(eta, std::log(0.5 * eta));
}

// Section 3: the table is cut off at chi_min such that the photons ignored below it
// carry a fraction `frac` of the spectrum's energy: int_0^{chi_min} F = frac int_0^{eta/2} F.
// Safeguarded Newton iteration in s = ln chi (d/ds of the energy integral is chi F).
double cutoff_chi(double eta, double frac) {
  const double stop = std::log(0.5 * eta);
  const double target = frac * energy_below(eta, stop);
  double lo = stop - kTailSpan, hi = stop;
  // starting point from the power law: int_0^chi F = (3/4) chi F(chi) at small chi
  double s = stop - 10.0;
  for (int it = 0; it < 200; ++it) {
    const double approx = 0.75 * std::exp(s) * synch_F_s(eta, s, stop);
    if (approx > target) hi = s; else lo = s;
    if (hi - lo < 1e-3) break;
    s = 0.5 * (lo + hi);
  }
  lo = stop - kTailSpan;
  hi = stop;
  for (int it = 0; it < 100; ++it) {
    const double chi = std::exp(s);
    const double G = energy_below(eta, s) - target;
    if (G > 0) hi = std::min(hi, s); else lo = std::max(lo, s);
    const double dG = chi * synch_F_s(eta, s, stop);
    double next = s - G / dG;
    if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    const double step = next - s;
    s = next;
    if (std::fabs(step) < 1e-15 * std::fabs(s) + 1e-300) break;
  }
  return std::exp(s);
}

// ----------------------------------------------------------------------------
// 3. pair production: T_pm(chi), p_f(f, chi), k(chi)   (Appendix B)
// ----------------------------------------------------------------------------

// T_pm(chi) ~= 0.16 K_{1/3}^2(2/(3 chi)) / chi
double pair_T(double chi) {
  if (!(chi > 0.0)) return 0.0;
  const double k = bessel_k(1.0 / 3.0, 2.0 / (3.0 * chi));
  return 0.16 * k * k / chi;
}

// unnormalised p_f: [2 + f(1-f)] / [f(1-f)] K_{2/3}(1 / (3 chi f(1-f)))
double pair_split_unnorm(double f, double chi) {
  if (!(f > 0.0) || !(f < 1.0)) return 0.0;
  const double g = f * (1.0 - f);
  return (2.0 + g) / g * bessel_k(2.0 / 3.0, 1.0 / (3.0 * chi * g));
}

double pair_split_integral(double chi, double fa, double fb, double abs_tol = 0.0) {
  auto q = [&](double f) { return pair_split_unnorm(f, chi); };
  return integrate(q, fa, fb, 1e-13, 2, abs_tol);
}

// k(chi) = int_0^1 of the unnormalised p_f
double pair_k(double chi) {
  // split at f = 1/2 so that each half integrates a one-sided feature
  return pair_split_integral(chi, 0.0, 0.5) + pair_split_integral(chi, 0.5, 1.0);
}

// ----------------------------------------------------------------------------
// 4. Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 64x64->128
// multiplies with the published multipliers and Weyl key increments.
// ----------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ULL;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ULL;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73BULL;

void philox4x64_10(const uint64_t in[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const unsigned __int128 p0 = (unsigned __int128)kPhiloxM0 * c0;
    const unsigned __int128 p1 = (unsigned __int128)kPhiloxM1 * c2;
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// open-interval uniform from the top 53 bits of a 64-bit word: (m + 1/2) 2^-53
double unit_open(uint64_t r) { return ((double)(r >> 11) + 0.5) * 0x1.0p-53; }

// Section 3: the optical depth at which a particle next reacts, from P = 1 - exp(-tau)
// with P uniform: tau = -ln(1 - P), and 1 - P is itself uniform on (0, 1).
double cr_log(double x);  // correctly rounded natural log, defined below
double optical_depth_draw(uint64_t r) { return -cr_log(unit_open(r)); }

// ----------------------------------------------------------------------------
// Correctly rounded exp, log, sin, cos for the Monte-Carlo step.  Each is evaluated in
// double-double arithmetic (Dekker's exact sum and product splits; ~2^-100 relative) and
// rounded once, which gives the correctly rounded double except within ~2^-100 of a
// rounding midpoint.  Two implementations that both round correctly agree bit for bit,
// whatever their algorithms.
//   exp: x = k ln2 + r (ln2 in three parts), e^r = sum r^n/n! summed until negligible.
//   log: x = m 2^e, log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1)/(m + 1).
//   sin, cos: x = k pi/2 + r (pi/2 in three parts), Taylor series of sin r and cos r.
// ----------------------------------------------------------------------------
struct DD {
  double hi, lo;
};
DD dd_norm(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return {s, b - (s - a)};
}
DD dd_sum(double a, double b) {
  const double s = a + b, v = s - a;
  return {s, (a - (s - v)) + (b - v)};
}
DD dd_prod(double a, double b) {
  const double p = a * b;
  return {p, std::fma(a, b, -p)};
}
DD operator+(DD a, DD b) {
  DD s = dd_sum(a.hi, b.hi);
  DD t = dd_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_norm(s.hi, s.lo);
  s.lo += t.lo;
  return dd_norm(s.hi, s.lo);
}
DD operator*(DD a, DD b) {
  DD p = dd_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_norm(p.hi, p.lo);
}
DD operator*(DD a, double b) {
  DD p = dd_prod(a.hi, b);
  p.lo += a.lo * b;
  return dd_norm(p.hi, p.lo);
}
DD operator/(DD a, double b) {
  const double q1 = a.hi / b;
  const DD p = dd_prod(q1, b);
  const double rem = ((a.hi - p.hi) - p.lo) + a.lo;
  return dd_norm(q1, rem / b);
}
DD operator/(DD a, DD b) {
  const double q1 = a.hi / b.hi;
  const DD r = a + DD{-(b * q1).hi, -(b * q1).lo};
  const double q2 = r.hi / b.hi;
  const DD r2 = r + DD{-(b * q2).hi, -(b * q2).lo};
  const double q3 = r2.hi / b.hi;
  return dd_norm(q1, q2) + DD{q3, 0.0};
}
double dd_round(DD a) { return a.hi + a.lo; }

// ln 2 and pi/2 split into a short leading part (exact multiples) and two tails
constexpr double kLn2P1 = 0x1.62e42fefa3800p-1, kLn2P2 = 0x1.ef35793c76730p-45, kLn2P3 = 0x1.f97b57a079a19p-103;
constexpr double kHalfPiP1 = 0x1.921fb54400000p+0, kHalfPiP2 = 0x1.0b4611a626331p-34,
                 kHalfPiP3 = 0x1.1701b839a2520p-88;

DD reduce(double x, double k, double p1, double p2, double p3) {
  DD r = DD{x - k * p1, 0.0} + dd_prod(-k, p2);
  return dd_norm(r.hi, r.lo - k * p3);
}

double cr_exp(double x) {
  if (!(x < 709.0) || !(x > -700.0)) return std::exp(x);
  const double k = std::nearbyint(x / 0.6931471805599453);
  const DD r = reduce(x, k, kLn2P1, kLn2P2, kLn2P3);
  DD sum = {1.0, 0.0}, term = {1.0, 0.0};
  for (int n = 1; n < 40; ++n) {
    term = term * r / (double)n;
    sum = sum + term;
    if (std::fabs(term.hi) < 1e-36) break;
  }
  return std::ldexp(dd_round(sum), (int)k);
}

double cr_log(double x) {
  if (!(x > 0.0) || !std::isfinite(x)) return std::log(x);
  int e;
  double m = std::frexp(x, &e);
  if (m < 0.7071067811865476) {
    m *= 2.0;
    --e;
  }
  // s = (m - 1)/(m + 1): m - 1 is exact (Sterbenz), m + 1 as a double-double
  const DD s = DD{m - 1.0, 0.0} / dd_sum(m, 1.0);
  const DD s2 = s * s;
  DD sum = s, pw = s;
  for (int n = 3; n < 200; n += 2) {
    pw = pw * s2;
    const DD t = pw / (double)n;
    sum = sum + t;
    if (std::fabs(t.hi) < 1e-36 * std::fabs(sum.hi) + 1e-300) break;
  }
  const DD ln2 = DD{0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56};
  return dd_round(ln2 * (double)e + sum * 2.0);
}

void cr_sincos(double x, double* sn, double* cs) {
  if (!(std::fabs(x) < 1048576.0)) {
    *sn = std::sin(x);
    *cs = std::cos(x);
    return;
  }
  const double k = std::nearbyint(x / 1.5707963267948966);
  const DD r = reduce(x, k, kHalfPiP1, kHalfPiP2, kHalfPiP3);
  const DD r2 = r * r;
  DD sn_sum = r, cs_sum = {1.0, 0.0}, ts = r, tc = {1.0, 0.0};
  for (int n = 1; n < 30; ++n) {
    // terms (-1)^n r^(2n+1)/(2n+1)! and (-1)^n r^(2n)/(2n)!
    tc = tc * r2 / (double)((2 * n - 1) * (2 * n));
    ts = ts * r2 / (double)((2 * n) * (2 * n + 1));
    tc = DD{-tc.hi, -tc.lo};
    ts = DD{-ts.hi, -ts.lo};
    cs_sum = cs_sum + tc;
    sn_sum = sn_sum + ts;
    if (std::fabs(tc.hi) < 1e-36 && std::fabs(ts.hi) < 1e-36 * std::fabs(r.hi)) break;
  }
  const double sv = dd_round(sn_sum), cv = dd_round(cs_sum);
  long q = (long)std::fmod(k, 4.0);
  if (q < 0) q += 4;
  *sn = q == 0 ? sv : q == 1 ? cv : q == 2 ? -sv : -cv;
  *cs = q == 0 ? cv : q == 1 ? -sv : q == 2 ? -cv : sv;
}

double cr_sin(double x) {
  double s, c;
  cr_sincos(x, &s, &c);
  return s;
}

double cr_cos(double x) {
  double s, c;
  cr_sincos(x, &s, &c);
  return c;
}

}  // namespace

// ============================================================================
// C interface used by the Python test wrapper (oracle/__init__.py)
// ============================================================================
extern "C" {

// ---- special functions (for pins) ----
double oracle_bessel_k(double nu, double y) { return bessel_k(nu, y); }
double oracle_bessel_k_tail(double nu, double y) { return bessel_k_tail(nu, y); }
double oracle_F(double eta, double chi) { return synch_F(eta, chi); }
double oracle_h(double eta) { return synch_h(eta); }
double oracle_g(double eta) { return synch_g(eta); }
double oracle_energy_below(double eta, double chi) { return energy_below(eta, std::log(chi)); }
double oracle_cutoff_chi(double eta, double frac) { return cutoff_chi(eta, frac); }
double oracle_T(double chi) { return pair_T(chi); }
double oracle_pair_k(double chi) { return pair_k(chi); }
double oracle_pf(double f, double chi) { return pair_split_unnorm(f, chi) / pair_k(chi); }
// Cumulative emission number int_0^{chi_i} F/chi' dchi' (Appendix A) at n ascending chi_i,
// integrated piece by piece between them (chi above eta/2 gives h(eta)).
void oracle_number_cumulative(double eta, const double* chi, int n, double* out) {
  const double stop = std::log(0.5 * eta), s0 = stop - kTailSpan;
  double acc = 0.0, s_prev = s0;
  bool started = false;
  for (int i = 0; i < n; ++i) {
    const double s = chi[i] > 0.0 ? std::min(std::log(chi[i]), stop) : -INFINITY;
    if (s <= s0) {  // below the quadrature span: the small-chi power law, int_0^chi F/chi = 3 F(chi)
      out[i] = s == -INFINITY ? 0.0 : 3.0 * synch_F_s(eta, s, stop);
      continue;
    }
    if (!started) {
      acc = 3.0 * synch_F_s(eta, s0, stop);
      s_prev = s0;
      started = true;
    }
    // pieces are resolved to 1e-16 of h (a piece in the exponential tail has no relative scale)
    if (s > s_prev) acc += number_integral(eta, s_prev, s, 1e-16 * synch_h(eta));
    s_prev = std::max(s_prev, s);
    out[i] = acc;
  }
}
// Cumulative normalised energy split int_0^{f_i} p_f(f', chi) df' (Appendix B) at n ascending
// f_i in [0, 1].
void oracle_pf_cumulative(double chi, const double* f, int n, double* out) {
  const double k = pair_k(chi);
  if (!(k > 0.0)) {  // chi so small that p_f underflows everywhere (no pairs are made there)
    for (int i = 0; i < n; ++i) out[i] = 0.0;
    return;
  }
  double acc = 0.0, prev = 0.0;
  for (int i = 0; i < n; ++i) {
    const double fi = std::min(std::max(f[i], 0.0), 1.0);
    if (fi > prev) {
      // the integrand has one-sided features at both ends: split at 1/2
      const double tol = 1e-16 * k;  // pieces where p_f is exponentially small have no relative scale
      if (prev < 0.5 && fi > 0.5)
        acc += pair_split_integral(chi, prev, 0.5, tol) + pair_split_integral(chi, 0.5, fi, tol);
      else
        acc += pair_split_integral(chi, prev, fi, tol);
      prev = fi;
    }
    out[i] = acc / k;
  }
}
void oracle_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out) { philox4x64_10(ctr, key, out); }
double oracle_cr_exp(double x) { return cr_exp(x); }
double oracle_cr_log(double x) { return cr_log(x); }
double oracle_cr_sin(double x) { return cr_sin(x); }
double oracle_cr_cos(double x) { return cr_cos(x); }
void oracle_gauss_legendre(int n, double* x, double* w) {
  GaussLegendre r = make_gauss_legendre(n);
  for (int i = 0; i < n; ++i) {
    x[i] = r.x[i];
    w[i] = r.w[i];
  }
}

// ---- tables (Section 3: h, T_pm, P_chi, P_f) ----
typedef struct {
  int32_t n_eta;
  double eta_min, eta_max;
  int32_t n_chi;
  double cutoff_energy_frac;
  int32_t n_chi_pair;
  double chi_pair_min, chi_pair_max;
  int32_t n_f;
} oracle_table_params;

// Caller-allocated outputs:
//   h[n_eta], lnchi_min[n_eta], dlnchi[n_eta], P_chi[n_eta*n_chi],
//   T[n_chi_pair], f_grid[n_f], P_f[n_chi_pair*n_f], k_norm[n_chi_pair], and g[n_eta]
//   (may be NULL): the quantum reduction g(eta_i) of the radiated power (Appendix A).
// Row i of P_chi holds P(eta_i, chi_ij) on ln chi_ij = lnchi_min[i] + j dlnchi[i],
// from chi_min (the 1e-9 energy cut) to eta_i/2; P(eta_i, chi_min) is the share of
// emissions below the cut and the last column is exactly 1.
int oracle_build_tables(const oracle_table_params* p, double* h, double* lnchi_min, double* dlnchi,
                        double* P_chi, double* T, double* f_grid, double* P_f, double* k_norm, double* g) {
  const int ne = p->n_eta, nc = p->n_chi, np = p->n_chi_pair, nf = p->n_f;
  if (ne < 2 || nc < 2 || np < 2 || nf < 3) return -1;
  const double le0 = std::log(p->eta_min), le1 = std::log(p->eta_max);
  const double dle = (le1 - le0) / (ne - 1);

#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < ne; ++i) {
    const double eta = std::exp(le0 + i * dle);
    const double stop = std::log(0.5 * eta);
    const double s0 = stop - kTailSpan;
    const double chimin = cutoff_chi(eta, p->cutoff_energy_frac);
    const double smin = std::log(chimin);
    const double ds = (stop - smin) / (nc - 1);
    std::vector<double> cum(nc);
    // segments are resolved to 1e-17 of the row total (well below the FP64 spacing of P)
    const double seg_tol = 1e-17 * synch_h(eta);
    // number of emissions below the cut: power-law tail below s0 plus [s0, smin]
    cum[0] = 3.0 * synch_F_s(eta, s0, stop) + number_integral(eta, s0, smin);
    for (int j = 1; j < nc; ++j) {
      const double sa = smin + (j - 1) * ds;
      const double sb = (j == nc - 1) ? stop : smin + j * ds;
      cum[j] = cum[j - 1] + number_integral(eta, sa, sb, seg_tol);
    }
    const double hval = cum[nc - 1];
    h[i] = hval;
    if (g) g[i] = synch_g(eta);
    lnchi_min[i] = smin;
    dlnchi[i] = ds;
    for (int j = 0; j < nc - 1; ++j) P_chi[(size_t)i * nc + j] = cum[j] / hval;
    P_chi[(size_t)i * nc + nc - 1] = 1.0;
  }

  // f grid: f_l = sin^2(pi l / (2 (n_f - 1))), clustered at f = 0 and f = 1
  for (int l = 0; l < nf; ++l) {
    const double s = std::sin(kPi * l / (2.0 * (nf - 1)));
    f_grid[l] = s * s;
  }
  f_grid[0] = 0.0;
  f_grid[nf - 1] = 1.0;

  const double lc0 = std::log(p->chi_pair_min), lc1 = std::log(p->chi_pair_max);
  const double dlc = (lc1 - lc0) / (np - 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < np; ++k) {
    const double chi = std::exp(lc0 + k * dlc);
    T[k] = pair_T(chi);
    std::vector<double> cum(nf);
    cum[0] = 0.0;
    const double seg_tol = 1e-17 * pair_k(chi);
    for (int l = 1; l < nf; ++l) cum[l] = cum[l - 1] + pair_split_integral(chi, f_grid[l - 1], f_grid[l], seg_tol);
    const double kn = cum[nf - 1];
    k_norm[k] = kn;
    for (int l = 0; l < nf - 1; ++l) P_f[(size_t)k * nf + l] = cum[l] / kn;
    P_f[(size_t)k * nf] = 0.0;
    P_f[(size_t)k * nf + nf - 1] = 1.0;
  }
  return 0;
}

}  // extern "C"

// ============================================================================
// 5. the Monte-Carlo step (Section 3, Section 3.2)
// ============================================================================
namespace {

enum : uint32_t {
  FLAG_EMIT = 1u,
  FLAG_PAIRS = 2u,
  FLAG_PROPAGATE = 4u,
  FLAG_RR_QUANTUM = 8u,    // continuous radiation reaction with the quantum reduction g(eta)
  FLAG_RR_CLASSICAL = 16u  // continuous radiation reaction with the classical power (g = 1)
};
enum : uint64_t { KIND_INIT = 0, KIND_EMIT = 1, KIND_PAIR = 2 };
enum : int32_t {
  FIELD_UNIFORM = 0,      // p[0..2] = E, p[3..5] = B
  FIELD_LP_PULSE = 1,     // p = {E0, Psi, psi0, phase}: E_y = B_z = E0 env(psi) cos(psi + phase)
  FIELD_CP_WAVE = 2,      // p = {E0, phase}: E = E0 (cos, sin) in (y, z), B = x_hat cross E
  FIELD_CP_STANDING = 3,  // p = {E0}: two counter-propagating circularly polarised waves
  FIELD_GRID_CP_STANDING = 4,  // same source sampled on a 2-D Yee grid (FP32) and gathered (CIC)
  FIELD_GRID_FDTD = 5  // p = {Q}: the fields of a 2-D Yee grid (FP64) advanced by Maxwell's equations
                       // with the current of the leptons (charge q Q per macro-particle); gathered (CIC)
};

struct Tables {
  int n_eta;
  double le0, dle;
  const double* h;
  const double* g;  // may be null when no step uses FLAG_RR_QUANTUM
  int n_chi;
  const double* lnchi_min;
  const double* dlnchi;
  const double* P;
  int n_cp;
  double lc0, dlc;
  const double* T;
  int n_f;
  const double* f;
  const double* Pf;
};

struct Grid {
  int nx, ny;
  double dx, dy, x0, y0;
};

struct Config {
  int32_t field;
  double fp[16];
  Grid grid;
  int32_t dims;
  double dt, t0;
  int64_t step0, n_steps;
  uint64_t seed, instance;
  uint32_t flags;
  double kappa, a_gamma, a_pair, a_rr;
  double* fdtd = nullptr;  // FIELD_GRID_FDTD: 9 planes of ny x nx nodes, Ex Ey Ez Bx By Bz Jx Jy Jz
};

struct Vec3 {
  double x, y, z;
};
inline Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 operator*(double s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline Vec3 cross(Vec3 a, Vec3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// --- analytic sources -----------------------------------------------------
void cp_standing(double E0, double x, double t, double out[6]) {
  // E_y = 2E0 cos t cos x, E_z = 2E0 sin t cos x, B_y = 2E0 cos t sin x, B_z = 2E0 sin t sin x
  const double ct = cr_cos(t), st = cr_sin(t), cx = cr_cos(x), sx = cr_sin(x);
  out[0] = 0.0;
  out[1] = 2.0 * E0 * ct * cx;
  out[2] = 2.0 * E0 * st * cx;
  out[3] = 0.0;
  out[4] = 2.0 * E0 * ct * sx;
  out[5] = 2.0 * E0 * st * sx;
}

// Yee staggering of the six components on the (x, y) grid, in cell units:
// Ex(i+1/2, j), Ey(i, j+1/2), Ez(i, j), Bx(i, j+1/2), By(i+1/2, j), Bz(i+1/2, j+1/2)
constexpr double kYeeOx[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
constexpr double kYeeOy[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};

// value stored at node (i, j) of component c: the analytic source in FP64 rounded to FP32
double grid_node(const Config& c, int comp, int64_t i, int64_t j, double t) {
  const double xn = c.grid.x0 + ((double)i + kYeeOx[comp]) * c.grid.dx;
  double f[6];
  cp_standing(c.fp[0], xn, t, f);
  (void)j;  // the standing wave does not depend on y
  return (double)(float)f[comp];
}

int64_t wrap(int64_t i, int n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

// first-order (cloud-in-cell) gather of component comp at (x, y): bilinear weights over the four
// nodes around the point on that component's staggered grid; node(i, j) gives a node's value
template <class NodeFn>
double cic_gather(const Grid& g, int comp, double x, double y, NodeFn node) {
  const double gx = (x - g.x0) / g.dx - kYeeOx[comp];
  const double gy = (y - g.y0) / g.dy - kYeeOy[comp];
  const double fx = std::floor(gx), fy = std::floor(gy);
  const double wx = gx - fx, wy = gy - fy;
  const int64_t i0 = (int64_t)fx, j0 = (int64_t)fy;
  const int64_t ia = wrap(i0, g.nx), ib = wrap(i0 + 1, g.nx);
  const int64_t ja = wrap(j0, g.ny), jb = wrap(j0 + 1, g.ny);
  return (1.0 - wx) * (1.0 - wy) * node(ia, ja) + wx * (1.0 - wy) * node(ib, ja) + (1.0 - wx) * wy * node(ia, jb) +
         wx * wy * node(ib, jb);
}

// --- field feedback (Sec. 3.2: charge and current of the macro-particles on the grid, then
// Maxwell's equations for E and B).  Code units: dE/dt = curl B - J, dB/dt = -curl E, and
// div E = rho; a macro-particle of charge Q (per unit length along z) has the density
// Q S_x S_y / (dx dy) with the first-order (cloud-in-cell) shape S of the gather.

// Current of one macro-particle of charge Q moving in one step from (x0, y0) to (x1, y1), less
// than a cell in each direction, with out-of-plane velocity vz: the charge-conserving split of
// Esirkepov (Comput. Phys. Commun. 135, 144, 2001) for first-order shapes in 2-D.  With the
// old and new shape factors S0, S1 of the (up to) three nodes per direction the particle
// touches and D = S1 - S0:
//   Wx = Dx (S0y + Dy/2),   Wy = Dy (S0x + Dx/2),
//   Wz = S0x S0y + Dx S0y / 2 + S0x Dy / 2 + Dx Dy / 3,
//   Jx(i+1/2, j) = -Q/(dy dt) sum_{i' <= i} Wx(i', j),   Jy(i, j+1/2) = -Q/(dx dt) sum_{j' <= j} Wy(i, j'),
//   Jz(i, j) = Q vz Wz(i, j) / (dx dy),
// so that (rho1 - rho0)/dt + (Jx(i+1/2) - Jx(i-1/2))/dx + (Jy(j+1/2) - Jy(j-1/2))/dy = 0 node by
// node.  J holds the planes Jx, Jy, Jz (ny x nx each, Jx at Ex's nodes, Jy at Ey's, Jz at Ez's).
void deposit_current(const Grid& g, double Q, double dt, double x0, double y0, double x1, double y1, double vz,
                     double* J) {
  const double gx0 = (x0 - g.x0) / g.dx, gy0 = (y0 - g.y0) / g.dy;
  const double gx1 = (x1 - g.x0) / g.dx, gy1 = (y1 - g.y0) / g.dy;
  const double bx = std::floor(std::min(gx0, gx1)), by = std::floor(std::min(gy0, gy1));
  const int64_t I = (int64_t)bx, Jn = (int64_t)by;
  double S0x[3], S1x[3], S0y[3], S1y[3];
  for (int a = 0; a < 3; ++a) {
    S0x[a] = std::max(0.0, 1.0 - std::fabs(gx0 - (bx + a)));
    S1x[a] = std::max(0.0, 1.0 - std::fabs(gx1 - (bx + a)));
    S0y[a] = std::max(0.0, 1.0 - std::fabs(gy0 - (by + a)));
    S1y[a] = std::max(0.0, 1.0 - std::fabs(gy1 - (by + a)));
  }
  const int64_t plane = (int64_t)g.nx * g.ny;
  const double cx = -Q / (g.dy * dt), cy = -Q / (g.dx * dt), cz = Q * vz / (g.dx * g.dy);
  for (int b = 0; b < 3; ++b) {
    const int64_t j = wrap(Jn + b, g.ny);
    double run = 0.0;
    for (int a = 0; a < 3; ++a) {
      const int64_t i = wrap(I + a, g.nx);
      const double dxa = S1x[a] - S0x[a], dyb = S1y[b] - S0y[b];
      run += dxa * (S0y[b] + 0.5 * dyb);
      J[j * g.nx + i] += cx * run;
      const double wz = S0x[a] * S0y[b] + 0.5 * dxa * S0y[b] + 0.5 * S0x[a] * dyb + dxa * dyb / 3.0;
      J[2 * plane + j * g.nx + i] += cz * wz;
    }
  }
  for (int a = 0; a < 3; ++a) {
    const int64_t i = wrap(I + a, g.nx);
    double run = 0.0;
    for (int b = 0; b < 3; ++b) {
      const int64_t j = wrap(Jn + b, g.ny);
      const double dxa = S1x[a] - S0x[a], dyb = S1y[b] - S0y[b];
      run += dyb * (S0x[a] + 0.5 * dxa);
      J[plane + j * g.nx + i] += cy * run;
    }
  }
}

// One step of Maxwell's equations on the Yee grid (periodic), leapfrog in the form that keeps E
// and B at the same time level: B advanced half a step with E^n, E a full step with that B and
// the current J^{n+1/2}, B the second half step with E^{n+1}.  In cell indices (each component
// stored at its own staggered node, index (i, j)):
//   Bx(i,j) -= (dt/2) (Ez(i,j+1) - Ez(i,j))/dy
//   By(i,j) += (dt/2) (Ez(i+1,j) - Ez(i,j))/dx
//   Bz(i,j) -= (dt/2) ((Ey(i+1,j) - Ey(i,j))/dx - (Ex(i,j+1) - Ex(i,j))/dy)
//   Ex(i,j) += dt ((Bz(i,j) - Bz(i,j-1))/dy - Jx(i,j))
//   Ey(i,j) += dt (-(Bz(i,j) - Bz(i-1,j))/dx - Jy(i,j))
//   Ez(i,j) += dt ((By(i,j) - By(i-1,j))/dx - (Bx(i,j) - Bx(i,j-1))/dy - Jz(i,j))
// F holds the nine planes Ex Ey Ez Bx By Bz Jx Jy Jz.
void fdtd_half_b(const Grid& g, double dt, double* F) {
  const int64_t P = (int64_t)g.nx * g.ny;
  const double h = 0.5 * dt;
  std::vector<double> bx(P), by(P), bz(P);
  for (int64_t j = 0; j < g.ny; ++j)
    for (int64_t i = 0; i < g.nx; ++i) {
      const int64_t k = j * g.nx + i, ip = j * g.nx + wrap(i + 1, g.nx), jp = wrap(j + 1, g.ny) * g.nx + i;
      const double* Ex = F;
      const double* Ey = F + P;
      const double* Ez = F + 2 * P;
      bx[k] = F[3 * P + k] - h * ((Ez[jp] - Ez[k]) / g.dy);
      by[k] = F[4 * P + k] + h * ((Ez[ip] - Ez[k]) / g.dx);
      bz[k] = F[5 * P + k] - h * ((Ey[ip] - Ey[k]) / g.dx - (Ex[jp] - Ex[k]) / g.dy);
    }
  std::copy(bx.begin(), bx.end(), F + 3 * P);
  std::copy(by.begin(), by.end(), F + 4 * P);
  std::copy(bz.begin(), bz.end(), F + 5 * P);
}
void fdtd_full_e(const Grid& g, double dt, double* F) {
  const int64_t P = (int64_t)g.nx * g.ny;
  std::vector<double> ex(P), ey(P), ez(P);
  for (int64_t j = 0; j < g.ny; ++j)
    for (int64_t i = 0; i < g.nx; ++i) {
      const int64_t k = j * g.nx + i, im = j * g.nx + wrap(i - 1, g.nx), jm = wrap(j - 1, g.ny) * g.nx + i;
      const double* Bx = F + 3 * P;
      const double* By = F + 4 * P;
      const double* Bz = F + 5 * P;
      ex[k] = F[k] + dt * ((Bz[k] - Bz[jm]) / g.dy - F[6 * P + k]);
      ey[k] = F[P + k] + dt * (-(Bz[k] - Bz[im]) / g.dx - F[7 * P + k]);
      ez[k] = F[2 * P + k] + dt * ((By[k] - By[im]) / g.dx - (Bx[k] - Bx[jm]) / g.dy - F[8 * P + k]);
    }
  std::copy(ex.begin(), ex.end(), F);
  std::copy(ey.begin(), ey.end(), F + P);
  std::copy(ez.begin(), ez.end(), F + 2 * P);
}
void fdtd_step(const Grid& g, double dt, double* F) {
  fdtd_half_b(g, dt, F);
  fdtd_full_e(g, dt, F);
  fdtd_half_b(g, dt, F);
}

void fields_at(const Config& c, double x, double y, double z, double t, Vec3* E, Vec3* B) {
  double f[6] = {0, 0, 0, 0, 0, 0};
  switch (c.field) {
    case FIELD_UNIFORM:
      for (int k = 0; k < 6; ++k) f[k] = c.fp[k];
      break;
    case FIELD_LP_PULSE: {
      const double psi = t - x - c.fp[2];
      if (psi >= 0.0 && psi <= c.fp[1]) {
        const double s = cr_sin(kPi * psi / c.fp[1]);
        const double e = c.fp[0] * s * s * cr_cos(psi + c.fp[3]);
        f[1] = e;
        f[5] = e;
      }
      break;
    }
    case FIELD_CP_WAVE: {
      const double psi = t - x + c.fp[1];
      const double ey = c.fp[0] * cr_cos(psi), ez = c.fp[0] * cr_sin(psi);
      f[1] = ey;
      f[2] = ez;
      f[4] = -ez;
      f[5] = ey;
      break;
    }
    case FIELD_CP_STANDING:
      cp_standing(c.fp[0], x, t, f);
      break;
    case FIELD_GRID_CP_STANDING: {
      // first-order (cloud-in-cell) gather from each staggered component grid
      for (int comp = 0; comp < 6; ++comp)
        f[comp] = cic_gather(c.grid, comp, x, y, [&](int64_t i, int64_t j) { return grid_node(c, comp, i, j, t); });
      break;
    }
    case FIELD_GRID_FDTD: {
      // the same gather from the solver's grid as it stands at this step
      const int64_t plane = (int64_t)c.grid.nx * c.grid.ny;
      for (int comp = 0; comp < 6; ++comp)
        f[comp] = cic_gather(c.grid, comp, x, y,
                             [&](int64_t i, int64_t j) { return c.fdtd[comp * plane + j * c.grid.nx + i]; });
      break;
    }
    default:
      break;
  }
  (void)z;
  *E = {f[0], f[1], f[2]};
  *B = {f[3], f[4], f[5]};
}

// --- table look-ups (Section 3: linear interpolation in the look-up tables) -----

// h(eta): linear in value between nodes on a uniform ln(eta) grid; clamped to the end
// values outside [eta_min, eta_max] (above the range is counted).
double lookup_h(const Tables& tb, double eta, int64_t* range_hi) {
  const double s = (cr_log(eta) - tb.le0) / tb.dle;
  if (!(s > 0.0)) return tb.h[0];
  if (s >= tb.n_eta - 1) {
    ++*range_hi;
    return tb.h[tb.n_eta - 1];
  }
  const int i = (int)std::floor(s);
  const double w = s - i;
  return (1.0 - w) * tb.h[i] + w * tb.h[i + 1];
}

// g(eta): on the grid of h, interpolated and clamped the same way.
double lookup_g(const Tables& tb, double eta, int64_t* range_hi) {
  const double s = (cr_log(eta) - tb.le0) / tb.dle;
  if (!(s > 0.0)) return tb.g[0];
  if (s >= tb.n_eta - 1) {
    ++*range_hi;
    return tb.g[tb.n_eta - 1];
  }
  const int i = (int)std::floor(s);
  const double w = s - i;
  return (1.0 - w) * tb.g[i] + w * tb.g[i + 1];
}

// T(chi): as h, but zero below chi_pair_min where T < 1e-58.
double lookup_T(const Tables& tb, double chi, int64_t* range_hi) {
  if (!(chi > 0.0)) return 0.0;
  const double s = (cr_log(chi) - tb.lc0) / tb.dlc;
  if (s < 0.0) return 0.0;
  if (s >= tb.n_cp - 1) {
    ++*range_hi;
    return tb.T[tb.n_cp - 1];
  }
  const int k = (int)std::floor(s);
  const double w = s - k;
  return (1.0 - w) * tb.T[k] + w * tb.T[k + 1];
}

// Inverse of one tabulated cumulative row P[0..n-1] (non-decreasing, P[n-1] = 1):
// j is the largest index with P[j] < u, so that P[j] < u <= P[j+1]; `frac` is the
// position of u inside that segment, for linear interpolation of the abscissa.
int row_inverse(const double* P, int n, double u, double* frac) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (P[mid] < u) lo = mid; else hi = mid;
  }
  *frac = (u - P[lo]) / (P[hi] - P[lo]);
  return lo;
}

// Section 3: chi from the tabulated cumulative P_chi at the emitter's eta.
// Returns false when the draw falls below the low-energy cut-off in either row used.
bool sample_chi(const Tables& tb, double eta, double u, double* chi) {
  const double leta = cr_log(eta);
  const double s = (leta - tb.le0) / tb.dle;
  auto Q = [&](int r, double* q) {
    const double* P = tb.P + (size_t)r * tb.n_chi;
    if (u <= P[0]) return false;
    double fr;
    const int j = row_inverse(P, tb.n_chi, u, &fr);
    *q = tb.lnchi_min[r] + (j + fr) * tb.dlnchi[r];
    return true;
  };
  double lnchi;
  if (!(s > 0.0)) {
    // below the table: classical scaling chi ~ eta^2 at fixed cumulative probability
    double q0;
    if (!Q(0, &q0)) return false;
    lnchi = q0 + 2.0 * (leta - tb.le0);
  } else if (s >= tb.n_eta - 1) {
    // above the table: fixed photon energy fraction 2 chi / eta
    double q1;
    if (!Q(tb.n_eta - 1, &q1)) return false;
    lnchi = q1 + (leta - (tb.le0 + (tb.n_eta - 1) * tb.dle));
  } else {
    const int i = (int)std::floor(s);
    const double w = s - i;
    double qa, qb;
    const bool ok_a = Q(i, &qa);
    const bool ok_b = Q(i + 1, &qb);
    if (!ok_a || !ok_b) return false;
    lnchi = (1.0 - w) * qa + w * qb;
  }
  *chi = cr_exp(lnchi);
  return true;
}

// Section 3: the positron's energy fraction f from the tabulated P_f, by the same
// procedure: rows at the two nodes bracketing ln chi, linear in f inside a row,
// blended linearly in ln chi.
double sample_f(const Tables& tb, double chi, double u) {
  const double s = (cr_log(chi) - tb.lc0) / tb.dlc;
  auto frow = [&](int r) {
    double fr;
    const int j = row_inverse(tb.Pf + (size_t)r * tb.n_f, tb.n_f, u, &fr);
    return tb.f[j] + fr * (tb.f[j + 1] - tb.f[j]);
  };
  if (!(s > 0.0)) return frow(0);
  if (s >= tb.n_cp - 1) return frow(tb.n_cp - 1);
  const int k = (int)std::floor(s);
  const double w = s - k;
  return (1.0 - w) * frow(k) + w * frow(k + 1);
}

// --- particles and families ------------------------------------------------
struct Particle {
  double x, y, z, ux, uy, uz, tau;  // photons: x, y, z is the position at step `birth`
  uint64_t uid;
  int64_t birth;  // photons: step at whose start the photon sits at (x, y, z)
  int species;  // 0 electron, 1 positron, 2 photon
  double margin;  // smallest |tau| seen after a decrement (threshold-straddle flag)
  bool alive;
};

struct Tally {
  int64_t particle_steps = 0;  // particles advanced, one per particle per step
  double work = 0.0;       // sum of field work on leptons (Boris identity)
  double defect_emit = 0.0;
  double defect_pair = 0.0;
  double radiated = 0.0;   // energy removed by continuous radiation reaction
  int64_t n_emit = 0, n_null = 0, n_pair = 0, n_range = 0, n_nonfinite = 0;
};

void draw(const Config& c, uint64_t uid, int64_t step, uint64_t kind, uint64_t sub, uint64_t out[4]) {
  const uint64_t ctr[4] = {uid, (uint64_t)step, kind, sub};
  const uint64_t key[2] = {c.seed, c.instance};
  philox4x64_10(ctr, key, out);
}

double gamma_of(double ux, double uy, double uz) { return std::sqrt(1.0 + ux * ux + uy * uy + uz * uz); }

// eta = |F_{mu nu} p^nu| / (m c E_s) = sqrt(|gamma E + u x B|^2 - (u.E)^2) of a lepton with
// momentum u (gamma = g) in the fields E, B (Sec. 2.1, eq. 1)
double eta_of(Vec3 E, Vec3 B, Vec3 u, double g) {
  const Vec3 a = g * E + cross(u, B);
  const double ue = dot(u, E);
  return std::sqrt(std::max(0.0, dot(a, a) - ue * ue));
}

// chi = (eps/2) sqrt(|E + n x B|^2 - (n.E)^2) of a photon with momentum k = eps n (the chi of
// eq. 1, half the usual chi_gamma)
double chi_of(Vec3 E, Vec3 B, Vec3 nh, double eps) {
  const Vec3 a = E + cross(nh, B);
  const double ne = dot(nh, E);
  return 0.5 * eps * std::sqrt(std::max(0.0, dot(a, a) - ne * ne));
}

// one step of an electron (q = -1) or positron (q = +1); children are appended to `fam`.
// vz_push (optional) receives the z velocity u1z/gamma1 of the push (the one that moved it).
void step_lepton(Particle& p, const Config& c, const Tables& tb, int64_t n, std::vector<Particle>& fam,
                 Tally& tl, double* vz_push = nullptr) {
  const double t = c.t0 + (double)n * c.dt;
  Vec3 E, B;
  fields_at(c, p.x, p.y, p.z, t, &E, &B);
  const double q = (p.species == 0) ? -1.0 : 1.0;

  // Boris push (Section 3.2: the Lorentz push precedes the emission step)
  const Vec3 u0 = {p.ux, p.uy, p.uz};
  const double g0 = gamma_of(u0.x, u0.y, u0.z);
  const double hq = 0.5 * q * c.kappa * c.dt;
  const Vec3 um = u0 + hq * E;
  const double gm = std::sqrt(1.0 + dot(um, um));
  const Vec3 tv = (hq / gm) * B;
  const Vec3 sv = (2.0 / (1.0 + dot(tv, tv))) * tv;
  const Vec3 up = um + cross(um, tv);
  const Vec3 upl = um + cross(up, sv);
  const Vec3 u1 = upl + hq * E;
  const double g1 = std::sqrt(1.0 + dot(u1, u1));
  // energy gained from the field in the push, from |u1|^2 - |u0|^2 = 2 hq E.(upl + um)
  tl.work += 2.0 * hq * dot(E, upl + um) / (g1 + g0);
  p.x += c.dt * u1.x / g1;
  p.y += c.dt * u1.y / g1;
  if (c.dims == 3) p.z += c.dt * u1.z / g1;
  if (vz_push) *vz_push = u1.z / g1;
  p.ux = u1.x;
  p.uy = u1.y;
  p.uz = u1.z;

  if (c.flags & (FLAG_RR_QUANTUM | FLAG_RR_CLASSICAL)) {
    // continuous radiation reaction: the lepton loses the radiated power P_c g(eta)
    // (eqs. 8 and 9 with Appendix A's g; g = 1 for the classical power) over dt,
    // dgamma = -(2/3) alpha kappa eta^2 g dt, along its momentum and never below rest
    const double eta = eta_of(E, B, u1, g1);
    if (eta > 0.0) {
      const double gfac = (c.flags & FLAG_RR_QUANTUM) ? lookup_g(tb, eta, &tl.n_range) : 1.0;
      const double g2 = std::max(g1 - c.a_rr * eta * eta * gfac * c.dt, 1.0);
      const double umag = std::sqrt(dot(u1, u1));
      const double scale = umag > 0.0 ? std::sqrt((g2 - 1.0) * (g2 + 1.0)) / umag : 0.0;
      p.ux = scale * u1.x;
      p.uy = scale * u1.y;
      p.uz = scale * u1.z;
      tl.radiated += g1 - gamma_of(p.ux, p.uy, p.uz);
    }
  }

  if (c.flags & FLAG_EMIT) {
    const double eta = eta_of(E, B, u1, g1);
    if (eta > 0.0) {
      const double h = lookup_h(tb, eta, &tl.n_range);
      p.tau -= c.a_gamma * (eta / g1) * h * c.dt;  // first-order Euler in the optical depth
      p.margin = std::min(p.margin, std::fabs(p.tau));
      if (p.tau <= 0.0) {
        uint64_t r[4];
        draw(c, p.uid, n, KIND_EMIT, 0, r);
        double chi;
        if (sample_chi(tb, eta, unit_open(r[0]), &chi)) {
          // recoil: the photon carries momentum xi u along the emitter's direction
          const double xi = 2.0 * chi / eta;
          const Vec3 k = xi * u1;
          const Vec3 u2 = u1 - k;
          const double g2 = std::sqrt(1.0 + dot(u2, u2));
          const double eps = std::sqrt(dot(k, k));
          tl.defect_emit += g2 + eps - g1;
          p.ux = u2.x;
          p.uy = u2.y;
          p.uz = u2.z;
          Particle ph;
          ph.x = p.x;
          ph.y = p.y;
          ph.z = p.z;
          ph.ux = k.x;
          ph.uy = k.y;
          ph.uz = k.z;
          ph.tau = optical_depth_draw(r[3]);
          ph.uid = r[2];
          ph.birth = n + 1;  // first stepped in the next step, from the emitter's new position
          ph.species = 2;
          ph.margin = INFINITY;
          ph.alive = true;
          fam.push_back(ph);
          ++tl.n_emit;
        } else {
          ++tl.n_null;
        }
        p.tau = optical_depth_draw(r[1]);
      }
    }
  }
  if (!std::isfinite(p.tau) || !std::isfinite(p.ux) || !std::isfinite(p.uy) || !std::isfinite(p.uz)) ++tl.n_nonfinite;
}

// one step of a photon: it moves at c along k (eq. 5: null geodesics), so its position
// at the start of step n is x_b + (n - birth) dt k/|k|; then the pair optical depth (eq. 3)
void step_photon(Particle& p, const Config& c, const Tables& tb, int64_t n, std::vector<Particle>& fam,
                 Tally& tl) {
  const double t = c.t0 + (double)n * c.dt;
  const Vec3 k = {p.ux, p.uy, p.uz};
  const double eps = std::sqrt(dot(k, k));
  const Vec3 nh = {k.x / eps, k.y / eps, k.z / eps};
  const double age = (double)(n - p.birth) * c.dt;
  const Vec3 xn = {p.x + age * nh.x, p.y + age * nh.y, c.dims == 3 ? p.z + age * nh.z : 0.0};
  Vec3 E, B;
  fields_at(c, xn.x, xn.y, xn.z, t, &E, &B);
  if (c.flags & FLAG_PAIRS) {
    const double chi = chi_of(E, B, nh, eps);
    const double T = lookup_T(tb, chi, &tl.n_range);
    if (T > 0.0) {
      p.tau -= c.a_pair * chi * T / eps * c.dt;
      p.margin = std::min(p.margin, std::fabs(p.tau));
      if (p.tau <= 0.0) {
        uint64_t r0[4], r1[4];
        draw(c, p.uid, n, KIND_PAIR, 0, r0);
        draw(c, p.uid, n, KIND_PAIR, 1, r1);
        const double f = sample_f(tb, chi, unit_open(r0[0]));
        const Vec3 up = f * k;            // positron takes the fraction f
        const Vec3 ue = (1.0 - f) * k;    // electron the rest
        tl.defect_pair += gamma_of(up.x, up.y, up.z) + gamma_of(ue.x, ue.y, ue.z) - eps;
        // the pair appears where the photon is at the end of the step
        const double age1 = age + c.dt;
        Particle e, po;
        e.x = po.x = p.x + age1 * nh.x;
        e.y = po.y = p.y + age1 * nh.y;
        e.z = po.z = c.dims == 3 ? p.z + age1 * nh.z : 0.0;
        e.birth = po.birth = 0;
        e.ux = ue.x;
        e.uy = ue.y;
        e.uz = ue.z;
        po.ux = up.x;
        po.uy = up.y;
        po.uz = up.z;
        e.uid = r0[1];
        po.uid = r0[2];
        e.tau = optical_depth_draw(r0[3]);
        po.tau = optical_depth_draw(r1[0]);
        e.species = 0;
        po.species = 1;
        e.margin = po.margin = INFINITY;
        e.alive = po.alive = true;
        fam.push_back(e);
        fam.push_back(po);
        p.alive = false;  // the photon is annihilated
        ++tl.n_pair;
      }
    }
  }
  if (p.alive && (!std::isfinite(p.tau) || !std::isfinite(eps))) ++tl.n_nonfinite;
}

}  // namespace

extern "C" {

typedef struct {
  int32_t field_kind;
  double field[16];
  int32_t grid_nx, grid_ny;
  double grid_dx, grid_dy, grid_x0, grid_y0;
  int32_t dims;
  double dt, t0;
  int64_t step0, n_steps;
  uint64_t seed, instance;
  uint32_t flags;
  int32_t draw_initial_tau;  // 1: tau = -ln u, u from counter (uid, 0, INIT, 0)
  double lambda_L;           // laser wavelength defining the code units, metres
} oracle_config;

typedef struct {
  // table arrays as produced by oracle_build_tables
  int32_t n_eta;
  double eta_min, eta_max;
  const double* h;
  int32_t n_chi;
  const double* lnchi_min;
  const double* dlnchi;
  const double* P_chi;
  int32_t n_chi_pair;
  double chi_pair_min, chi_pair_max;
  const double* T;
  int32_t n_f;
  const double* f_grid;
  const double* P_f;
  const double* g;  // g(eta) on the h grid; needed only with the quantum reaction flag
} oracle_tables;

typedef struct {
  double *x, *y, *z, *ux, *uy, *uz, *tau, *margin;
  uint64_t* uid;
  int64_t* birth;    // photons: step at whose start the photon sits at (x, y, z) (optional on input)
  int64_t* family;   // out only (optional): index of the input particle the family grew from
  int64_t count;     // in: number of input particles; out: number written
  int64_t capacity;  // out only: room in the arrays
} oracle_species;

typedef struct {
  double energy0[3];   // sum of gamma (leptons) / |k| (photons) at the start
  double energy[3];    // at the end, live particles only
  int64_t count[3];    // live particles at the end
  double work, defect_emit, defect_pair;
  int64_t n_emit, n_null, n_pair, n_range, n_nonfinite;
  int64_t particle_steps;  // live particles advanced, summed over steps
  double radiated;         // energy removed by continuous radiation reaction
} oracle_ledger;

// Runs n_steps steps starting at step0 for every family rooted at an input particle.
// A family is one input particle and all its descendants; families are independent
// (incoherent emission, Section 2.3), so they run in parallel.  Within a family the
// particles present at the start of a step are advanced in creation order; children
// first move in the following step.  Outputs are written family by family in input
// order, each family in creation order.  Returns -1 if an output array is too small
// (the counts then hold the required sizes).
static Config config_of(const oracle_config* cfg) {
  Config c;
  c.field = cfg->field_kind;
  std::memcpy(c.fp, cfg->field, sizeof(c.fp));
  c.grid = {cfg->grid_nx, cfg->grid_ny, cfg->grid_dx, cfg->grid_dy, cfg->grid_x0, cfg->grid_y0};
  c.dims = cfg->dims;
  c.dt = cfg->dt;
  c.t0 = cfg->t0;
  c.step0 = cfg->step0;
  c.n_steps = cfg->n_steps;
  c.seed = cfg->seed;
  c.instance = cfg->instance;
  c.flags = cfg->flags;
  c.kappa = cfg->lambda_L / kLambdaCompton;
  c.a_gamma = std::sqrt(3.0) * kAlpha * c.kappa / (2.0 * kPi);
  c.a_pair = kAlpha * c.kappa;
  c.a_rr = 2.0 / 3.0 * kAlpha * c.kappa;
  return c;
}

// The fields of the configuration at (x, y, z, t) (Sec. 3.2: the fields the step sees), and the
// eta of a lepton / chi of a photon with the given momentum there.
void oracle_fields(const oracle_config* cfg, double x, double y, double z, double t, double* E, double* B) {
  const Config c = config_of(cfg);
  Vec3 e, b;
  fields_at(c, x, y, z, t, &e, &b);
  E[0] = e.x;
  E[1] = e.y;
  E[2] = e.z;
  B[0] = b.x;
  B[1] = b.y;
  B[2] = b.z;
}

// The gather of the configuration's grid for component comp from caller-given node values
// (nodes[j * nx + i], the component's own staggered grid), at (x, y).
double oracle_grid_gather(const oracle_config* cfg, int comp, const double* nodes, double x, double y) {
  const Config c = config_of(cfg);
  return cic_gather(c.grid, comp, x, y, [&](int64_t i, int64_t j) { return nodes[j * c.grid.nx + i]; });
}

double oracle_eta(const oracle_config* cfg, double x, double y, double z, double t, double ux, double uy,
                  double uz) {
  const Config c = config_of(cfg);
  Vec3 E, B;
  fields_at(c, x, y, z, t, &E, &B);
  return eta_of(E, B, {ux, uy, uz}, gamma_of(ux, uy, uz));
}

double oracle_chi(const oracle_config* cfg, double x, double y, double z, double t, double kx, double ky,
                  double kz) {
  const Config c = config_of(cfg);
  Vec3 E, B;
  fields_at(c, x, y, z, t, &E, &B);
  const double eps = std::sqrt(kx * kx + ky * ky + kz * kz);
  return chi_of(E, B, {kx / eps, ky / eps, kz / eps}, eps);
}

int oracle_run(const oracle_config* cfg, const oracle_tables* tab, const oracle_species* in,
               oracle_species* out, oracle_ledger* led) {
  const Config c = config_of(cfg);
  if ((c.flags & FLAG_RR_QUANTUM) && (c.flags & FLAG_RR_CLASSICAL)) return -2;
  if ((c.flags & (FLAG_RR_QUANTUM | FLAG_RR_CLASSICAL)) && (c.flags & FLAG_EMIT)) return -2;
  if ((c.flags & FLAG_RR_QUANTUM) && !tab->g) return -2;

  Tables tb;
  tb.n_eta = tab->n_eta;
  tb.le0 = std::log(tab->eta_min);
  tb.dle = (std::log(tab->eta_max) - tb.le0) / (tab->n_eta - 1);
  tb.h = tab->h;
  tb.g = tab->g;
  tb.n_chi = tab->n_chi;
  tb.lnchi_min = tab->lnchi_min;
  tb.dlnchi = tab->dlnchi;
  tb.P = tab->P_chi;
  tb.n_cp = tab->n_chi_pair;
  tb.lc0 = std::log(tab->chi_pair_min);
  tb.dlc = (std::log(tab->chi_pair_max) - tb.lc0) / (tab->n_chi_pair - 1);
  tb.T = tab->T;
  tb.n_f = tab->n_f;
  tb.f = tab->f_grid;
  tb.Pf = tab->P_f;

  // roots of the families, species by species
  std::vector<Particle> roots;
  for (int s = 0; s < 3; ++s) {
    for (int64_t i = 0; i < in[s].count; ++i) {
      Particle p;
      p.x = in[s].x[i];
      p.y = in[s].y[i];
      p.z = in[s].z ? in[s].z[i] : 0.0;
      p.ux = in[s].ux[i];
      p.uy = in[s].uy[i];
      p.uz = in[s].uz[i];
      p.uid = in[s].uid[i];
      p.birth = in[s].birth ? in[s].birth[i] : 0;
      p.species = s;
      p.margin = INFINITY;
      p.alive = true;
      if (cfg->draw_initial_tau) {
        uint64_t r[4];
        draw(c, p.uid, 0, KIND_INIT, 0, r);
        p.tau = optical_depth_draw(r[0]);
      } else {
        p.tau = in[s].tau[i];
      }
      roots.push_back(p);
    }
  }
  const int64_t nf = (int64_t)roots.size();
  std::vector<std::vector<Particle>> fams(nf);
  std::vector<Tally> tallies(nf);
  std::vector<double> e0(nf);

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t f = 0; f < nf; ++f) {
    std::vector<Particle>& fam = fams[f];
    Tally& tl = tallies[f];
    fam.clear();
    fam.push_back(roots[f]);
    const Particle& r = roots[f];
    e0[f] = (r.species == 2) ? std::sqrt(r.ux * r.ux + r.uy * r.uy + r.uz * r.uz) : gamma_of(r.ux, r.uy, r.uz);
    for (int64_t n = c.step0; n < c.step0 + c.n_steps; ++n) {
      const size_t present = fam.size();
      for (size_t i = 0; i < present; ++i) {
        if (!fam[i].alive) continue;
        // copy: push_back may reallocate while the particle is being advanced
        Particle p = fam[i];
        if (p.species == 2) {
          if (c.flags & FLAG_PROPAGATE) {
            step_photon(p, c, tb, n, fam, tl);
            ++tl.particle_steps;
          }
        } else {
          step_lepton(p, c, tb, n, fam, tl);
          ++tl.particle_steps;
        }
        fam[i] = p;
      }
    }
  }

  // gather outputs and the ledger in family order
  int64_t need[3] = {0, 0, 0};
  for (int64_t f = 0; f < nf; ++f)
    for (const Particle& p : fams[f])
      if (p.alive) ++need[p.species];
  bool fits = true;
  for (int s = 0; s < 3; ++s) {
    if (need[s] > out[s].capacity) fits = false;
  }
  std::memset(led, 0, sizeof(*led));
  for (int64_t f = 0; f < nf; ++f) {
    led->energy0[roots[f].species] += e0[f];
    const Tally& tl = tallies[f];
    led->work += tl.work;
    led->defect_emit += tl.defect_emit;
    led->defect_pair += tl.defect_pair;
    led->radiated += tl.radiated;
    led->n_emit += tl.n_emit;
    led->n_null += tl.n_null;
    led->n_pair += tl.n_pair;
    led->n_range += tl.n_range;
    led->n_nonfinite += tl.n_nonfinite;
    led->particle_steps += tl.particle_steps;
  }
  int64_t w[3] = {0, 0, 0};
  for (int64_t f = 0; f < nf; ++f) {
    for (const Particle& p : fams[f]) {
      if (!p.alive) continue;
      const int s = p.species;
      led->energy[s] += (s == 2) ? std::sqrt(p.ux * p.ux + p.uy * p.uy + p.uz * p.uz) : gamma_of(p.ux, p.uy, p.uz);
      led->count[s] += 1;
      if (fits) {
        const int64_t k = w[s]++;
        out[s].x[k] = p.x;
        out[s].y[k] = p.y;
        if (out[s].z) out[s].z[k] = p.z;
        out[s].ux[k] = p.ux;
        out[s].uy[k] = p.uy;
        out[s].uz[k] = p.uz;
        out[s].tau[k] = p.tau;
        out[s].uid[k] = p.uid;
        if (out[s].margin) out[s].margin[k] = p.margin;
        if (out[s].family) out[s].family[k] = f;
        if (out[s].birth) out[s].birth[k] = p.birth;
      }
    }
  }
  for (int s = 0; s < 3; ++s) out[s].count = need[s];
  return fits ? 0 : -1;
}

// Runs n_steps steps of configuration FIELD_GRID_FDTD with field feedback (Sec. 3.2): every
// step, each particle present at its start is advanced with the fields of the grid as they
// stand (leptons first pushed, then the emission step; photons the pair step), each lepton's
// current is deposited from its positions before and after the push, and then the grid
// advances one step of Maxwell's equations with that current.  Families are coupled through
// the grid, so the run goes step by step over all particles (one thread).  `fields` holds the
// nine planes Ex Ey Ez Bx By Bz Jx Jy Jz (ny x nx each) in and out; the current planes on
// return hold the last step's current.  Outputs and ledger as oracle_run.
int oracle_run_pic(const oracle_config* cfg, const oracle_tables* tab, const oracle_species* in,
                   oracle_species* out, oracle_ledger* led, double* fields) {
  Config c = config_of(cfg);
  if (c.field != FIELD_GRID_FDTD || c.dims != 2) return -2;
  if (c.flags & (FLAG_RR_QUANTUM | FLAG_RR_CLASSICAL)) return -2;
  c.fdtd = fields;
  Tables tb;
  tb.n_eta = tab->n_eta;
  tb.le0 = std::log(tab->eta_min);
  tb.dle = (std::log(tab->eta_max) - tb.le0) / (tab->n_eta - 1);
  tb.h = tab->h;
  tb.g = tab->g;
  tb.n_chi = tab->n_chi;
  tb.lnchi_min = tab->lnchi_min;
  tb.dlnchi = tab->dlnchi;
  tb.P = tab->P_chi;
  tb.n_cp = tab->n_chi_pair;
  tb.lc0 = std::log(tab->chi_pair_min);
  tb.dlc = (std::log(tab->chi_pair_max) - tb.lc0) / (tab->n_chi_pair - 1);
  tb.T = tab->T;
  tb.n_f = tab->n_f;
  tb.f = tab->f_grid;
  tb.Pf = tab->P_f;

  std::vector<Particle> all;
  std::vector<int64_t> family;
  std::memset(led, 0, sizeof(*led));
  for (int s = 0; s < 3; ++s) {
    for (int64_t i = 0; i < in[s].count; ++i) {
      Particle p;
      p.x = in[s].x[i];
      p.y = in[s].y[i];
      p.z = 0.0;
      p.ux = in[s].ux[i];
      p.uy = in[s].uy[i];
      p.uz = in[s].uz[i];
      p.uid = in[s].uid[i];
      p.birth = in[s].birth ? in[s].birth[i] : 0;
      p.species = s;
      p.margin = INFINITY;
      p.alive = true;
      if (cfg->draw_initial_tau) {
        uint64_t r[4];
        draw(c, p.uid, 0, KIND_INIT, 0, r);
        p.tau = optical_depth_draw(r[0]);
      } else {
        p.tau = in[s].tau[i];
      }
      led->energy0[s] += (s == 2) ? std::sqrt(p.ux * p.ux + p.uy * p.uy + p.uz * p.uz) : gamma_of(p.ux, p.uy, p.uz);
      family.push_back((int64_t)all.size());
      all.push_back(p);
    }
  }
  const int64_t plane = (int64_t)c.grid.nx * c.grid.ny;
  double* J = fields + 6 * plane;
  Tally tl;
  for (int64_t n = c.step0; n < c.step0 + c.n_steps; ++n) {
    std::fill(J, J + 3 * plane, 0.0);
    const size_t present = all.size();
    for (size_t i = 0; i < present; ++i) {
      if (!all[i].alive) continue;
      Particle p = all[i];  // copy: push_back may reallocate while the particle is advanced
      const size_t before = all.size();
      if (p.species == 2) {
        if (c.flags & FLAG_PROPAGATE) {
          step_photon(p, c, tb, n, all, tl);
          ++tl.particle_steps;
        }
      } else {
        const double x0 = p.x, y0 = p.y;
        double vz = 0.0;
        step_lepton(p, c, tb, n, all, tl, &vz);
        ++tl.particle_steps;
        const double Q = (p.species == 0 ? -1.0 : 1.0) * c.fp[0];
        deposit_current(c.grid, Q, c.dt, x0, y0, p.x, p.y, vz, J);
      }
      all[i] = p;
      for (size_t k = before; k < all.size(); ++k) family.push_back(family[i]);
    }
    fdtd_step(c.grid, c.dt, fields);
  }

  led->work = tl.work;
  led->defect_emit = tl.defect_emit;
  led->defect_pair = tl.defect_pair;
  led->n_emit = tl.n_emit;
  led->n_null = tl.n_null;
  led->n_pair = tl.n_pair;
  led->n_range = tl.n_range;
  led->n_nonfinite = tl.n_nonfinite;
  led->particle_steps = tl.particle_steps;
  int64_t need[3] = {0, 0, 0};
  for (const Particle& p : all)
    if (p.alive) ++need[p.species];
  bool fits = true;
  for (int s = 0; s < 3; ++s)
    if (need[s] > out[s].capacity) fits = false;
  int64_t w[3] = {0, 0, 0};
  for (size_t i = 0; i < all.size(); ++i) {
    const Particle& p = all[i];
    if (!p.alive) continue;
    const int s = p.species;
    led->energy[s] += (s == 2) ? std::sqrt(p.ux * p.ux + p.uy * p.uy + p.uz * p.uz) : gamma_of(p.ux, p.uy, p.uz);
    led->count[s] += 1;
    if (fits) {
      const int64_t k = w[s]++;
      out[s].x[k] = p.x;
      out[s].y[k] = p.y;
      if (out[s].z) out[s].z[k] = p.z;
      out[s].ux[k] = p.ux;
      out[s].uy[k] = p.uy;
      out[s].uz[k] = p.uz;
      out[s].tau[k] = p.tau;
      out[s].uid[k] = p.uid;
      if (out[s].margin) out[s].margin[k] = p.margin;
      if (out[s].family) out[s].family[k] = family[i];
      if (out[s].birth) out[s].birth[k] = p.birth;
    }
  }
  for (int s = 0; s < 3; ++s) out[s].count = need[s];
  return fits ? 0 : -1;
}

// The current of one macro-particle move (deposit_current) added to the three planes J, and one
// step of the Yee solver on the nine planes F, for tests of the two pieces alone.
void oracle_deposit(const oracle_config* cfg, double Q, double x0, double y0, double x1, double y1, double vz,
                    double* J) {
  const Config c = config_of(cfg);
  deposit_current(c.grid, Q, c.dt, x0, y0, x1, y1, vz, J);
}
void oracle_fdtd_step(const oracle_config* cfg, double* F) {
  const Config c = config_of(cfg);
  fdtd_step(c.grid, c.dt, F);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// threads of the following runs (the run's results do not depend on it: families are
// independent and every sum is exact)
void oracle_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

}  // extern "C"
