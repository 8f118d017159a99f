// Look-up table construction on the device (FP64), Sec. 3 of the paper with the
// functions of Appendix A (quantum synchrotron spectrum F, h) and Appendix B (T_pm, p_f).
//
// Quadrature design (independent of any CPU reference):
//  * K_nu(y) and int_y^inf K_nu(t) dt from the integral representation
//      e^{-y} int_0^inf exp(-2 y sinh^2(t/2)) cosh(nu t) [/ cosh t] dt
//    by the trapezoid rule in t, which converges geometrically for this entire,
//    doubly-exponentially decaying integrand (step 0.2, or 0.7/sqrt(y) for large y).
//  * synchrotron integrals in v = ln y, y = 2 xi / (3 eta (1 - xi)), xi = 2 chi/eta:
//      xi = a y / (1 + a y), 1 - xi = 1 / (1 + a y), a = 3 eta / 2,
//      dchi/chi = (1 - xi) dv,
//    so both ends of the spectrum are resolved without cancellation.  Composite
//    16-point Gauss-Legendre panels no wider than 0.25 in v; below v0 = -70 the
//    spectrum follows its chi^{1/3} power law and the tail is added in closed form.
//  * pair splits in theta with f = sin^2 theta (the table's own f grid is uniform
//    in theta), f (1 - f) = sin^2 theta cos^2 theta.
// One workgroup per table row; reductions in a fixed order (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qed_device.h"

namespace qedk {

struct GL16 {
  double x[16], w[16];
};

constexpr double kV0 = -70.0;       // lower end of the v = ln y integrals
constexpr double kPanel = 0.25;     // widest panel in v
constexpr int kRowThreads = 256;

// K_{nu_k}(y) and, if want_j, int_y^inf K_{nu_j}; 0 when y > 745 (below the FP64 range)
__device__ void bessel_trap(double y, double nu_k, double nu_j, bool want_j, double* K, double* J) {
  *K = 0.0;
  if (J) *J = 0.0;
  if (!(y < 745.0)) return;
  const double h = y > 12.25 ? 0.7 / sqrt(y) : 0.2;
  double sk = 0.5, sj = want_j ? 0.5 : 0.0;  // node t = 0: cosh = 1
  double prev = 1.0;
  for (int k = 1; k < 4000; ++k) {
    const double t = k * h;
    const double sh = sinh(0.5 * t);
    const double e = exp(-2.0 * y * sh * sh);
    const double fk = e * cosh(nu_k * t);
    sk += fk;
    if (want_j) sj += e * cosh(nu_j * t) / cosh(t);
    // unimodal integrand: stop once it is falling and negligible
    if (fk < prev && fk < 1e-18 * sk && e < 1e-3) break;
    prev = fk;
  }
  const double ey = exp(-y);
  *K = h * sk * ey;
  if (J) *J = h * sj * ey;
}

// F(eta, chi) at v = ln y for an eta row with a = 3 eta / 2; also returns xi and 1 - xi
__device__ double synch_F_v(double a, double v, double* xi, double* omxi) {
  const double y = exp(v);
  const double ay = a * y;
  *omxi = 1.0 / (1.0 + ay);
  *xi = ay * *omxi;
  double k23, j53;
  bessel_trap(y, 2.0 / 3.0, 5.0 / 3.0, true, &k23, &j53);
  return (*xi) * (*xi) * y * k23 + (*omxi) * y * j53;
}

// number density in v: F / chi dchi = F (1 - xi) dv
__device__ double dens_number(double a, double v) {
  double xi, om;
  const double F = synch_F_v(a, v, &xi, &om);
  return F * om;
}

// energy density in v, in units of eta/2: F dchi = (eta/2) F xi (1 - xi) dv
__device__ double dens_energy(double a, double v) {
  double xi, om;
  const double F = synch_F_v(a, v, &xi, &om);
  return F * xi * om;
}

// integral over [va, vb] of dens (0 number, 1 energy), panels of width <= kPanel, by one thread
__device__ double integrate_serial(const GL16& gl, double a, double va, double vb, int which) {
  if (!(vb > va)) return 0.0;
  const int np = (int)fmin(ceil((vb - va) / kPanel), 2048.0);
  const double w = (vb - va) / np;
  double s = 0.0;
  for (int p = 0; p < np; ++p) {
    const double c = va + (p + 0.5) * w, hw = 0.5 * w;
    double ps = 0.0;
    for (int q = 0; q < 16; ++q) {
      const double v = c + hw * gl.x[q];
      ps += gl.w[q] * (which ? dens_energy(a, v) : dens_number(a, v));
    }
    s += ps * hw;
  }
  return s;
}

__device__ double block_reduce(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// the same integral with the panel nodes spread over the workgroup
__device__ double integrate_block(const GL16& gl, double a, double va, double vb, int which, double* red) {
  double s = 0.0;
  if (vb > va) {
    const int np = (int)fmin(ceil((vb - va) / kPanel), 2048.0);
    const double w = (vb - va) / np, hw = 0.5 * w;
    for (int n = threadIdx.x; n < np * 16; n += blockDim.x) {
      const int p = n >> 4, q = n & 15;
      const double v = va + (p + 0.5) * w + hw * gl.x[q];
      s += gl.w[q] * hw * (which ? dens_energy(a, v) : dens_number(a, v));
    }
  }
  return block_reduce(s, red);
}

// Row i of h, g and P_chi.  Steps: total energy of the spectrum (and g from it); v_c of the 1e-9 energy cut
// (Newton on the cumulative energy); log-spaced chi grid from chi_min to eta/2; number
// integral of each segment; prefix sums normalised by h = the total number integral.
__global__ __launch_bounds__(kRowThreads) void k_build_eta_rows(qed_table_params p, GL16 gl, double* h,
                                                                  double* lnchi_min, double* dlnchi, double* P,
                                                                  double* g) {
  __shared__ double red[kRowThreads];
  __shared__ double seg[1024];
  __shared__ double sh_vc;
  const int i = blockIdx.x;
  const double le0 = log(p.eta_min), le1 = log(p.eta_max);
  const double eta = exp(le0 + i * ((le1 - le0) / (p.n_eta - 1)));
  const double a = 1.5 * eta;
  const double stop = log(0.5 * eta);
  const double vmax = log(745.0);

  // total energy (tail below kV0 ~ y^{4/3}: (3/4) of the density there)
  const double e_tail = 0.75 * dens_energy(a, kV0);
  const double e_tot = e_tail + integrate_block(gl, a, kV0, vmax, 1, red);
  const double target = p.cutoff_energy_frac * e_tot;
  // g = 3 sqrt3 / (2 pi eta^2) int_0^{eta/2} F dchi, and the energy density is in units of eta/2
  if (threadIdx.x == 0) g[i] = 3.0 * sqrt(3.0) / (4.0 * kPi * eta) * e_tot;

  // starting point: at small y the cumulative energy is (3/4) of the density (power law)
  if (threadIdx.x == 0) {
    double lo = kV0, hi = vmax;
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (0.75 * dens_energy(a, mid) > target) hi = mid; else lo = mid;
    }
    sh_vc = 0.5 * (lo + hi);
  }
  __syncthreads();
  double vc = sh_vc;
  // Newton on E(v) = tail + int_{v0}^{v} dens_energy = target
  for (int it = 0; it < 30; ++it) {
    const double E = e_tail + integrate_block(gl, a, kV0, vc, 1, red);
    const double d = (E - target) / dens_energy(a, vc);
    vc = fmin(fmax(vc - d, kV0), vmax);  // stay inside the integration range
    if (!(fabs(d) >= 1e-15 * fabs(vc))) break;
  }
  // ln chi_min = ln(eta/2) + ln xi_c, xi_c = a y_c / (1 + a y_c)
  const double smin = stop + vc + log(a) - log1p(a * exp(vc));
  const int n = p.n_chi;
  const double ds = (stop - smin) / (n - 1);

  // segment j covers [s_{j-1}, s_j]; in v: v = d - ln a - ln(-expm1(d)), d = s - ln(eta/2)
  auto v_of = [&](int j) {
    if (j == 0) return vc;
    if (j >= n - 1) return vmax;
    const double d = (smin + j * ds) - stop;
    const double v = d - log(a) - log(-expm1(d));
    return v < vmax ? v : vmax;
  };
  const double below = 3.0 * dens_number(a, kV0) + integrate_block(gl, a, kV0, vc, 0, red);
  for (int j = 1 + threadIdx.x; j < n; j += blockDim.x) {
    seg[j] = integrate_serial(gl, a, v_of(j - 1), v_of(j), 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double cum = below;
    seg[0] = below;
    for (int j = 1; j < n; ++j) {
      cum += seg[j];
      seg[j] = cum;
    }
    h[i] = cum;
    lnchi_min[i] = smin;
    dlnchi[i] = ds;
  }
  __syncthreads();
  const double hv = seg[n - 1];
  for (int j = threadIdx.x; j < n; j += blockDim.x) P[(size_t)i * n + j] = (j == n - 1) ? 1.0 : seg[j] / hv;
}

// unnormalised pair split density times df/dtheta, at f = sin^2 theta:
// (2 + g)/g K_{2/3}(1/(3 chi g)) sin(2 theta), g = f(1 - f) = sin^2 theta cos^2 theta
__device__ double pair_integrand(double chi, double theta) {
  double s, c;
  sincos(theta, &s, &c);
  const double g = s * s * c * c;
  if (!(g > 0.0)) return 0.0;
  double k23;
  bessel_trap(1.0 / (3.0 * chi * g), 2.0 / 3.0, 0.0, false, &k23, nullptr);
  return (2.0 + g) / g * k23 * (2.0 * s * c);
}

// Row k of T and P_f: T = 0.16 K_{1/3}^2(2/(3 chi)) / chi; f_l = sin^2(pi l / 2(n_f - 1));
// each segment by two 16-point Gauss-Legendre panels in theta; prefix sums normalised by k(chi)
__global__ __launch_bounds__(kRowThreads) void k_build_pair_rows(qed_table_params p, GL16 gl, double* T,
                                                                   double* fgrid, double* Pf, double* knorm) {
  __shared__ double seg[1024];
  const int k = blockIdx.x;
  const double lc0 = log(p.chi_pair_min), lc1 = log(p.chi_pair_max);
  const double chi = exp(lc0 + k * ((lc1 - lc0) / (p.n_chi_pair - 1)));
  const int n = p.n_f;
  const double dth = 0.5 * kPi / (n - 1);
  if (threadIdx.x == 0) {
    double k13;
    bessel_trap(2.0 / (3.0 * chi), 1.0 / 3.0, 0.0, false, &k13, nullptr);
    T[k] = 0.16 * k13 * k13 / chi;
  }
  for (int l = 1 + threadIdx.x; l < n; l += blockDim.x) {
    const double ta = (l - 1) * dth;
    double s = 0.0;
    for (int half = 0; half < 2; ++half) {
      const double c = ta + (half + 0.5) * 0.5 * dth, hw = 0.25 * dth;
      double ps = 0.0;
      for (int q = 0; q < 16; ++q) ps += gl.w[q] * pair_integrand(chi, c + hw * gl.x[q]);
      s += ps * hw;
    }
    seg[l] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double cum = 0.0;
    seg[0] = 0.0;
    for (int l = 1; l < n; ++l) {
      cum += seg[l];
      seg[l] = cum;
    }
    knorm[k] = cum;
  }
  __syncthreads();
  const double kn = seg[n - 1];
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    Pf[(size_t)k * n + l] = (l == 0) ? 0.0 : (l == n - 1 ? 1.0 : seg[l] / kn);
    if (k == 0) {
      const double s = sin(l * dth);
      fgrid[l] = (l == 0) ? 0.0 : (l == n - 1 ? 1.0 : s * s);
    }
  }
}

}  // namespace qedk

// host-side launchers (called from qed_capi.hip)
namespace qedk {

// 16-point Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_16 from the
// Chebyshev-like starting guesses cos(pi (i - 1/4) / (n + 1/2)).
static GL16 gauss_legendre16() {
  GL16 g;
  const int n = 16;
  for (int i = 0; i < n / 2; ++i) {
    double z = cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pk = 1.0, pkm1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double pkm2 = pkm1;
        pkm1 = pk;
        pk = ((2 * k - 1) * z * pkm1 - (k - 1) * pkm2) / k;
      }
      dp = n * (z * pk - pkm1) / (z * z - 1.0);
      const double dz = pk / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) {
        // refresh the derivative at the final node
        pk = 1.0;
        pkm1 = 0.0;
        for (int k = 1; k <= n; ++k) {
          const double pkm2 = pkm1;
          pkm1 = pk;
          pk = ((2 * k - 1) * z * pkm1 - (k - 1) * pkm2) / k;
        }
        dp = n * (z * pk - pkm1) / (z * z - 1.0);
        break;
      }
    }
    g.x[i] = -z;
    g.x[n - 1 - i] = z;
    g.w[i] = g.w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return g;
}

hipError_t launch_build_tables(const qed_table_params& p, double* h, double* lnchi_min, double* dlnchi, double* P,
                               double* T, double* fgrid, double* Pf, double* knorm, double* g, hipStream_t s) {
  const GL16 gl = gauss_legendre16();
  hipLaunchKernelGGL(k_build_eta_rows, dim3(p.n_eta), dim3(kRowThreads), 0, s, p, gl, h, lnchi_min, dlnchi, P, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_build_pair_rows, dim3(p.n_chi_pair), dim3(kRowThreads), 0, s, p, gl, T, fgrid, Pf, knorm);
  return hipGetLastError();
}

}  // namespace qedk
