// Device-side building blocks of the QED Monte-Carlo step (gfx950, wave64):
// constants, the Philox4x64-10 stream, field providers, the Boris push, table
// look-ups and wavefront-aggregated appends.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qed.h"
#include "qed_crmath.h"

namespace qedk {

// CODATA 2018
constexpr double kPi = 3.14159265358979323846;
constexpr double kAlpha = 7.2973525693e-3;             // fine-structure constant
constexpr double kLambdaCompton = 2.42631023867e-12;   // h/(m_e c) in metres

enum : uint64_t { KIND_INIT = 0, KIND_EMIT = 1, KIND_PAIR = 2 };

// Device copy of the tables plus their grid constants.
struct Tabs {
  int n_eta;
  double le0, dle;             // ln eta_min, ln-spacing of the eta rows
  const double* h;
  const float* h32;
  int n_chi;
  const double* lnchi_min;     // per row: ln chi_0 and ln-spacing of the columns
  const double* dlnchi;
  const double* P;             // [n_eta][n_chi]
  int n_cp;
  double lc0, dlc;             // ln chi_pair_min, ln-spacing of the pair rows
  const double* T;
  const float* T32;
  int n_f;
  const double* f;             // f grid
  const double* Pf;            // [n_cp][n_f]
};

// Step constants derived from qed_step_params.
struct StepConst {
  double t0, dt;
  double kappa;     // lambda_L / lambda_c = m c^2 / (hbar w)
  double a_gamma;   // sqrt(3) alpha kappa / (2 pi): eq. 2 in code time
  double a_pair;    // alpha kappa: eq. 3 in code time
  uint32_t flags;
};

// Per-instance device accumulators and step scratch.
struct InstAcc {
  int64_t n_start[3];          // particles present at the start of the step (or pass)
  int64_t n_live;              // compaction: live photons
  int64_t mover_off;           // compaction: offset of this instance's mover list
  unsigned long long hole_ctr, mover_ctr;
  double work, defect_emit, defect_pair, dropped_energy;
  double led_energy[3];
  unsigned long long led_count[3];
  unsigned long long n_emit, n_null, n_pair, n_dropped, n_range, n_nonfinite, n_field;
  unsigned long long particle_steps[3];  // particles (photon slots) present at the start of each step
};

// Workspace-global device state.
struct Glob {
  int64_t step_cur, step_next;   // device clock: index of the running / next step
  int64_t n_chunks[2];           // chunk-list lengths: 0 leptons, 1 photons
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): counter (uid, step, kind, sub), key (seed, instance)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1, uint64_t out[4]) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// uniform on (0, 1) from the top 53 bits: (m + 1/2) 2^-53
__device__ __forceinline__ double unit_open(uint64_t r) { return ((double)(r >> 11) + 0.5) * 0x1.0p-53; }

// optical depth at which the next reaction happens: P = 1 - exp(-tau) uniform (Sec. 3)
__device__ __forceinline__ double optical_depth(uint64_t r) { return -cr_log(unit_open(r)); }

// ---------------------------------------------------------------------------
// fields at a point (FP64); the grid kind gathers FP32 node values with CIC weights
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t wrap_index(int64_t i, int n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

// EXACT selects correctly rounded trigonometry (bit-reproducible momenta); the fast variant
// (device library, <= 1 ulp) serves quantities that only feed an optical-depth decrement.
template <int FK, bool EXACT = true>
__device__ __forceinline__ void field_at(const qed_field& F, double x, double y, double t, double E[3],
                                         double B[3]) {
  E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
  if (FK == QED_FIELD_UNIFORM) {
    E[0] = F.p[0];
    E[1] = F.p[1];
    E[2] = F.p[2];
    B[0] = F.p[3];
    B[1] = F.p[4];
    B[2] = F.p[5];
  } else if (FK == QED_FIELD_LP_PULSE) {
    const double psi = t - x - F.p[2];
    if (psi >= 0.0 && psi <= F.p[1]) {
      const double s = EXACT ? cr_sin(kPi * psi / F.p[1]) : sin(kPi * psi / F.p[1]);
      const double e = F.p[0] * s * s * (EXACT ? cr_cos(psi + F.p[3]) : cos(psi + F.p[3]));
      E[1] = e;
      B[2] = e;
    }
  } else if (FK == QED_FIELD_CP_WAVE) {
    const double psi = t - x + F.p[1];
    double sn, cs;
    if (EXACT) cr_sincos(psi, &sn, &cs);
    else sincos(psi, &sn, &cs);
    const double ey = F.p[0] * cs, ez = F.p[0] * sn;
    E[1] = ey;
    E[2] = ez;
    B[1] = -ez;
    B[2] = ey;
  } else if (FK == QED_FIELD_CP_STANDING) {
    double st, ct, sx, cx;
    if (EXACT) {
      cr_sincos(t, &st, &ct);
      cr_sincos(x, &sx, &cx);
    } else {
      sincos(t, &st, &ct);
      sincos(x, &sx, &cx);
    }
    E[1] = 2.0 * F.p[0] * ct * cx;
    E[2] = 2.0 * F.p[0] * st * cx;
    B[1] = 2.0 * F.p[0] * ct * sx;
    B[2] = 2.0 * F.p[0] * st * sx;
  } else if (FK == QED_FIELD_GRID_CP_STANDING) {
    // first-order shape: bilinear weights on each staggered component grid
    const double ox[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
    const double oy[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};
    const int64_t plane = (int64_t)F.nx * F.ny;
    double v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double gx = (x - F.x0) / F.dx - ox[c];
      const double gy = (y - F.y0) / F.dy - oy[c];
      const double fx = floor(gx), fy = floor(gy);
      const double wx = gx - fx, wy = gy - fy;
      const int64_t i0 = (int64_t)fx, j0 = (int64_t)fy;
      const int64_t ia = wrap_index(i0, F.nx), ib = wrap_index(i0 + 1, F.nx);
      const int64_t ja = wrap_index(j0, F.ny), jb = wrap_index(j0 + 1, F.ny);
      const float* g = F.grid_dev + c * plane;
      const double g00 = g[ja * F.nx + ia], g10 = g[ja * F.nx + ib];
      const double g01 = g[jb * F.nx + ia], g11 = g[jb * F.nx + ib];
      v[c] = (1.0 - wx) * (1.0 - wy) * g00 + wx * (1.0 - wy) * g10 + (1.0 - wx) * wy * g01 + wx * wy * g11;
    }
    E[0] = v[0];
    E[1] = v[1];
    E[2] = v[2];
    B[0] = v[3];
    B[1] = v[4];
    B[2] = v[5];
  }
}

// ---------------------------------------------------------------------------
// table look-ups (Sec. 3: linear interpolation in the look-up tables)
// ---------------------------------------------------------------------------

// h(eta) from an LDS copy; clamped outside [eta_min, eta_max], counting eta > eta_max.  The
// rate only feeds the optical-depth decrement, so the device library's log serves.
__device__ __forceinline__ double lookup_h(const double* sh, const Tabs& tb, double eta, unsigned& range) {
  const double s = (log(eta) - tb.le0) / tb.dle;
  if (!(s > 0.0)) return sh[0];
  if (s >= tb.n_eta - 1) {
    ++range;
    return sh[tb.n_eta - 1];
  }
  const int i = (int)floor(s);
  const double w = s - i;
  return (1.0 - w) * sh[i] + w * sh[i + 1];
}

// T(chi) from an LDS copy; zero below chi_pair_min (T < 1e-58 there); feeds only the
// optical-depth decrement
__device__ __forceinline__ double lookup_T(const double* sT, const Tabs& tb, double chi, unsigned& range) {
  if (!(chi > 0.0)) return 0.0;
  const double s = (log(chi) - tb.lc0) / tb.dlc;
  if (s < 0.0) return 0.0;
  if (s >= tb.n_cp - 1) {
    ++range;
    return sT[tb.n_cp - 1];
  }
  const int k = (int)floor(s);
  const double w = s - k;
  return (1.0 - w) * sT[k] + w * sT[k + 1];
}

// Largest j with P[j] < u (so P[j] < u <= P[j+1]; P[n-1] = 1 > u) and the position of u in
// that segment.  Flat segments (P[j] == P[j+1]) are never selected.
__device__ __forceinline__ int row_inverse(const double* __restrict__ P, int n, double u, double* frac) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (P[mid] < u) lo = mid; else hi = mid;
  }
  *frac = (u - P[lo]) / (P[hi] - P[lo]);
  return lo;
}

// chi from P_chi at the emitter's eta (rows i, i+1 blended in ln eta); false below the cut-off
__device__ inline bool sample_chi(const Tabs& tb, double eta, double u, double* chi) {
  const double leta = cr_log(eta);
  const double s = (leta - tb.le0) / tb.dle;
  double lnchi;
  auto Q = [&](int r, double* q) {
    const double* P = tb.P + (size_t)r * tb.n_chi;
    if (u <= P[0]) return false;
    double fr;
    const int j = row_inverse(P, tb.n_chi, u, &fr);
    *q = tb.lnchi_min[r] + (j + fr) * tb.dlnchi[r];
    return true;
  };
  if (!(s > 0.0)) {
    double q0;
    if (!Q(0, &q0)) return false;
    lnchi = q0 + 2.0 * (leta - tb.le0);  // classical scaling chi ~ eta^2 below the table
  } else if (s >= tb.n_eta - 1) {
    double q1;
    if (!Q(tb.n_eta - 1, &q1)) return false;
    lnchi = q1 + (leta - (tb.le0 + (tb.n_eta - 1) * tb.dle));  // fixed 2 chi/eta above it
  } else {
    const int i = (int)floor(s);
    const double w = s - i;
    double qa, qb;
    const bool oka = Q(i, &qa);
    const bool okb = Q(i + 1, &qb);
    if (!oka || !okb) return false;
    lnchi = (1.0 - w) * qa + w * qb;
  }
  *chi = cr_exp(lnchi);
  return true;
}

// positron energy fraction f from P_f (rows blended in ln chi, linear in f within a row)
__device__ inline double sample_f(const Tabs& tb, double chi, double u) {
  const double s = (cr_log(chi) - tb.lc0) / tb.dlc;
  auto frow = [&](int r) {
    double fr;
    const int j = row_inverse(tb.Pf + (size_t)r * tb.n_f, tb.n_f, u, &fr);
    return tb.f[j] + fr * (tb.f[j + 1] - tb.f[j]);
  };
  if (!(s > 0.0)) return frow(0);
  if (s >= tb.n_cp - 1) return frow(tb.n_cp - 1);
  const int k = (int)floor(s);
  const double w = s - k;
  return (1.0 - w) * frow(k) + w * frow(k + 1);
}

// ---------------------------------------------------------------------------
// wavefront-aggregated append: one atomic per wave reserves slots for every lane that wants
// one; lanes receive consecutive slots in lane order.  Call from wave-convergent code.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long wave_reserve(bool want, int64_t* counter) {
  const unsigned long long mask = __ballot(want);
  if (mask == 0ull) return -1;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  const int total = __popcll(mask);
  const int prefix = __popcll(mask & ((1ull << lane) - 1ull));
  long long base = 0;
  if (lane == leader) base = (long long)atomicAdd((unsigned long long*)counter, (unsigned long long)total);
  base = __shfl(base, leader);
  return want ? base + prefix : -1;
}

// block-wide sums of a few accumulators; result valid in thread 0.  Every thread must call.
template <int ND, int NU>
__device__ inline void block_sum(double (&d)[ND], unsigned (&u)[NU], double* sd, unsigned* su) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < ND; ++a) d[a] += __shfl_down(d[a], off);
#pragma unroll
    for (int a = 0; a < NU; ++a) u[a] += __shfl_down(u[a], off);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < ND; ++a) sd[wave * ND + a] = d[a];
#pragma unroll
    for (int a = 0; a < NU; ++a) su[wave * NU + a] = u[a];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) {
#pragma unroll
      for (int a = 0; a < ND; ++a) d[a] += sd[w * ND + a];
#pragma unroll
      for (int a = 0; a < NU; ++a) u[a] += su[w * NU + a];
    }
  }
  __syncthreads();
}

}  // namespace qedk
