// FP32-mixed form of the step kernels.
//
// Precision split: the push, the field evaluation, eta/chi and the h / T look-ups run in
// FP32; positions and momenta of leptons are stored as FP32 (hi, lo) pairs and updated by
// compensated (two-sum) addition of FP32 increments, so the stored value keeps ~48 bits;
// photons are stored in FP32 (birth position, momentum).  The optical depth, the sampling
// of chi and f from the cumulative tables, the recoil bookkeeping and every energy that
// enters the ledger stay FP64.  Field phases are formed and range-reduced in FP64 before
// the FP32 trigonometry.
#pragma once

#include "qed_device.h"

namespace qedk {

// (hi, lo) += d with an FP32 two-sum and renormalisation
__device__ __forceinline__ void comp_add(float& hi, float& lo, float d) {
  const float s = hi + d;
  const float bb = s - hi;
  const float err = (hi - (s - bb)) + (d - bb);
  const float l = lo + err;
  hi = s + l;
  lo = l - (hi - s);
}

__device__ __forceinline__ void split_double(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

// phase psi reduced to [-pi, pi] in FP64, returned as float
__device__ __forceinline__ float reduce_phase(double psi) {
  const double two_pi = 2.0 * kPi;
  return (float)(psi - two_pi * rint(psi * kInvTwoPi));
}

template <int FK>
__device__ __forceinline__ void field_at32(const qed_field& F, const FieldK& K, double x, double y, double t, float E[3],
                                           float B[3]) {
  E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0f;
  if (FK == QED_FIELD_UNIFORM) {
    E[0] = (float)F.p[0];
    E[1] = (float)F.p[1];
    E[2] = (float)F.p[2];
    B[0] = (float)F.p[3];
    B[1] = (float)F.p[4];
    B[2] = (float)F.p[5];
  } else if (FK == QED_FIELD_LP_PULSE) {
    const double psi = t - x - F.p[2];
    if (psi >= 0.0 && psi <= F.p[1]) {
      float s, c, d;
      fast_sincosf((float)(psi * K.pi_over_len), &s, &d);
      fast_sincosf(reduce_phase(psi + F.p[3]), &d, &c);
      const float e = (float)F.p[0] * s * s * c;
      E[1] = e;
      B[2] = e;
    }
  } else if (FK == QED_FIELD_CP_WAVE) {
    float sn, cs;
    fast_sincosf(reduce_phase(t - x + F.p[1]), &sn, &cs);
    const float e0 = (float)F.p[0];
    E[1] = e0 * cs;
    E[2] = e0 * sn;
    B[1] = -e0 * sn;
    B[2] = e0 * cs;
  } else if (FK == QED_FIELD_CP_STANDING) {
    float st, ct, sx, cx;
    fast_sincosf(reduce_phase(t), &st, &ct);
    fast_sincosf(reduce_phase(x), &sx, &cx);
    const float e2 = 2.0f * (float)F.p[0];
    E[1] = e2 * ct * cx;
    E[2] = e2 * st * cx;
    B[1] = e2 * ct * sx;
    B[2] = e2 * st * sx;
  } else if (FK == QED_FIELD_GRID_FDTD) {
    // (the binding runs this kind in FP64 only; the gather is here for completeness)
    double e[3], b[3];
    cic_gather6(F, (const double*)F.fdtd_dev, x, y, e, b);
    for (int k = 0; k < 3; ++k) {
      E[k] = (float)e[k];
      B[k] = (float)b[k];
    }
  } else if (FK == QED_FIELD_GRID_CP_STANDING) {
    const float ox[6] = {0.5f, 0.0f, 0.0f, 0.0f, 0.5f, 0.5f};
    const float oy[6] = {0.0f, 0.5f, 0.0f, 0.5f, 0.0f, 0.5f};
    const int64_t plane = (int64_t)F.nx * F.ny;
    // cell coordinates in FP64 (large domains), weights in FP32
    const double cxd = (x - F.x0) / F.dx, cyd = (y - F.y0) / F.dy;
    float v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double gx = cxd - ox[c], gy = cyd - oy[c];
      const double fx = floor(gx), fy = floor(gy);
      const float wx = (float)(gx - fx), wy = (float)(gy - fy);
      const int64_t i0 = (int64_t)fx, j0 = (int64_t)fy;
      const int64_t ia = wrap_index(i0, F.nx), ib = wrap_index(i0 + 1, F.nx);
      const int64_t ja = wrap_index(j0, F.ny), jb = wrap_index(j0 + 1, F.ny);
      gptr<const float> g = as_global((const float*)F.grid_dev + c * plane);
      v[c] = (1.0f - wx) * (1.0f - wy) * g[ja * F.nx + ia] + wx * (1.0f - wy) * g[ja * F.nx + ib] +
             (1.0f - wx) * wy * g[jb * F.nx + ia] + wx * wy * g[jb * F.nx + ib];
    }
    E[0] = v[0];
    E[1] = v[1];
    E[2] = v[2];
    B[0] = v[3];
    B[1] = v[4];
    B[2] = v[5];
  }
}

// rate look-up in FP32: `idl` is the reciprocal of the table's ln-spacing
__device__ __forceinline__ float lookup32(const float* tab, int n, double l0, double idl, float arg, unsigned& range,
                                          bool zero_below) {
  if (!(arg > 0.0f)) return zero_below ? 0.0f : tab[0];
  const float s = (logf(arg) - (float)l0) * (float)idl;
  if (!(s > 0.0f)) return zero_below ? (s < 0.0f ? 0.0f : tab[0]) : tab[0];
  if (s >= (float)(n - 1)) {
    ++range;
    return tab[n - 1];
  }
  const int i = (int)floorf(s);
  const float w = s - (float)i;
  return (1.0f - w) * tab[i] + w * tab[i + 1];
}

}  // namespace qedk
