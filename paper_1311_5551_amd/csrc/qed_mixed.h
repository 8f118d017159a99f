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
  return (float)(psi - two_pi * rint(psi / two_pi));
}

template <int FK>
__device__ __forceinline__ void field_at32(const qed_field& F, double x, double y, double t, float E[3], float B[3]) {
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
      fast_sincosf((float)(kPi * (psi / F.p[1])), &s, &d);
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

__device__ __forceinline__ float lookup32(const float* tab, int n, double l0, double dl, float arg, unsigned& range,
                                          bool zero_below) {
  if (!(arg > 0.0f)) return zero_below ? 0.0f : tab[0];
  const float s = (logf(arg) - (float)l0) / (float)dl;
  if (!(s > 0.0f)) return zero_below ? (s < 0.0f ? 0.0f : tab[0]) : tab[0];
  if (s >= (float)(n - 1)) {
    ++range;
    return tab[n - 1];
  }
  const int i = (int)floorf(s);
  const float w = s - (float)i;
  return (1.0f - w) * tab[i] + w * tab[i + 1];
}

template <int FK>
__global__ __launch_bounds__(256) void k_lepton_f32(StepArgs a) {
  extern __shared__ double smem[];
  double* sred = smem;
  unsigned* sredu = (unsigned*)(sred + 16 * 3);
  float* sh = (float*)(sredu + 16 * 5);
  for (int i = threadIdx.x; i < a.tb.n_eta; i += blockDim.x) sh[i] = a.tb.h32[i];
  __syncthreads();

  const int64_t step = a.glob->step_cur;
  const double t = a.sc.t0 + (double)step * a.sc.dt;
  const float dt = (float)a.sc.dt;
  const int64_t nch = a.glob->n_chunks[0];
  const int B = blockDim.x;
  const int64_t CH = (int64_t)B * a.ppt;
  const bool emit = (a.sc.flags & QED_EMIT) != 0;
  const float agdt = (float)(a.sc.a_gamma * a.sc.dt);

  for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    int lo_ = 0, hi_ = a.n_base - 1;
    while (lo_ < hi_) {
      const int mid = (lo_ + hi_ + 1) >> 1;
      if (a.base[mid] <= c) lo_ = mid; else hi_ = mid - 1;
    }
    const int idx = lo_;
    const int ii = idx >> 1, sp = idx & 1;
    const qed_instance& I = a.inst[ii];
    const qed_species& S = I.s[sp];
    const qed_species& G = I.s[2];
    const int64_t n = a.acc[ii].n_start[sp];
    const int64_t k0 = (c - a.base[idx]) * CH;
    const float hq = (float)(0.5 * (sp == 0 ? -1.0 : 1.0) * a.sc.kappa * a.sc.dt);
    const bool d3 = I.dims == 3;
    float* X = (float*)S.x_dev;
    float* Y = (float*)S.y_dev;
    float* Z = (float*)S.z_dev;
    float* UX = (float*)S.ux_dev;
    float* UY = (float*)S.uy_dev;
    float* UZ = (float*)S.uz_dev;

    double dacc[3] = {0.0, 0.0, 0.0};
    unsigned uacc[5] = {0, 0, 0, 0, 0};

    for (int j = 0; j < a.ppt; ++j) {
      const int64_t k = k0 + (int64_t)j * B + threadIdx.x;
      const bool active = k < n;
      bool child = false;
      double cx = 0, cy = 0, cz = 0;
      float ckx = 0, cky = 0, ckz = 0;
      double ctau = 0;
      uint64_t cuid = 0;
      if (active) {
        float xh = X[k], xl = S.x_lo_dev[k], yh = Y[k], yl = S.y_lo_dev[k];
        float zh = d3 ? Z[k] : 0.0f, zl = d3 ? S.z_lo_dev[k] : 0.0f;
        float uxh = UX[k], uxl = S.ux_lo_dev[k], uyh = UY[k], uyl = S.uy_lo_dev[k], uzh = UZ[k], uzl = S.uz_lo_dev[k];
        double tau = S.tau_dev[k];
        const double ux0 = (double)uxh + uxl, uy0 = (double)uyh + uyl, uz0 = (double)uzh + uzl;
        const double g0d = sqrt(1.0 + (ux0 * ux0 + uy0 * uy0 + uz0 * uz0));
        float E[3], Bf[3];
        field_at32<FK>(I.field, (double)xh + xl, (double)yh + yl, t, E, Bf);
        // Boris push in FP32 on the high words; the increment is added with compensation
        const float umx = uxh + hq * E[0], umy = uyh + hq * E[1], umz = uzh + hq * E[2];
        const float gm = sqrtf(1.0f + (umx * umx + umy * umy + umz * umz));
        const float tx = hq / gm * Bf[0], ty = hq / gm * Bf[1], tz = hq / gm * Bf[2];
        const float sf = 2.0f / (1.0f + (tx * tx + ty * ty + tz * tz));
        const float sx = sf * tx, sy = sf * ty, sz = sf * tz;
        const float upx = umx + (umy * tz - umz * ty), upy = umy + (umz * tx - umx * tz),
                    upz = umz + (umx * ty - umy * tx);
        // rotation increment (u+ - u-) formed directly, without cancellation
        const float rx = upy * sz - upz * sy, ry = upz * sx - upx * sz, rz = upx * sy - upy * sx;
        comp_add(uxh, uxl, 2.0f * hq * E[0] + rx);
        comp_add(uyh, uyl, 2.0f * hq * E[1] + ry);
        comp_add(uzh, uzl, 2.0f * hq * E[2] + rz);
        const float g1 = sqrtf(1.0f + (uxh * uxh + uyh * uyh + uzh * uzh));
        comp_add(xh, xl, dt * uxh / g1);
        comp_add(yh, yl, dt * uyh / g1);
        if (d3) comp_add(zh, zl, dt * uzh / g1);
        // field work from the stored states (FP64), so the ledger closes on what is stored
        double ux1 = (double)uxh + uxl, uy1 = (double)uyh + uyl, uz1 = (double)uzh + uzl;
        const double g1d = sqrt(1.0 + (ux1 * ux1 + uy1 * uy1 + uz1 * uz1));
        dacc[0] += g1d - g0d;
        if (emit) {
          const float ax = g1 * E[0] + (uyh * Bf[2] - uzh * Bf[1]);
          const float ay = g1 * E[1] + (uzh * Bf[0] - uxh * Bf[2]);
          const float az = g1 * E[2] + (uxh * Bf[1] - uyh * Bf[0]);
          const float ue = uxh * E[0] + uyh * E[1] + uzh * E[2];
          const float r2 = (ax * ax + ay * ay + az * az) - ue * ue;
          const float eta = sqrtf(r2 > 0.0f ? r2 : 0.0f);
          if (eta > 0.0f) {
            const float h = lookup32(sh, a.tb.n_eta, a.tb.le0, a.tb.dle, eta, uacc[2], false);
            tau -= (double)(agdt * (eta / g1) * h);
            if (tau <= 0.0) {
              uint64_t r[4];
              philox4x64_10(S.uid_dev[k], (uint64_t)step, KIND_EMIT, 0, I.seed, I.key_instance, r);
              double chi;
              const double etad = (double)eta;
              if (sample_chi(a.tb, etad, unit_open(r[0]), &chi)) {
                const double xi = 2.0 * chi / etad;
                ckx = (float)(xi * ux1);
                cky = (float)(xi * uy1);
                ckz = (float)(xi * uz1);
                // recoil: the emitter loses exactly the stored photon momentum
                ux1 -= (double)ckx;
                uy1 -= (double)cky;
                uz1 -= (double)ckz;
                split_double(ux1, uxh, uxl);
                split_double(uy1, uyh, uyl);
                split_double(uz1, uzh, uzl);
                const double u2x = (double)uxh + uxl, u2y = (double)uyh + uyl, u2z = (double)uzh + uzl;
                const double g2 = sqrt(1.0 + (u2x * u2x + u2y * u2y + u2z * u2z));
                const double eps = sqrt((double)ckx * ckx + (double)cky * cky + (double)ckz * ckz);
                dacc[1] += g2 + eps - g1d;
                child = true;
                cx = (double)xh + xl;
                cy = (double)yh + yl;
                cz = (double)zh + zl;
                ctau = optical_depth(r[3]);
                cuid = r[2];
                ++uacc[0];
              } else {
                ++uacc[1];
              }
              tau = optical_depth(r[1]);
            }
          }
        }
        if (!isfinite(tau) || !isfinite(uxh) || !isfinite(uyh) || !isfinite(uzh)) ++uacc[3];
        X[k] = xh;
        S.x_lo_dev[k] = xl;
        Y[k] = yh;
        S.y_lo_dev[k] = yl;
        if (d3) {
          Z[k] = zh;
          S.z_lo_dev[k] = zl;
        }
        UX[k] = uxh;
        S.ux_lo_dev[k] = uxl;
        UY[k] = uyh;
        S.uy_lo_dev[k] = uyl;
        UZ[k] = uzh;
        S.uz_lo_dev[k] = uzl;
        S.tau_dev[k] = tau;
      }
      const long long slot = wave_reserve(child, G.count_dev);
      if (child) {
        if (slot < G.capacity) {
          ((float*)G.x_dev)[slot] = (float)cx;
          ((float*)G.y_dev)[slot] = (float)cy;
          if (d3) ((float*)G.z_dev)[slot] = (float)cz;
          ((float*)G.ux_dev)[slot] = ckx;
          ((float*)G.uy_dev)[slot] = cky;
          ((float*)G.uz_dev)[slot] = ckz;
          G.tau_dev[slot] = ctau;
          G.uid_dev[slot] = cuid;
          G.birth_step_dev[slot] = (int32_t)(step + 1);
        } else {
          ++uacc[4];
          dacc[2] += sqrt((double)ckx * ckx + (double)cky * cky + (double)ckz * ckz);
        }
      }
    }
    block_sum(dacc, uacc, sred, sredu);
    if (threadIdx.x == 0) {
      InstAcc& A = a.acc[ii];
      if (dacc[0] != 0.0) atomicAdd(&A.work, dacc[0]);
      if (dacc[1] != 0.0) atomicAdd(&A.defect_emit, dacc[1]);
      if (dacc[2] != 0.0) atomicAdd(&A.dropped_energy, dacc[2]);
      if (uacc[0]) atomicAdd(&A.n_emit, (unsigned long long)uacc[0]);
      if (uacc[1]) atomicAdd(&A.n_null, (unsigned long long)uacc[1]);
      if (uacc[2]) atomicAdd(&A.n_range, (unsigned long long)uacc[2]);
      if (uacc[3]) atomicAdd(&A.n_nonfinite, (unsigned long long)uacc[3]);
      if (uacc[4]) atomicAdd(&A.n_dropped, (unsigned long long)uacc[4]);
    }
  }
}

}  // namespace qedk
