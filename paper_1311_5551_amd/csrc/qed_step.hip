// Per-step kernels of the QED Monte-Carlo step (Sec. 3 and 3.2 of the paper):
//   k_step_begin   snapshot of the live counts, chunk lists, device clock
//   k_grid_refresh analytic refresh of the 2-D Yee grid (grid field kind)
//   k_lepton       push + eta + emission optical depth (electrons and positrons)
//   k_emit_events  photon emission by the leptons whose optical depth reached zero
//   k_photon       ballistic photons + chi + pair optical depth
//   k_pair_events  pair creation by the photons whose optical depth reached zero
// and the auxiliary passes: optical-depth initialisation, compaction of dead photons and
// the energy-ledger reduction.
//
// Work decomposition: every species of every bound instance is cut into chunks of
// blockDim * ppt consecutive particles; a prefix array over (instance, species) maps a
// global chunk index to its particles.  Each block of a persistent grid takes a contiguous run
// of that list, so one launch serves one instance or hundreds of instances of very different
// sizes, and the counts never leave the device (the step sequence can be captured in a HIP
// graph).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#include "qed_device.h"
#include "qed_kernels.h"
#include "qed_mixed.h"

namespace qedk {

// ---------------------------------------------------------------------------
// snapshot at the start of a step or pass
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_step_begin(const qed_instance* __restrict__ inst, int n_inst,
                                                    InstAcc* __restrict__ acc, Glob* __restrict__ glob,
                                                    EvCtl* __restrict__ evc, EvCtl* __restrict__ emc,
                                                    int64_t* __restrict__ base_lep, int64_t* __restrict__ base_ph,
                                                    int chunk_lep, int chunk_ph, int advance_clock, int count_photons) {
  // each thread takes a contiguous range of instances: counts, then a block scan of the chunk
  // totals, then the chunk-list prefix of its range
  __shared__ int64_t s_lep[256], s_ph[256];
  const int per = (n_inst + blockDim.x - 1) / blockDim.x;
  const int b = min(n_inst, (int)threadIdx.x * per), e = min(n_inst, b + per);
  int64_t sl = 0, sp = 0;
  for (int i = b; i < e; ++i) {
    // the three counts are read before anything is written (one memory round trip)
    int64_t* cp[3];
    int64_t cv[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) cp[s] = inst[i].s[s].count_dev;
#pragma unroll
    for (int s = 0; s < 3; ++s) cv[s] = cp[s] ? *cp[s] : 0;
    for (int s = 0; s < 3; ++s) {
      const qed_species& S = inst[i].s[s];
      int64_t c = cv[s];
      if (cp[s]) {
        if (c > S.capacity) {
          // appends past the end were dropped (and counted) by the kernel that made them
          *cp[s] = S.capacity;
          c = S.capacity;
        }
        if (c < 0) c = 0;
      }
      acc[i].n_start[s] = c;
      if (s == 0 && advance_clock)
        for (int q = 0; q < kFixRunning; ++q) fix_normalise(acc[i].fx[q]);
      if (s == 2 && acc[i].n_front > c) acc[i].n_front = c;
      // the photon sweep's chunks start after the front, at a chunk boundary
      if (s == 2) acc[i].ph_first = acc[i].n_front / chunk_ph * chunk_ph;
      // particle-steps: leptons every step; photon slots in steps that run the photon pass
      if (advance_clock && (s < 2 || count_photons)) acc[i].particle_steps[s] += (unsigned long long)c;
      if (s < 2) sl += (c + chunk_lep - 1) / chunk_lep;
      else sp += (c - acc[i].ph_first + chunk_ph - 1) / chunk_ph;
    }
  }
  s_lep[threadIdx.x] = sl;
  s_ph[threadIdx.x] = sp;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {  // inclusive scans of the per-thread totals
    const int64_t vl = threadIdx.x >= o ? s_lep[threadIdx.x - o] : 0;
    const int64_t vp = threadIdx.x >= o ? s_ph[threadIdx.x - o] : 0;
    __syncthreads();
    s_lep[threadIdx.x] += vl;
    s_ph[threadIdx.x] += vp;
    __syncthreads();
  }
  int64_t rl = s_lep[threadIdx.x] - sl, rp = s_ph[threadIdx.x] - sp;
  for (int i = b; i < e; ++i) {
    for (int s = 0; s < 2; ++s) {
      base_lep[2 * i + s] = rl;
      rl += (acc[i].n_start[s] + chunk_lep - 1) / chunk_lep;
    }
    base_ph[i] = rp;
    rp += (acc[i].n_start[2] - acc[i].ph_first + chunk_ph - 1) / chunk_ph;
  }
  if (threadIdx.x == blockDim.x - 1) {
    glob->n_chunks[0] = s_lep[threadIdx.x];
    glob->n_chunks[1] = s_ph[threadIdx.x];
    if (advance_clock) {
      glob->step_cur = glob->step_next;
      glob->step_next = glob->step_cur + 1;
    }
    evc->count = 0;
    evc->overflow = 0;
    emc->count = 0;
    emc->overflow = 0;
  }
}

// Sets the next step.  The partition's front holds photons whose window ended before the step of
// the last compaction, and the live masks have lost the photons whose window ended before the
// last step swept; at an earlier step they may be inside their windows again, so the front is
// emptied (the next compaction rebuilds it) and the launcher rebuilds the masks at the new step.
__global__ void k_set_step(Glob* glob, InstAcc* acc, int n_inst, int64_t step) {
  if (blockIdx.x == 0 && threadIdx.x == 0) glob->step_next = step;
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) acc[i].n_front = 0;
}

// Empties the partition's front (after the photons were reordered another way: the next
// compaction sorts them all).
__global__ void k_front_clear(InstAcc* acc, int n_inst) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) acc[i].n_front = 0;
}

// largest idx with base[idx] <= c (lands on a non-empty entry; see the chunk-list layout)
__device__ __forceinline__ int find_entry(const int64_t* __restrict__ base, int n, int64_t c) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// analytic refresh of the grid: the standing wave at t^n, in FP64, stored as FP32
// ---------------------------------------------------------------------------
__global__ void k_grid_refresh(const qed_instance* __restrict__ inst, int n_inst, const Glob* __restrict__ glob,
                               StepConst sc) {
  // the wave is uniform in y: one thread per column and strip of kRows rows evaluates the two
  // column factors once and writes the strip (consecutive threads: consecutive columns)
  constexpr int kRows = 16;
  const double t = sc.t0 + (double)glob->step_cur * sc.dt;
  double st, ct;
  cr_sincos(t, &st, &ct);
  for (int ii = 0; ii < n_inst; ++ii) {
    const qed_field& F = inst[ii].field;
    if (F.kind != QED_FIELD_GRID_CP_STANDING) continue;
    const int64_t plane = (int64_t)F.nx * F.ny;
    const int64_t strips = (F.ny + kRows - 1) / kRows;
    const double e2 = 2.0 * F.p[0];
    gptr<float> g = as_global(F.grid_dev);
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < F.nx * strips;
         q += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = q % F.nx, j0 = (q / F.nx) * kRows;
      // components at x offsets 0 (Ey, Ez, Bx) and 1/2 (Ex, By, Bz)
      const double xa = F.x0 + (double)i * F.dx;
      const double xb = F.x0 + ((double)i + 0.5) * F.dx;
      const double ca = cr_cos(xa), cb = cr_sin(xb);
      const float ey = (float)(e2 * ct * ca), ez = (float)(e2 * st * ca);
      const float by = (float)(e2 * ct * cb), bz = (float)(e2 * st * cb);
      const int64_t j1 = min((int64_t)F.ny, j0 + kRows);
      for (int64_t j = j0; j < j1; ++j) {
        const int64_t c = j * F.nx + i;
        g[c] = 0.0f;              // Ex
        g[plane + c] = ey;        // Ey(i, j+1/2)
        g[2 * plane + c] = ez;    // Ez(i, j)
        g[3 * plane + c] = 0.0f;  // Bx
        g[4 * plane + c] = by;    // By(i+1/2, j)
        g[5 * plane + c] = bz;    // Bz(i+1/2, j+1/2)
      }
    }
  }
}

// ---------------------------------------------------------------------------
// leptons, both precisions.
//
// The sweep (k_lepton) pushes every electron and positron (Boris, field at the start-of-step
// position), evaluates eta and decrements the emission optical depth; a lepton whose depth
// reached zero is queued with its eta, and the emission pass (k_emit_events) samples chi,
// applies the recoil, appends the photon and draws a new depth.  In the plane-wave pulse the
// leptons outside the pulse see no field, where the Boris step reduces exactly to
// x += dt u / gamma with u and tau unchanged: the sweep does only that for them (same values
// as the full step, a third of its memory traffic).
//
// FP32-mixed form: the push, eta and h(eta) in FP32 on the high words; position and momentum
// stored as (hi, lo) FP32 pairs updated by compensated addition; tau, chi sampling, recoil and
// every ledger energy in FP64.
// ---------------------------------------------------------------------------
template <bool MIXED>
struct LepPtr {
  using Real = typename std::conditional<MIXED, float, double>::type;
  gptr<Real> x, y, z, ux, uy, uz;
  gptr<float> xl, yl, zl, uxl, uyl, uzl;
  gptr<double> tau;
};

template <int FK, int PPT, bool MIXED>
// (three waves per SIMD: the register budget of 168 that allows it costs at most a few spilled
// words in the larger instantiations, and the sweep is latency-bound)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FK == QED_FIELD_GRID_FDTD ? 1 : 3))) void k_lepton(StepArgs a) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ double smem[];
  __shared__ qed_field sF;
  __shared__ double sLog[2 * kLogTab];
  double* sh = smem;
  float* sh32 = (float*)smem;
  long long* s_ll = (long long*)(smem + a.tb.n_eta);  // 16 waves x 2 sums x 4 words
  unsigned* sredu = (unsigned*)(s_ll + 16 * 2 * 4);
  // field feedback: the current of a chunk's particles is summed in LDS over the chunk's node box
  // (3 x kDepNodes words) and added to the grid once per node
  constexpr bool DEP = FK == QED_FIELD_GRID_FDTD;
  double* const sJ = (double*)(sredu + 16 * 3);
  // deterministic radiation reaction (QED_RR_*) replaces emission; its g table takes h's place
  const bool rr = (a.sc.flags & (QED_RR_QUANTUM | QED_RR_CLASSICAL)) != 0;
  const bool rr_q = (a.sc.flags & QED_RR_QUANTUM) != 0;
  for (int i = threadIdx.x; i < a.tb.n_eta; i += blockDim.x) {
    if (rr_q) sh[i] = a.tb.g[i];
    else if (MIXED) sh32[i] = a.tb.h32[i];
    else sh[i] = a.tb.h[i];
  }
  for (int i = threadIdx.x; i < 16 * 2 * 4; i += blockDim.x) s_ll[i] = 0;
  if (!MIXED) stage_logtab(sLog);

  const int64_t step = uni64(a.glob->step_cur);
  const double t = a.sc.t0 + (double)step * a.sc.dt;
  const double dt = a.sc.dt;
  const float dtf = (float)dt;
  const int64_t nch = uni64(a.glob->n_chunks[0]);
  const int B = blockDim.x;
  const int64_t CH = (int64_t)B * PPT;
  const bool emit = (a.sc.flags & QED_EMIT) != 0;
  const double agdt = a.sc.a_gamma * dt;

  int cur = -1;  // chunk-list entry (2 instance + species) the context belongs to
  int64_t cb = 0, ce = 0, n = 0;
  LepPtr<MIXED> P{};
  bool d3 = false;
  double hq = 0.0;
  double qch = 0.0;  // charge of the species (-1 electrons, +1 positrons)
  float tpf0 = 0.0f, psif_max = 0.0f;
  FieldK fK{0.0};
  // field work and energy radiated (deterministic reaction): exact fixed-point words per wave in
  // LDS, fed with the sum of each group of 64 slots (fix_group_add), so the totals do not depend
  // on the launch shape
  long long* const fx_work = s_ll + (threadIdx.x >> 6) * 8;
  long long* const fx_rad = fx_work + 4;
  unsigned uacc[3] = {0, 0, 0};        // in-field steps, eta above the table, non-finite state
  auto flush = [&](int entry) {
    InstAcc& A = a.acc[entry >> 1];
    long long* const dst[2] = {A.fx[FX_WORK], A.fx[FX_RADIATED]};
    fix_block_flush<2>(s_ll, dst);
    block_sum_u(uacc, sredu);
    if (threadIdx.x == 0) {
      if (uacc[0]) atomicAdd(&A.n_field_lepton, (unsigned long long)uacc[0]);
      if (uacc[1]) atomicAdd(&A.n_range, (unsigned long long)uacc[1]);
      if (uacc[2]) atomicAdd(&A.n_nonfinite, (unsigned long long)uacc[2]);
    }
    uacc[0] = uacc[1] = uacc[2] = 0;
  };

  // each block takes a contiguous run of chunks, so it changes instance at most once per
  // instance boundary inside its run
  const int64_t per_block = (nch + gridDim.x - 1) / gridDim.x;
  const int64_t c_end = min(nch, (int64_t)blockIdx.x * per_block + per_block);
  // this wave's segment of the emission queue and its event count
  const int wave_id = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t q_seg = (int64_t)wave_id * (per_block * PPT * 64);
  int64_t q_run = 0;
  for (int64_t c = (int64_t)blockIdx.x * per_block; c < c_end; ++c) {
    if (c >= ce) {
      if (cur >= 0) flush(cur);
      const int idx = uni32(find_entry(a.base, a.n_base, c));
      cur = idx;
      cb = uni64(a.base[idx]);
      ce = idx + 1 < a.n_base ? uni64(a.base[idx + 1]) : nch;
      const int ii = idx >> 1, sp = idx & 1;
      const qed_instance& I = a.inst[ii];
      const qed_species& S = I.s[sp];
      P.x = as_global((Real*)uni_ptr(S.x_dev));
      P.y = as_global((Real*)uni_ptr(S.y_dev));
      P.z = as_global((Real*)uni_ptr(S.z_dev));
      P.ux = as_global((Real*)uni_ptr(S.ux_dev));
      P.uy = as_global((Real*)uni_ptr(S.uy_dev));
      P.uz = as_global((Real*)uni_ptr(S.uz_dev));
      if (MIXED) {
        P.xl = as_global(uni_ptr(S.x_lo_dev));
        P.yl = as_global(uni_ptr(S.y_lo_dev));
        P.zl = as_global(uni_ptr(S.z_lo_dev));
        P.uxl = as_global(uni_ptr(S.ux_lo_dev));
        P.uyl = as_global(uni_ptr(S.uy_lo_dev));
        P.uzl = as_global(uni_ptr(S.uz_lo_dev));
      }
      P.tau = as_global(uni_ptr(S.tau_dev));
      n = uni64(a.acc[ii].n_start[sp]);
      d3 = uni32(I.dims) == 3;
      qch = sp == 0 ? -1.0 : 1.0;
      hq = 0.5 * qch * a.sc.kappa * dt;
      __syncthreads();
      const uint64_t* src = (const uint64_t*)&I.field;
      for (int w = threadIdx.x; w < (int)(sizeof(qed_field) / 8); w += B) ((uint64_t*)&sF)[w] = src[w];
      __syncthreads();
      tpf0 = (float)sF.p[2];
      psif_max = (float)sF.p[1];
      fK.pi_over_len = uni_f64(field_k(sF).pi_over_len);
    }
    const int64_t k0 = uni64((c - cb) * CH);
    const int64_t rem = n - k0;
    // buffer resources over the chunk's live slots (uniform); lane offsets in bytes
    const uint32_t nlive = (uint32_t)(rem < CH ? rem : CH);
    const uint32_t rb = nlive * (uint32_t)sizeof(Real);
    struct {
      bufres x, y, z, ux, uy, uz, xl, yl, zl, uxl, uyl, uzl, tau;
    } C;
    C.x = make_buf(P.x + k0, rb);
    C.y = make_buf(P.y + k0, rb);
    C.z = make_buf(P.z + k0, d3 ? rb : 0u);
    C.ux = make_buf(P.ux + k0, rb);
    C.uy = make_buf(P.uy + k0, rb);
    C.uz = make_buf(P.uz + k0, rb);
    if (MIXED) {
      C.xl = make_buf(P.xl + k0, nlive * 4u);
      C.yl = make_buf(P.yl + k0, nlive * 4u);
      C.zl = make_buf(P.zl + k0, d3 ? nlive * 4u : 0u);
      C.uxl = make_buf(P.uxl + k0, nlive * 4u);
      C.uyl = make_buf(P.uyl + k0, nlive * 4u);
      C.uzl = make_buf(P.uzl + k0, nlive * 4u);
    }
    C.tau = make_buf(P.tau + k0, nlive * 8u);
    constexpr uint32_t SR = sizeof(Real);

    // field feedback: the box of cells holding the chunk's particles (before the push; a move
    // stays within a cell of it, and the deposit stencil spans cells I - 1 .. I + 2); where its
    // nodes fit the LDS budget, the chunk deposits there, else straight to the grid
    DepositSink sink;
    if constexpr (DEP) {
      __shared__ int sbox[4];
      if (threadIdx.x == 0) {
        sbox[0] = INT_MAX;
        sbox[1] = INT_MIN;
        sbox[2] = INT_MAX;
        sbox[3] = INT_MIN;
      }
      __syncthreads();
      int lx0 = INT_MAX, lx1 = INT_MIN, ly0 = INT_MAX, ly1 = INT_MIN;
      for (int j = 0; j < PPT; ++j) {
        const unsigned off = threadIdx.x + j * B;
        if ((int64_t)off >= rem) continue;
        const double gx = ((double)buf_ld<Real>(C.x, off * SR) - sF.x0) / sF.dx;
        const double gy = ((double)buf_ld<Real>(C.y, off * SR) - sF.y0) / sF.dy;
        if (fabs(gx) < 1e9 && fabs(gy) < 1e9) {
          const int ix = (int)floor(gx), iy = (int)floor(gy);
          lx0 = min(lx0, ix);
          lx1 = max(lx1, ix);
          ly0 = min(ly0, iy);
          ly1 = max(ly1, iy);
        } else {  // far or non-finite: the chunk takes the global path
          lx0 = INT_MIN;
          lx1 = INT_MAX;
        }
      }
      atomicMin(&sbox[0], lx0);
      atomicMax(&sbox[1], lx1);
      atomicMin(&sbox[2], ly0);
      atomicMax(&sbox[3], ly1);
      __syncthreads();
      const int bx0 = sbox[0], bx1 = sbox[1], by0 = sbox[2], by1 = sbox[3];
      __syncthreads();  // every thread has read the box before thread 0 resets it for the next chunk
      if (bx0 <= bx1 && by0 <= by1 && bx0 != INT_MIN && bx1 != INT_MAX) {
        const int64_t W = (int64_t)bx1 - bx0 + 4, H = (int64_t)by1 - by0 + 4;
        if (W * H <= kDepNodes) {
          sink.lds = sJ;
          sink.ox = (int64_t)bx0 - 1;
          sink.oy = (int64_t)by0 - 1;
          sink.W = (int)W;
          sink.H = (int)H;
          for (int i = threadIdx.x; i < 3 * W * H; i += B) sJ[i] = 0.0;
          __syncthreads();
        }
      }
    }

    // position and momentum of one lepton (slots past the chunk's live ones read as zero)
    struct LepState {
      Real x, y, z, ux, uy, uz;
      float xl, yl, zl, uxl, uyl, uzl;  // FP32-mixed low words
    };
    auto load_state = [&](unsigned off) -> LepState {
      LepState st;
      st.x = buf_ld<Real>(C.x, off * SR);
      st.y = buf_ld<Real>(C.y, off * SR);
      st.z = d3 ? buf_ld<Real>(C.z, off * SR) : Real(0);
      st.ux = buf_ld<Real>(C.ux, off * SR);
      st.uy = buf_ld<Real>(C.uy, off * SR);
      st.uz = buf_ld<Real>(C.uz, off * SR);
      if (MIXED) {
        st.xl = buf_ld<float>(C.xl, off * 4u);
        st.yl = buf_ld<float>(C.yl, off * 4u);
        st.zl = d3 ? buf_ld<float>(C.zl, off * 4u) : 0.0f;
        st.uxl = buf_ld<float>(C.uxl, off * 4u);
        st.uyl = buf_ld<float>(C.uyl, off * 4u);
        st.uzl = buf_ld<float>(C.uzl, off * 4u);
      } else {
        st.xl = st.yl = st.zl = st.uxl = st.uyl = st.uzl = 0.0f;
      }
      return st;
    };
    // field-free drift of one lepton (outside the plane-wave pulse the Boris step reduces
    // exactly to x += dt u / gamma, with u and tau unchanged)
    auto drift = [&](unsigned off, const LepState& st) {
      if (!MIXED) {
        const double g1 = sqrt(1.0 + (st.ux * st.ux + st.uy * st.uy + st.uz * st.uz));
        buf_st(C.x, off * SR, (Real)(st.x + dt * st.ux / g1));
        buf_st(C.y, off * SR, (Real)(st.y + dt * st.uy / g1));
        if (d3) buf_st(C.z, off * SR, (Real)(st.z + dt * st.uz / g1));
        if (!isfinite(g1)) ++uacc[2];
      } else {
        const float g1 = sqrtf(1.0f + ((float)st.ux * (float)st.ux + (float)st.uy * (float)st.uy +
                                       (float)st.uz * (float)st.uz));
        float xh = (float)st.x, xlo = st.xl, yh = (float)st.y, ylo = st.yl;
        comp_add(xh, xlo, dtf * (float)st.ux / g1);
        comp_add(yh, ylo, dtf * (float)st.uy / g1);
        buf_st(C.x, off * SR, (Real)xh);
        buf_st(C.xl, off * 4u, xlo);
        buf_st(C.y, off * SR, (Real)yh);
        buf_st(C.yl, off * 4u, ylo);
        if (d3) {
          float zh = (float)st.z, zlo = st.zl;
          comp_add(zh, zlo, dtf * (float)st.uz / g1);
          buf_st(C.z, off * SR, (Real)zh);
          buf_st(C.zl, off * 4u, zlo);
        }
        if (!isfinite(g1)) ++uacc[2];
      }
    };
    // full step of one lepton; returns true (and its eta) when its optical depth reached zero
    auto full = [&](unsigned off, const LepState& st, double* eta_out, double* wk, double* rd) -> bool {
      bool pend = false;
      if (!MIXED) {
        double x = st.x, y = st.y, z = st.z;
        const double ux = st.ux, uy = st.uy, uz = st.uz;
        double tau = buf_ld<double>(C.tau, off * 8u);
        double E[3], Bf[3];
        field_at<FK>(sF, x, y, t, E, Bf);
        const double g0 = sqrt(1.0 + (ux * ux + uy * uy + uz * uz));
        const double umx = ux + hq * E[0], umy = uy + hq * E[1], umz = uz + hq * E[2];
        const double gm = sqrt(1.0 + (umx * umx + umy * umy + umz * umz));
        const double tx = hq / gm * Bf[0], ty = hq / gm * Bf[1], tz = hq / gm * Bf[2];
        const double sf = 2.0 / (1.0 + (tx * tx + ty * ty + tz * tz));
        const double sx = sf * tx, sy = sf * ty, sz = sf * tz;
        const double upx = umx + (umy * tz - umz * ty), upy = umy + (umz * tx - umx * tz),
                     upz = umz + (umx * ty - umy * tx);
        const double ulx = umx + (upy * sz - upz * sy), uly = umy + (upz * sx - upx * sz),
                     ulz = umz + (upx * sy - upy * sx);
        const double u1x = ulx + hq * E[0], u1y = uly + hq * E[1], u1z = ulz + hq * E[2];
        const double g1 = sqrt(1.0 + (u1x * u1x + u1y * u1y + u1z * u1z));
        *wk = 2.0 * hq * (E[0] * (ulx + umx) + E[1] * (uly + umy) + E[2] * (ulz + umz)) / (g1 + g0);
        x += dt * u1x / g1;
        y += dt * u1y / g1;
        if (d3) z += dt * u1z / g1;
        // field feedback: the current of this move onto the solver's grid (or the chunk's LDS box)
        if constexpr (DEP) deposit_current(sF, qch * sF.p[0], dt, st.x, st.y, x, y, u1z / g1, sink);
        double wx = u1x, wy = u1y, wz = u1z;  // stored momentum
        if (rr) {
          // continuous reaction (eqs. 8, 9): gamma -> max(gamma - (2/3) alpha kappa eta^2 g dt, 1)
          // along u; the energy removed is what the stored momentum lost
          const double ax = g1 * E[0] + (u1y * Bf[2] - u1z * Bf[1]);
          const double ay = g1 * E[1] + (u1z * Bf[0] - u1x * Bf[2]);
          const double az = g1 * E[2] + (u1x * Bf[1] - u1y * Bf[0]);
          const double ue = u1x * E[0] + u1y * E[1] + u1z * E[2];
          const double r2 = (ax * ax + ay * ay + az * az) - ue * ue;
          const double eta = sqrt(r2 > 0.0 ? r2 : 0.0);
          if (eta > 0.0) {
            const double gq = rr_q ? lookup_g(sh, a.tb, eta, uacc[1]) : 1.0;
            const double gn = fmax(g1 - a.sc.a_rr * eta * eta * gq * dt, 1.0);
            const double um = sqrt(u1x * u1x + u1y * u1y + u1z * u1z);
            const double sc = um > 0.0 ? sqrt((gn - 1.0) * (gn + 1.0)) / um : 0.0;
            wx = sc * u1x;
            wy = sc * u1y;
            wz = sc * u1z;
            *rd = g1 - sqrt(1.0 + (wx * wx + wy * wy + wz * wz));
          }
        }
        if (emit) {
          const double ax = g1 * E[0] + (u1y * Bf[2] - u1z * Bf[1]);
          const double ay = g1 * E[1] + (u1z * Bf[0] - u1x * Bf[2]);
          const double az = g1 * E[2] + (u1x * Bf[1] - u1y * Bf[0]);
          const double ue = u1x * E[0] + u1y * E[1] + u1z * E[2];
          const double r2 = (ax * ax + ay * ay + az * az) - ue * ue;
          const double eta = sqrt(r2 > 0.0 ? r2 : 0.0);
          if (eta > 0.0) {
            const double h = lookup_h(sh, sLog, a.tb, eta, uacc[1]);
            tau -= a.sc.a_gamma * (eta / g1) * h * dt;
            if (tau <= 0.0) {
              pend = true;
              *eta_out = eta;
            }
          }
        }
        if (!isfinite(tau) || !isfinite(wx) || !isfinite(wy) || !isfinite(wz)) ++uacc[2];
        buf_st(C.x, off * SR, (Real)(x));
        buf_st(C.y, off * SR, (Real)(y));
        if (d3) buf_st(C.z, off * SR, (Real)(z));
        buf_st(C.ux, off * SR, (Real)(wx));
        buf_st(C.uy, off * SR, (Real)(wy));
        buf_st(C.uz, off * SR, (Real)(wz));
        buf_st(C.tau, off * 8u, (double)(tau));
      } else {
        float xh = st.x, xl = st.xl, yh = st.y, yl = st.yl, zh = st.z, zl = st.zl;
        float uxh = st.ux, uxl = st.uxl, uyh = st.uy, uyl = st.uyl, uzh = st.uz, uzl = st.uzl;
        double tau = buf_ld<double>(C.tau, off * 8u);
        const double ux0 = (double)uxh + uxl, uy0 = (double)uyh + uyl, uz0 = (double)uzh + uzl;
        const double g0d = sqrt(1.0 + (ux0 * ux0 + uy0 * uy0 + uz0 * uz0));
        float E[3], Bf[3];
        field_at32<FK>(sF, fK, (double)xh + xl, (double)yh + yl, t, E, Bf);
        const float hqf = (float)hq;
        const float umx = uxh + hqf * E[0], umy = uyh + hqf * E[1], umz = uzh + hqf * E[2];
        const float gm = sqrtf(1.0f + (umx * umx + umy * umy + umz * umz));
        const float tx = hqf / gm * Bf[0], ty = hqf / gm * Bf[1], tz = hqf / gm * Bf[2];
        const float sf = 2.0f / (1.0f + (tx * tx + ty * ty + tz * tz));
        const float sx = sf * tx, sy = sf * ty, sz = sf * tz;
        const float upx = umx + (umy * tz - umz * ty), upy = umy + (umz * tx - umx * tz),
                    upz = umz + (umx * ty - umy * tx);
        // rotation increment (u+ - u-) formed directly, without cancellation
        const float rx = upy * sz - upz * sy, ry = upz * sx - upx * sz, rz = upx * sy - upy * sx;
        comp_add(uxh, uxl, 2.0f * hqf * E[0] + rx);
        comp_add(uyh, uyl, 2.0f * hqf * E[1] + ry);
        comp_add(uzh, uzl, 2.0f * hqf * E[2] + rz);
        const float g1 = sqrtf(1.0f + (uxh * uxh + uyh * uyh + uzh * uzh));
        comp_add(xh, xl, dtf * uxh / g1);
        comp_add(yh, yl, dtf * uyh / g1);
        if (d3) comp_add(zh, zl, dtf * uzh / g1);
        // field work from the stored states (FP64), so the ledger closes on what is stored
        const double ux1 = (double)uxh + uxl, uy1 = (double)uyh + uyl, uz1 = (double)uzh + uzl;
        const double g1d = sqrt(1.0 + (ux1 * ux1 + uy1 * uy1 + uz1 * uz1));
        *wk = g1d - g0d;
        if (rr) {
          // continuous reaction with eta in FP32 (as for emission) and the energy update in
          // FP64 on the stored momentum; the energy removed is what the stored pairs lost
          const float ax = g1 * E[0] + (uyh * Bf[2] - uzh * Bf[1]);
          const float ay = g1 * E[1] + (uzh * Bf[0] - uxh * Bf[2]);
          const float az = g1 * E[2] + (uxh * Bf[1] - uyh * Bf[0]);
          const float ue = uxh * E[0] + uyh * E[1] + uzh * E[2];
          const float r2 = (ax * ax + ay * ay + az * az) - ue * ue;
          const double eta = (double)sqrtf(r2 > 0.0f ? r2 : 0.0f);
          if (eta > 0.0) {
            const double gq = rr_q ? lookup_g(sh, a.tb, eta, uacc[1]) : 1.0;
            const double gn = fmax(g1d - a.sc.a_rr * eta * eta * gq * dt, 1.0);
            const double um = sqrt(ux1 * ux1 + uy1 * uy1 + uz1 * uz1);
            const double sc = um > 0.0 ? sqrt((gn - 1.0) * (gn + 1.0)) / um : 0.0;
            split_double(sc * ux1, uxh, uxl);
            split_double(sc * uy1, uyh, uyl);
            split_double(sc * uz1, uzh, uzl);
            const double vx = (double)uxh + uxl, vy = (double)uyh + uyl, vz = (double)uzh + uzl;
            *rd = g1d - sqrt(1.0 + (vx * vx + vy * vy + vz * vz));
          }
        }
        if (emit) {
          const float ax = g1 * E[0] + (uyh * Bf[2] - uzh * Bf[1]);
          const float ay = g1 * E[1] + (uzh * Bf[0] - uxh * Bf[2]);
          const float az = g1 * E[2] + (uxh * Bf[1] - uyh * Bf[0]);
          const float ue = uxh * E[0] + uyh * E[1] + uzh * E[2];
          const float r2 = (ax * ax + ay * ay + az * az) - ue * ue;
          const float eta = sqrtf(r2 > 0.0f ? r2 : 0.0f);
          if (eta > 0.0f) {
            const float h = lookup32(sh32, a.tb.n_eta, a.tb.le0, a.tb.idle, eta, uacc[1], false);
            tau -= agdt * ((double)eta / (double)g1) * (double)h;  // FP32 look-up, FP64 decrement
            if (tau <= 0.0) {
              pend = true;
              *eta_out = (double)eta;
            }
          }
        }
        if (!isfinite(tau) || !isfinite(uxh) || !isfinite(uyh) || !isfinite(uzh)) ++uacc[2];
        buf_st(C.x, off * SR, (Real)(xh));
        buf_st(C.xl, off * 4u, (float)(xl));
        buf_st(C.y, off * SR, (Real)(yh));
        buf_st(C.yl, off * 4u, (float)(yl));
        if (d3) {
          buf_st(C.z, off * SR, (Real)(zh));
          buf_st(C.zl, off * 4u, (float)(zl));
        }
        buf_st(C.ux, off * SR, (Real)(uxh));
        buf_st(C.uxl, off * 4u, (float)(uxl));
        buf_st(C.uy, off * SR, (Real)(uyh));
        buf_st(C.uyl, off * 4u, (float)(uyl));
        buf_st(C.uz, off * SR, (Real)(uzh));
        buf_st(C.uzl, off * 4u, (float)(uzl));
        buf_st(C.tau, off * 8u, (double)(tau));
      }
      return pend;
    };
    auto enqueue = [&](unsigned off, bool pend, double eta) {
      // into the wave's own segment of the queue (EmitQueue): no atomics, no barriers.  (Atomics
      // on one device-wide counter serialise at ~10 ns each, and there is an event in nearly every
      // wave during a collision.)
      const unsigned long long m = __ballot(pend);
      if (pend) {
        const int64_t slot = q_seg + q_run + __popcll(m & ((1ull << __lane_id()) - 1ull));
        if (slot < a.qe.cap) {
          a.qe.ent[slot].key = ((uint64_t)(cur >> 1) << 41) | ((uint64_t)(cur & 1) << 40) | (uint64_t)(k0 + off);
          a.qe.ent[slot].eta = eta;
        } else {
          a.qe.ctl->overflow = 1;  // cannot happen: the queue holds one entry per lepton slot
        }
      }
      q_run += __popcll(m);
    };

    if (FK == QED_FIELD_LP_PULSE) {
      // outside the pulse (an FP32 test of the phase with a margin far above its rounding error)
      // the drift, inside it the full step
      const float tpf = (float)t - tpf0;
      const float mt = fabsf((float)t) + fabsf(tpf0);
#pragma unroll 1
      for (int j = 0; j < PPT; ++j) {
        const unsigned off = threadIdx.x + j * B;
        bool pend = false, in = false;
        double eta = 0.0, wk = 0.0, rd = 0.0;
        if ((int64_t)off < rem) {
          const LepState st = load_state(off);
          const float xf = (float)st.x;
          const float psif = tpf - xf;
          const float m = 1e-5f * (mt + fabsf(xf)) + 1e-30f;
          in = psif >= -m && psif <= psif_max + m;
          if (in) {
            ++uacc[0];
            pend = full(off, st, &eta, &wk, &rd);
          } else {
            drift(off, st);
          }
        }
        if (__ballot(in)) {  // wave-uniform: the energy sums of the wave's group of 64 slots
          fix_group_add(wk, fx_work);
          if (rr) fix_group_add(rd, fx_rad);
        }
        if (emit) enqueue(off, pend, eta);  // emit is uniform over the block
      }
    } else {
#pragma unroll 1
      for (int j = 0; j < PPT; ++j) {
        const unsigned off = threadIdx.x + j * B;
        bool pend = false;
        double eta = 0.0, wk = 0.0, rd = 0.0;
        const bool in = (int64_t)off < rem;
        if (in) {
          ++uacc[0];
          pend = full(off, load_state(off), &eta, &wk, &rd);
        }
        if (__ballot(in)) {
          fix_group_add(wk, fx_work);
          if (rr) fix_group_add(rd, fx_rad);
        }
        if (emit) enqueue(off, pend, eta);  // emit is uniform over the block
      }
    }
    if constexpr (DEP) {
      if (sink.W) {  // block-uniform: the box's sums onto the grid, one atomic per non-zero node
        __syncthreads();
        const int64_t WH = (int64_t)sink.W * sink.H, plane = (int64_t)sF.nx * sF.ny;
        for (int64_t i = threadIdx.x; i < 3 * WH; i += B) {
          const double v = sJ[i];
          if (v == 0.0) continue;
          const int comp = (int)(i / WH);
          const int64_t r = i - comp * WH, ly = r / sink.W, lx = r - ly * sink.W;
          const int64_t gi = wrap_index(sink.ox + lx, sF.nx), gj = wrap_index(sink.oy + ly, sF.ny);
          unsafeAtomicAdd(sF.fdtd_dev + (6 + comp) * plane + gj * sF.nx + gi, v);
        }
        __syncthreads();  // the box is zeroed again by the next chunk
      }
    }
  }
  if (cur >= 0) flush(cur);
  if (emit && (threadIdx.x & 63) == 0) a.qe.wave_cnt[wave_id] = (int32_t)q_run;
}

// Emission by the queued leptons: chi from the 2-D inverse CDF at the emitter's eta, photon
// momentum (2 chi / eta) u along the emitter's momentum, recoil, photon appended at the
// emitter's post-push position (born at the start of the next step), new optical depth.
//
// The events sit in the lepton sweep's per-wave segments (EmitQueue); every block forms the prefix
// of the per-wave counts in LDS and takes a contiguous range of the events.  A round whose events
// all belong to one instance (the usual case: the segments follow the chunk list, which is ordered
// by instance) reserves its photon slots and adds its statistics with one atomic per block; rounds
// across instances use per-wave atomics.
template <int FK, bool MIXED>
__global__ __launch_bounds__(256) void k_emit_events(StepArgs a) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ int s_pref[];                  // per-wave event counts, then their prefix
  __shared__ int s_scan[256];
  __shared__ int s_key[48];
  __shared__ unsigned s_wave[16];
  __shared__ long long s_base;
  __shared__ long long s_ll[16 * 8];
  __shared__ unsigned s_u[16 * 3];
  const int64_t step = a.glob->step_cur;
  const int NW = a.qe.grid * a.qe.waves;
  const int64_t nch = a.glob->n_chunks[0];
  const int64_t seg_len = (nch + a.qe.grid - 1) / a.qe.grid * a.qe.ppt * 64;
  // exclusive prefix of the per-wave counts: the counts land in LDS from coalesced loads that are
  // all in flight together (32 per thread: the 8192 waves of 256 CUs in one memory round trip),
  // then thread t sums a contiguous run, a block scan of the run totals, then the run's prefixes
  {
    constexpr int kRound = 32;
    for (int i0 = 0; i0 < NW; i0 += kRound * (int)blockDim.x) {
      int v[kRound];
#pragma unroll
      for (int j = 0; j < kRound; ++j) {
        const int i = i0 + (int)threadIdx.x + j * (int)blockDim.x;
        v[j] = i < NW ? a.qe.wave_cnt[i] : 0;
      }
#pragma unroll
      for (int j = 0; j < kRound; ++j) {
        const int i = i0 + (int)threadIdx.x + j * (int)blockDim.x;
        if (i < NW) s_pref[i] = v[j];
      }
    }
    __syncthreads();
    const int per = (NW + blockDim.x - 1) / blockDim.x;
    const int b = min(NW, (int)threadIdx.x * per), e = min(NW, b + per);
    int loc = 0;
    for (int i = b; i < e; ++i) loc += s_pref[i];
    s_scan[threadIdx.x] = loc;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      const int v = threadIdx.x >= o ? s_scan[threadIdx.x - o] : 0;
      __syncthreads();
      s_scan[threadIdx.x] += v;
      __syncthreads();
    }
    int run = s_scan[threadIdx.x] - loc;
    for (int i = b; i < e; ++i) {
      const int c = s_pref[i];
      s_pref[i] = run;
      run += c;
    }
    if (threadIdx.x == blockDim.x - 1) s_pref[NW] = s_scan[threadIdx.x];
    __syncthreads();
  }
  const int total = s_pref[NW];
  // the blocks that take events: as many as one round of blockDim events each needs, up to the
  // grid; the others leave now, so a step with few events pays no atomics on the shared
  // counters for blocks without work
  const int G = max(1, min((int)gridDim.x, (total + (int)blockDim.x - 1) / (int)blockDim.x));
  if ((int)blockIdx.x >= G) return;
  const int per = (total + G - 1) / G;
  const int eb = min(total, (int)blockIdx.x * per), ee = min(total, eb + per);
  BlockEventStats bst;
  bst.clear();
  for (int e0 = eb; e0 < ee; e0 += blockDim.x) {  // block-uniform trip count
    const int e = e0 + (int)threadIdx.x;
    const bool want = e < ee;
    EmitEv ev{0, 0.0};
    if (want) {
      int lo = 0, hi = NW - 1;  // the last wave segment whose prefix is <= e
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pref[mid] <= e) lo = mid; else hi = mid - 1;
      }
      ev = a.qe.ent[(int64_t)lo * seg_len + (e - s_pref[lo])];
    }
    const int ii = (int)(ev.key >> 41), sp = (int)((ev.key >> 40) & 1);
    const int64_t k = (int64_t)(ev.key & ((1ull << 40) - 1));
    int bkey = 0;
    const bool uni = block_uniform_key(want, ii, s_key, &bkey);  // block-uniform
    // everything the event reads besides the tables, loaded before its first store (which the
    // compiler cannot tell apart from these words), so that the loads share a memory round trip
    const qed_instance& I = a.inst[ii];
    const qed_species S = I.s[sp], G = I.s[2];
    const qed_field F = I.field;
    const uint64_t seed = I.seed, key_inst = I.key_instance;
    const bool d3 = I.dims == 3;
    const int64_t moff = a.acc[ii].mover_off, lmoff = a.acc[ii].lmask_off;
    int64_t* const bcount = a.inst[bkey].s[2].count_dev;
    bool child = false;
    double defect = 0.0, cx = 0, cy = 0, cz = 0, ckx = 0, cky = 0, ckz = 0, ctau = 0;
    uint64_t cuid = 0;
    unsigned n_null = 0;
    if (want) {
      const uint64_t uid = S.uid_dev[k];
      gptr<Real> UX = as_global((Real*)S.ux_dev), UY = as_global((Real*)S.uy_dev), UZ = as_global((Real*)S.uz_dev);
      double ux1, uy1, uz1;
      if (MIXED) {
        ux1 = (double)UX[k] + S.ux_lo_dev[k];
        uy1 = (double)UY[k] + S.uy_lo_dev[k];
        uz1 = (double)UZ[k] + S.uz_lo_dev[k];
        cx = (double)((const float*)S.x_dev)[k] + S.x_lo_dev[k];
        cy = (double)((const float*)S.y_dev)[k] + S.y_lo_dev[k];
        cz = d3 ? (double)((const float*)S.z_dev)[k] + S.z_lo_dev[k] : 0.0;
      } else {
        ux1 = UX[k];
        uy1 = UY[k];
        uz1 = UZ[k];
        cx = ((const double*)S.x_dev)[k];
        cy = ((const double*)S.y_dev)[k];
        cz = d3 ? ((const double*)S.z_dev)[k] : 0.0;
      }
      uint64_t r[4];
      philox4x64_10(uid, (uint64_t)step, KIND_EMIT, 0, seed, key_inst, r);
      const double g1 = sqrt(1.0 + (ux1 * ux1 + uy1 * uy1 + uz1 * uz1));
      double chi;
      if (sample_chi(a.tb, ev.eta, unit_open(r[0]), &chi)) {
        const double xi = 2.0 * chi / ev.eta;
        double ux, uy, uz;
        if (MIXED) {
          // the emitter loses exactly the stored (FP32) photon momentum
          ckx = (float)(xi * ux1);
          cky = (float)(xi * uy1);
          ckz = (float)(xi * uz1);
          float h, l;
          split_double(ux1 - ckx, h, l); UX[k] = h; S.ux_lo_dev[k] = l; ux = (double)h + l;
          split_double(uy1 - cky, h, l); UY[k] = h; S.uy_lo_dev[k] = l; uy = (double)h + l;
          split_double(uz1 - ckz, h, l); UZ[k] = h; S.uz_lo_dev[k] = l; uz = (double)h + l;
        } else {
          ckx = xi * ux1;
          cky = xi * uy1;
          ckz = xi * uz1;
          ux = ux1 - ckx;
          uy = uy1 - cky;
          uz = uz1 - ckz;
          UX[k] = ux;
          UY[k] = uy;
          UZ[k] = uz;
        }
        const double g2 = sqrt(1.0 + (ux * ux + uy * uy + uz * uz));
        const double eps = sqrt(ckx * ckx + cky * cky + ckz * ckz);
        defect = g2 + eps - g1;
        child = true;
        ctau = optical_depth(r[3]);
        cuid = r[2];
      } else {
        n_null = 1;
      }
      S.tau_dev[k] = optical_depth(r[1]);
    }
    const long long slot = uni ? block_reserve(child, bcount, s_wave, &s_base)
                               : wave_reserve_grouped(child, ii, G.count_dev);
    double dropped_e = 0.0;
    unsigned n_drop = 0;
    uint64_t* lword = nullptr;  // the live mask word of a new photon that can still create a pair
    if (child) {
      if (slot < G.capacity) {
        if (MIXED) {
          ((float*)G.x_dev)[slot] = (float)cx;
          ((float*)G.y_dev)[slot] = (float)cy;
          if (d3) ((float*)G.z_dev)[slot] = (float)cz;
          ((float*)G.ux_dev)[slot] = (float)ckx;
          ((float*)G.uy_dev)[slot] = (float)cky;
          ((float*)G.uz_dev)[slot] = (float)ckz;
        } else {
          ((double*)G.x_dev)[slot] = cx;
          ((double*)G.y_dev)[slot] = cy;
          if (d3) ((double*)G.z_dev)[slot] = cz;
          ((double*)G.ux_dev)[slot] = ckx;
          ((double*)G.uy_dev)[slot] = cky;
          ((double*)G.uz_dev)[slot] = ckz;
        }
        G.tau_dev[slot] = ctau;
        G.uid_dev[slot] = cuid;
        G.birth_step_dev[slot] = (int32_t)(step + 1);
        // the steps in which the new photon can create a pair, from its stored state
        const double sx = MIXED ? (double)(float)cx : cx;
        const double skx = MIXED ? (double)(float)ckx : ckx, sky = MIXED ? (double)(float)cky : cky,
                     skz = MIXED ? (double)(float)ckz : ckz;
        const double sy = MIXED ? (double)(float)cy : cy;
        const int64_t pk = moff + slot;
        const uint32_t wn = pack_window(photon_window(F, pair_eps_min(F, a.tb.cp_min), a.tb.cp_min, a.sc.t0, a.sc.dt,
                                                      skx, sky, skz, sx, (int32_t)(step + 1)));
        a.win[pk] = wn;
        if (!window_over(wn, step + 1)) lword = a.lmask + lmoff + slot / kWinGroup;
        make_photon_rec<MIXED, FK>(((PhotonRecT<MIXED, FK>*)a.rec)[pk], F, a.sc.t0, a.sc.dt, skx, sky, skz, sx, sy,
                                   (int32_t)(step + 1));
      } else {
        n_drop = 1;
        dropped_e = sqrt(ckx * ckx + cky * cky + ckz * ckz);
      }
    }
    // the new photons' live bits (the words' other bits belong to other slots, some of them set
    // by other waves)
    wave_or_bit(lword, (int)(slot % kWinGroup));
    if (uni) {
      if (bkey != bst.inst && threadIdx.x == 0) {
        bst.flush(0, a.acc);
        bst.inst = bkey;
      }
      long long ld[4], le[4];
      fix_split(defect, ld);
      fix_split(dropped_e, le);
      bst.add(ld, le, child ? 1u : 0u, n_null, n_drop, s_ll, s_u);
    } else {
      add_event_stats(0, want, ii, a.acc, defect, dropped_e, child ? 1u : 0u, n_null, n_drop);
    }
  }
  if (threadIdx.x == 0) bst.flush(0, a.acc);
}

// ---------------------------------------------------------------------------
// photons, both precisions.  Position at the start of step n: x_b + (n - b) dt k/|k|.
//
// Each photon carries a window of steps outside which it has no pair rate (photon_window: below
// the energy that can reach chi_min in the field, or outside a pulse's support); it is set when
// the photon is appended and moves with it.  The sweep (k_photon) skips three ways: it starts
// after the front that the partition at compaction fills with photons whose window is over; it
// skips the groups of 64 slots whose live mask is empty; in the other groups a thread reads the
// window, record and optical depth of each photon it owns whose live bit is set (the live mask
// holds a bit for every photon whose window is not over, so only photons in their window, and
// the few whose window starts later, are read).  The photons inside their window evaluate chi
// and T(chi), with
// the device library's trigonometry and log, and, where T > 0, decrement the optical depth (these
// values only decide the event step).  A photon whose depth reaches zero is queued; the event
// pass (k_pair_events) recomputes chi from the stored photon with correctly rounded functions,
// samples the energy split and appends the pair.  Keeping the rare event work out of the sweep
// keeps the sweep's register footprint, and so its occupancy, at what streaming needs.
// ---------------------------------------------------------------------------
constexpr int kPhotonRun = 4;  // chunks per run of the photon sweep's round-robin deal

template <int FK, int PPT, bool MIXED>
__global__ __launch_bounds__(256) void k_photon(StepArgs a) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  constexpr bool NEED_X = FK != QED_FIELD_UNIFORM;
  constexpr bool NEED_Y = FK == QED_FIELD_GRID_CP_STANDING || FK == QED_FIELD_GRID_FDTD;
  extern __shared__ double smem[];
  __shared__ qed_field sF;  // field of the instance being processed
  __shared__ double sLog[2 * kLogTab];
  double* sT = smem;
  float* sT32 = (float*)smem;
  unsigned* sredu = (unsigned*)(smem + a.tb.n_cp);
  for (int i = threadIdx.x; i < a.tb.n_cp; i += blockDim.x) {
    if (MIXED) sT32[i] = a.tb.T32[i];
    else sT[i] = a.tb.T[i];
  }
  if (!MIXED) stage_logtab(sLog);

  const int64_t step = uni64(a.glob->step_cur);
  const double t = a.sc.t0 + (double)step * a.sc.dt;
  const double dt = a.sc.dt;
  const int64_t nch = uni64(a.glob->n_chunks[1]);
  const int B = blockDim.x;
  const int64_t CH = (int64_t)B * PPT;
  const double rate = a.sc.a_pair * dt;

  // context of the instance whose chunks the block is on (chunks [cb, ce) of the list)
  int cur = -1;
  int64_t cb = 0, ce = 0, n = 0;
  gptr<double> TAU = nullptr;
  gptr<uint32_t> WIN = nullptr;
  using Rec = PhotonRecT<MIXED, FK>;
  // dwords of a record the sweep reads: plane-wave {A, S, c}; general {k, x_b, y_b, birth step}
  constexpr int kRecDw = FK == QED_FIELD_LP_PULSE ? (MIXED ? 4 : 6) : (MIXED ? 6 : 11);
  gptr<const Rec> REC = nullptr;
  gptr<uint64_t> LM = nullptr;
  int64_t pfirst = 0;
  // live masks of the current run of chunks, one load per wave: lane r PPT + j holds the mask of
  // group j of the wave in chunk m0 + r (0 past the instance's chunks)
  int64_t m0 = -1;
  uint64_t mrun = 0;
  FieldK fK{0.0};
  // in-field steps, chi above the table, non-finite tau, in-window steps, window reads, mask reads
  unsigned uacc[6] = {0, 0, 0, 0, 0, 0};
  // the counters of the instance just left: lane sums through LDS atomics (few registers on
  // this rare path), then one global atomic per counter
  auto flush = [&](int ii) {
    if (threadIdx.x < 6) sredu[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (uacc[c]) atomicAdd(&sredu[c], uacc[c]);
    __syncthreads();
    if (threadIdx.x < 6 && sredu[threadIdx.x]) {
      InstAcc& A = a.acc[ii];
      unsigned long long* const dst[6] = {&A.n_field,  &A.n_range,     &A.n_nonfinite,
                                          &A.n_active, &A.n_win_reads, &A.n_group_reads};
      atomicAdd(dst[threadIdx.x], (unsigned long long)sredu[threadIdx.x]);
    }
    __syncthreads();  // sredu is reused by the next flush
    uacc[0] = uacc[1] = uacc[2] = uacc[3] = uacc[4] = uacc[5] = 0;
  };

  // the chunk list is dealt to the blocks in runs of kPhotonRun chunks, round robin: the photons
  // that need the in-field evaluation (the newest, at the end of the arrays) spread over all
  // blocks.  A block's chunks still only grow, so it changes instance at most once per instance
  // boundary it crosses.
  const int64_t stride = (int64_t)gridDim.x * kPhotonRun;
  for (int64_t c = (int64_t)blockIdx.x * kPhotonRun; c < nch; c += ((c + 1) % kPhotonRun) ? 1 : stride - kPhotonRun + 1) {
    if (c >= ce) {  // first chunk of another instance (c only grows)
      if (cur >= 0) flush(cur);
      const int ii = uni32(find_entry(a.base, a.n_base, c));
      cur = ii;
      cb = uni64(a.base[ii]);
      ce = ii + 1 < a.n_base ? uni64(a.base[ii + 1]) : nch;
      const qed_species& S = a.inst[ii].s[2];
      TAU = as_global(uni_ptr(S.tau_dev));
      WIN = as_global(uni_ptr(a.win)) + uni64(a.acc[ii].mover_off);
      REC = as_global((const Rec*)uni_ptr(a.rec)) + uni64(a.acc[ii].mover_off);
      LM = as_global(uni_ptr(a.lmask)) + uni64(a.acc[ii].lmask_off);
      pfirst = uni64(a.acc[ii].ph_first);
      m0 = -1;
      n = uni64(a.acc[ii].n_start[2]);
      __syncthreads();  // the previous field copy is no longer read
      const uint64_t* src = (const uint64_t*)&a.inst[ii].field;
      for (int w = threadIdx.x; w < (int)(sizeof(qed_field) / 8); w += B) ((uint64_t*)&sF)[w] = src[w];
      __syncthreads();
      fK.pi_over_len = uni_f64(field_k(sF).pi_over_len);
    }
    const int64_t k0 = uni64(pfirst + (c - cb) * CH);  // first slot of the chunk
    const int64_t rem = n - k0;               // slots of the chunk that exist: min(rem, CH)

    // buffer resources over the chunk's live slots (uniform); lane offsets in bytes
    const uint32_t nlive = (uint32_t)(rem < CH ? rem : CH);
    const bufres rtau = make_buf(TAU + k0, nlive * 8u), rwin = make_buf(WIN + k0, nlive * 4u);
    const bufres rrec = make_buf(REC + k0, nlive * (uint32_t)sizeof(Rec));
    // the optical-depth step of a photon with pair rate T > 0; true when its depth reached zero
    auto decrement = [&](unsigned off, double T, double dtau, double tau) -> bool {
      bool pend = false;
      if (T > 0.0) {
        if (!(tau < 0.0)) {  // tau < 0: converted in an earlier step
          ++uacc[0];
          tau -= dtau;
          if (tau <= 0.0) {
            pend = true;
            tau = fmax(tau, kTauPendingMin);
          }
          if (!isfinite(tau)) ++uacc[2];
          buf_st(rtau, off * 8u, tau);
        }
      }
      return pend;
    };
    // in-field part for one photon; true when its optical depth reached zero
    auto infield = [&](unsigned off, Real kx, Real ky, Real kz, Real xb, Real yb, int32_t bs, double tau) -> bool {
      const Real eps = sqrt(kx * kx + ky * ky + kz * kz);
      const Real inv = (Real)1 / eps;
      const Real nx = kx * inv, ny = ky * inv, nz = kz * inv;
      double x = 0.0, y = 0.0;
      if (NEED_X) {
        const double age = (double)(step - (int64_t)bs) * dt;
        x = (double)xb + age * nx;
        if (NEED_Y) y = (double)yb + age * ny;
      }
      double chi, T;
      if (MIXED) {
        float E[3], Bf[3];
        field_at32<FK>(sF, fK, x, y, t, E, Bf);
        const float ax = E[0] + (ny * Bf[2] - nz * Bf[1]);
        const float ay = E[1] + (nz * Bf[0] - nx * Bf[2]);
        const float az = E[2] + (nx * Bf[1] - ny * Bf[0]);
        const float ne = nx * E[0] + ny * E[1] + nz * E[2];
        const float r2 = (ax * ax + ay * ay + az * az) - ne * ne;
        const float chif = 0.5f * (float)eps * sqrtf(r2 > 0.0f ? r2 : 0.0f);
        chi = chif;
        T = lookup32(sT32, a.tb.n_cp, a.tb.lc0, a.tb.idlc, chif, uacc[1], true);
      } else {
        double E[3], Bf[3];
        field_at<FK, false>(sF, x, y, t, E, Bf, &fK);
        const double ax = E[0] + (ny * Bf[2] - nz * Bf[1]);
        const double ay = E[1] + (nz * Bf[0] - nx * Bf[2]);
        const double az = E[2] + (nx * Bf[1] - ny * Bf[0]);
        const double ne = nx * E[0] + ny * E[1] + nz * E[2];
        const double r2 = (ax * ax + ay * ay + az * az) - ne * ne;
        chi = 0.5 * (double)eps * sqrt(r2 > 0.0 ? r2 : 0.0);
        T = lookup_T(sT, sLog, a.tb, chi, uacc[1]);
      }
      return decrement(off, T, rate * chi * T * (double)inv, tau);  // FP64 (chi, T, 1/eps FP32 if mixed)
    };
    // the plane-wave pulse from the photon's record: psi(n) = A + n S, chi = c |e(psi)|, and the
    // decrement a_pair |e| T(chi) S / 2 (PhotonRecPW)
    auto infield_pw = [&](unsigned off, double A, double S, double cr, double tau) -> bool {
      const double psi = A + (double)step * S;
      double T = 0.0, ae = 0.0;
      if (psi >= 0.0 && psi <= sF.p[1]) {
        if (MIXED) {
          float sn, cs, d;
          fast_sincosf((float)(psi * fK.pi_over_len), &sn, &d);
          fast_sincosf(reduce_phase(psi + sF.p[3]), &d, &cs);
          const float e = fabsf((float)sF.p[0] * sn * sn * cs);
          ae = e;
          T = lookup32(sT32, a.tb.n_cp, a.tb.lc0, a.tb.idlc, (float)cr * e, uacc[1], true);
        } else {
          const double sn = fast_sin(psi * fK.pi_over_len), cs = fast_cos(psi + sF.p[3]);
          ae = fabs(sF.p[0] * sn * sn * cs);
          T = lookup_T(sT, sLog, a.tb, cr * ae, uacc[1]);
        }
      }
      return decrement(off, T, 0.5 * a.sc.a_pair * ae * T * S, tau);
    };
    auto enqueue = [&](unsigned off, bool pend) {
      const long long slot = wave_reserve(pend, &a.q.ctl->count);
      if (pend) {
        if (slot < a.q.cap) a.q.ent[slot] = ((uint64_t)cur << kEvSlotBits) | (uint64_t)(k0 + off);
        else a.q.ctl->overflow = 1;
      }
    };

    // phase 0: in each chunk a wave owns PPT whole groups (slots k0 + 64 w + j B + [0, 64)).
    // Their live masks are read for the whole run of chunks at once (lane r PPT + j: chunk m0 + r,
    // group j; PPT <= 16 and kPhotonRun = 4 fit a wave); a group whose mask is empty is not read
    // further (after the photons have left the field, that is every group)
    static_assert(PPT * kPhotonRun <= 64, "one mask per lane for a run of chunks");
    const int lane = threadIdx.x & 63;
    if (m0 < 0 || c / kPhotonRun != m0 / kPhotonRun) {  // first chunk of a run in this instance
      m0 = c;
      const int64_t cc = c + lane / PPT;
      const int64_t cend = min(ce, (c / kPhotonRun + 1) * kPhotonRun);  // end of the run
      mrun = 0;
      if (lane < PPT * kPhotonRun && cc < cend) {
        const int64_t g = (pfirst + (cc - cb) * CH) / kWinGroup + (threadIdx.x >> 6) +
                          (int64_t)(lane % PPT) * (B / kWinGroup);
        if (g * kWinGroup < n) {  // a group with photons (the last chunk may reach past them)
          mrun = LM[g];
          ++uacc[5];
        }
      }
    }
    uint64_t M[PPT];  // this chunk's masks of the wave's groups (wave-uniform: scalar registers)
    bool any = false;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int src = (int)(c - m0) * PPT + j;
      M[j] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mrun >> 32), src) << 32) |
             (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mrun, src);
      any = any || M[j] != 0ull;
    }
    if (!any) continue;
    // phase 1: the window, the record and the optical depth of every live slot of the chunk,
    // issued together, so that a chunk costs one memory round trip (loads past the chunk's live
    // slots return zero)
    uint32_t wv[PPT];
    uint32_t q[PPT][kRecDw];
    double tv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      wv[j] = kWinEmpty;
      tv[j] = 0.0;
      if ((M[j] >> lane) & 1ull) {
        const unsigned off = threadIdx.x + j * B;
        wv[j] = (uint32_t)buf_ld<int32_t>(rwin, off * 4u);
        load_dwords<kRecDw>(rrec, off * (unsigned)sizeof(Rec), q[j]);
        tv[j] = buf_ld<double>(rtau, off * 8u);
      }
    }
    unsigned gmask = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const bool exists = (int64_t)(threadIdx.x + j * B) < rem;
      const bool bit = (M[j] >> lane) & 1ull;
      if (exists && bit) ++uacc[4];
      if (exists && in_window(wv[j], step)) gmask |= 1u << j;
      // the mask for the next step loses the photons whose window is over then (a photon's
      // window only ends; the slots past the step's photons keep their bits: the emission pass
      // of this step may have set them)
      if (M[j] != 0ull) {  // wave-uniform
        const uint64_t nm = __ballot(bit && (!exists || !window_over(wv[j], step + 1)));
        if (nm != M[j] && lane == 0) LM[(k0 + threadIdx.x + j * B) / kWinGroup] = nm;
      }
    }
    if (__ballot(gmask != 0) != 0ull) {
      uacc[3] += __popc(gmask);
      // one photon inside its window, from the dwords of its record and its optical depth
      auto eval = [&](unsigned off, const uint32_t* w, double tau) -> bool {
        auto dbl = [&](int i) { return __hiloint2double((int)w[i + 1], (int)w[i]); };
        if constexpr (FK == QED_FIELD_LP_PULSE) {
          if (MIXED) return infield_pw(off, dbl(0), (double)__uint_as_float(w[2]), (double)__uint_as_float(w[3]), tau);
          else return infield_pw(off, dbl(0), dbl(2), dbl(4), tau);
        } else if (MIXED) {
          return infield(off, (Real)__uint_as_float(w[0]), (Real)__uint_as_float(w[1]), (Real)__uint_as_float(w[2]),
                         NEED_X ? (Real)__uint_as_float(w[3]) : Real(0), NEED_Y ? (Real)__uint_as_float(w[4]) : Real(0),
                         NEED_X ? (int32_t)w[5] : 0, tau);
        } else {
          return infield(off, (Real)dbl(0), (Real)dbl(2), (Real)dbl(4), NEED_X ? (Real)dbl(6) : Real(0),
                         NEED_Y ? (Real)dbl(8) : Real(0), NEED_X ? (int32_t)w[10] : 0, tau);
        }
      };
      // phase 2: the photons inside their windows, in place
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const unsigned off = threadIdx.x + j * B;
        bool pend = false;
        if ((gmask >> j) & 1u) pend = eval(off, q[j], tv[j]);
        enqueue(off, pend);
      }
    }
  }
  if (cur >= 0) flush(cur);
}

template <bool MIXED>
__device__ __forceinline__ void write_lepton(const qed_species& S, long long slot, double x, double y, double z,
                                             double ux, double uy, double uz, double tau, uint64_t uid, bool d3) {
  if (MIXED) {
    float h, l;
    split_double(x, h, l); ((float*)S.x_dev)[slot] = h; S.x_lo_dev[slot] = l;
    split_double(y, h, l); ((float*)S.y_dev)[slot] = h; S.y_lo_dev[slot] = l;
    if (d3) { split_double(z, h, l); ((float*)S.z_dev)[slot] = h; S.z_lo_dev[slot] = l; }
    split_double(ux, h, l); ((float*)S.ux_dev)[slot] = h; S.ux_lo_dev[slot] = l;
    split_double(uy, h, l); ((float*)S.uy_dev)[slot] = h; S.uy_lo_dev[slot] = l;
    split_double(uz, h, l); ((float*)S.uz_dev)[slot] = h; S.uz_lo_dev[slot] = l;
  } else {
    ((double*)S.x_dev)[slot] = x;
    ((double*)S.y_dev)[slot] = y;
    if (d3) ((double*)S.z_dev)[slot] = z;
    ((double*)S.ux_dev)[slot] = ux;
    ((double*)S.uy_dev)[slot] = uy;
    ((double*)S.uz_dev)[slot] = uz;
  }
  S.tau_dev[slot] = tau;
  S.uid_dev[slot] = uid;
}

// Pair creation by photon k of instance ii (when `want`): chi at the photon's position (FP64
// form: correctly rounded field), energy split f from the P_f table, electron with (1 - f) k
// and positron with f k at the position after the step, fresh optical depths, photon removed.
// Every lane of the wave calls this (the appends are wave-aggregated).
template <int FK, bool MIXED>
__device__ __forceinline__ void pair_event(const StepArgs& a, int ii, int64_t k, bool want, int64_t step, double t) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  const double dt = a.sc.dt;
  const qed_instance& I = a.inst[ii];
  const qed_species& S = I.s[2];
  const bool d3 = I.dims == 3;
  // the children's species and the photon's record offset, read before the first store (which the
  // compiler cannot tell apart from them), so that the loads share a memory round trip
  const qed_species Se = I.s[0], Sp = I.s[1];
  const int64_t moff = a.acc[ii].mover_off;
  double px = 0, py = 0, pz = 0, etau = 0, ptau = 0, ex = 0, ey = 0, ez = 0, pkx = 0, pky = 0, pkz = 0;
  double defect = 0.0, dropped_e = 0.0;
  unsigned n_drop = 0;
  uint64_t euid = 0, puid = 0;
  if (want) {
    const Real kxr = ((const Real*)S.ux_dev)[k], kyr = ((const Real*)S.uy_dev)[k], kzr = ((const Real*)S.uz_dev)[k];
    const Real xbr = ((const Real*)S.x_dev)[k], ybr = ((const Real*)S.y_dev)[k];
    const int32_t bs = S.birth_step_dev[k];
    const uint64_t uid = S.uid_dev[k];
    const Real eps = sqrt(kxr * kxr + kyr * kyr + kzr * kzr);
    const Real nx = kxr / eps, ny = kyr / eps, nz = kzr / eps;
    const double age = (double)(step - (int64_t)bs) * dt;
    const double x = (double)xbr + age * nx;
    const double y = (double)ybr + age * ny;
    double chi;
    if (MIXED) {
      float E[3], Bf[3];
      field_at32<FK>(I.field, field_k(I.field), x, y, t, E, Bf);
      const float ax = E[0] + (ny * Bf[2] - nz * Bf[1]);
      const float ay = E[1] + (nz * Bf[0] - nx * Bf[2]);
      const float az = E[2] + (nx * Bf[1] - ny * Bf[0]);
      const float ne = nx * E[0] + ny * E[1] + nz * E[2];
      const float r2 = (ax * ax + ay * ay + az * az) - ne * ne;
      chi = 0.5f * (float)eps * sqrtf(r2 > 0.0f ? r2 : 0.0f);
    } else {
      double E[3], Bf[3];
      field_at<FK, true>(I.field, x, y, t, E, Bf);
      const double ax = E[0] + (ny * Bf[2] - nz * Bf[1]);
      const double ay = E[1] + (nz * Bf[0] - nx * Bf[2]);
      const double az = E[2] + (nx * Bf[1] - ny * Bf[0]);
      const double ne = nx * E[0] + ny * E[1] + nz * E[2];
      const double r2 = (ax * ax + ay * ay + az * az) - ne * ne;
      chi = 0.5 * (double)eps * sqrt(r2 > 0.0 ? r2 : 0.0);
    }
    uint64_t r0[4], r1[4];
    philox4x64_10(uid, (uint64_t)step, KIND_PAIR, 0, I.seed, I.key_instance, r0);
    philox4x64_10(uid, (uint64_t)step, KIND_PAIR, 1, I.seed, I.key_instance, r1);
    const double f = sample_f(a.tb, chi, unit_open(r0[0]));
    const double kxd = kxr, kyd = kyr, kzd = kzr;
    pkx = f * kxd;
    pky = f * kyd;
    pkz = f * kzd;
    if (MIXED) {
      ex = kxd - pkx;
      ey = kyd - pky;
      ez = kzd - pkz;
    } else {
      ex = (1.0 - f) * kxd;
      ey = (1.0 - f) * kyd;
      ez = (1.0 - f) * kzd;
    }
    const double gp = sqrt(1.0 + (pkx * pkx + pky * pky + pkz * pkz));
    const double ge = sqrt(1.0 + (ex * ex + ey * ey + ez * ez));
    const double epsd = MIXED ? sqrt(kxd * kxd + kyd * kyd + kzd * kzd) : (double)eps;
    const double age1 = age + dt;
    px = (double)xbr + age1 * nx;
    py = (double)ybr + age1 * ny;
    pz = d3 ? (double)((const Real*)S.z_dev)[k] + age1 * nz : 0.0;
    euid = r0[1];
    puid = r0[2];
    etau = optical_depth(r0[3]);
    ptau = optical_depth(r1[0]);
    S.tau_dev[k] = kTauGone;
    a.win[moff + k] = kWinEmpty;
    defect = gp + ge - epsd;
  }
  // append electron and positron, one atomic per wave, instance and species
  long long se, spo;
  wave_reserve2_grouped(want, ii, Se.count_dev, Sp.count_dev, &se, &spo);
  if (want) {
    if (se < Se.capacity) {
      write_lepton<MIXED>(Se, se, px, py, pz, ex, ey, ez, etau, euid, d3);
    } else {
      ++n_drop;
      dropped_e += sqrt(1.0 + (ex * ex + ey * ey + ez * ez));
    }
    if (spo < Sp.capacity) {
      write_lepton<MIXED>(Sp, spo, px, py, pz, pkx, pky, pkz, ptau, puid, d3);
    } else {
      ++n_drop;
      dropped_e += sqrt(1.0 + (pkx * pkx + pky * pky + pkz * pkz));
    }
  }
  add_event_stats(1, want, ii, a.acc, defect, dropped_e, want ? 1u : 0u, 0u, n_drop);
}

// Event pass: the queued photons, or, when the queue overflowed, every photon whose optical
// depth is in the converting state.  Both loops advance whole waves together, as the
// wave-aggregated appends need.
template <int FK, bool MIXED>
__global__ __launch_bounds__(256) void k_pair_events(StepArgs a) {
  const int64_t step = a.glob->step_cur;
  const double t = a.sc.t0 + (double)step * a.sc.dt;
  const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t cnt = a.q.ctl->count;  // read with the overflow flag (one round trip)
  if (!a.q.ctl->overflow) {
    for (int64_t e0 = gtid - threadIdx.x % 64; e0 < cnt; e0 += stride) {
      // whole waves iterate together; lanes past the end take no event
      const int64_t e = e0 + threadIdx.x % 64;
      const bool want = e < cnt;
      const uint64_t ent = want ? a.q.ent[e] : 0;
      pair_event<FK, MIXED>(a, (int)(ent >> kEvSlotBits), (int64_t)(ent & ((1ull << kEvSlotBits) - 1)), want, step,
                            t);
    }
  } else {
    for (int ii = 0; ii < a.n_base; ++ii) {
      const int64_t n = a.acc[ii].n_start[2];
      const double* TAU = a.inst[ii].s[2].tau_dev;
      for (int64_t k0 = gtid - threadIdx.x % 64; k0 < n; k0 += stride) {
        const int64_t k = k0 + threadIdx.x % 64;
        bool want = false;
        if (k < n) {
          const double tau = TAU[k];
          want = tau <= 0.0 && tau >= kTauPendingMin;
        }
        pair_event<FK, MIXED>(a, ii, k, want, step, t);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// optical-depth initialisation: tau = -ln U, U from counter (uid, 0, INIT, 0)
// grid: x strides particles, y = instance * 3 + species
// ---------------------------------------------------------------------------
__global__ void k_init_tau(const qed_instance* __restrict__ inst) {
  const int ii = blockIdx.y / 3, s = blockIdx.y % 3;
  const qed_instance& I = inst[ii];
  const qed_species& S = I.s[s];
  if (!S.count_dev) return;
  int64_t n = *S.count_dev;
  if (n > S.capacity) n = S.capacity;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    if (s == 2 && S.tau_dev[k] < kTauPendingMin) continue;  // a converted photon keeps its mark
    uint64_t r[4];
    philox4x64_10(S.uid_dev[k], 0, KIND_INIT, 0, I.seed, I.key_instance, r);
    S.tau_dev[k] = optical_depth(r[0]);
  }
}

// ---------------------------------------------------------------------------
// energy ledger: sum of gamma (leptons) and |k| (live photons), and counts
// ---------------------------------------------------------------------------
__global__ void k_ledger_zero(InstAcc* acc, int n_inst) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    for (int s = 0; s < 3; ++s) {
      for (int k = 0; k < 4; ++k) acc[i].fx[FX_ENERGY + s][k] = 0;
      acc[i].led_count[s] = 0;
    }
    for (int q = 0; q < kFixRunning; ++q) fix_normalise(acc[i].fx[q]);
  }
}

template <bool MIXED>
__global__ __launch_bounds__(256) void k_ledger(const qed_instance* __restrict__ inst, InstAcc* __restrict__ acc) {
  __shared__ long long s_ll[16 * 4];
  __shared__ unsigned sredu[16 * 1];
  const int ii = blockIdx.y / 3, s = blockIdx.y % 3;
  const qed_species& S = inst[ii].s[s];
  long long fw[4] = {0, 0, 0, 0};  // energy, exact fixed point per lane
  unsigned u[1] = {0};
  auto add = [&](double e) {
    long long l[4];
    fix_split(e, l);
#pragma unroll
    for (int k = 0; k < 4; ++k) fw[k] += l[k];
  };
  if (S.count_dev) {
    int64_t n = *S.count_dev;
    if (n > S.capacity) n = S.capacity;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
      double ux, uy, uz;
      if (MIXED) {
        ux = (double)((const float*)S.ux_dev)[k];
        uy = (double)((const float*)S.uy_dev)[k];
        uz = (double)((const float*)S.uz_dev)[k];
        if (s < 2) {
          ux += (double)S.ux_lo_dev[k];
          uy += (double)S.uy_lo_dev[k];
          uz += (double)S.uz_lo_dev[k];
        }
      } else {
        ux = ((const double*)S.ux_dev)[k];
        uy = ((const double*)S.uy_dev)[k];
        uz = ((const double*)S.uz_dev)[k];
      }
      if (s == 2) {
        if (S.tau_dev[k] < 0.0) continue;
        add(sqrt(ux * ux + uy * uy + uz * uz));
      } else {
        add(sqrt(1.0 + (ux * ux + uy * uy + uz * uz)));
      }
      ++u[0];
    }
  }
  // per-lane words to wave sums (integers: any order), then the block's sum by thread 0
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    fw[k] = wave_sum_ll(fw[k]);
    if ((threadIdx.x & 63) == 0) s_ll[(threadIdx.x >> 6) * 4 + k] = fw[k];
  }
  long long* const dst[1] = {acc[ii].fx[FX_ENERGY + s]};
  fix_block_flush<1>(s_ll, dst);
  block_sum_u(u, sredu);
  if (threadIdx.x == 0 && u[0]) atomicAdd(&acc[ii].led_count[s], (unsigned long long)u[0]);
}

// ---------------------------------------------------------------------------
// compaction of dead photons (tau < 0): live photons from [n_live, n) fill the holes in [0, n_live)
// ---------------------------------------------------------------------------
// A photon leaves the arrays at compaction when it converted to a pair (tau < 0) or, with
// retirement on, when its pair window is over (it can never convert: it only moves ballistically,
// so it is booked into the ledger and the instance's photon spectrum and dropped).

struct RetireArgs {
  int on;                       // retirement enabled
  int n_bins;                   // spectrum bins, log-spaced in photon energy over [e_min, e_max]
  double le_min, inv_dle;       // ln e_min and 1 / ln-width of a bin
  unsigned long long* spec;     // per instance n_bins + 2 counts (below, bins, above)
  int64_t step;                 // the step after the compaction (windows over before it): set by
                                // each kernel from the device clock
};

__global__ void k_compact_prep(const qed_instance* __restrict__ inst, int n_inst, InstAcc* __restrict__ acc,
                               int retire) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    const qed_species& S = inst[i].s[2];
    int64_t n = S.count_dev ? *S.count_dev : 0;
    if (n > S.capacity) n = S.capacity;
    if (n < 0) n = 0;
    if (S.count_dev) *S.count_dev = n;
    acc[i].n_start[2] = n;
    acc[i].hole_ctr = 0;
    acc[i].mover_ctr = 0;
    // photons are removed only by pair creation: with no pair event since the last compaction
    // there is nothing to remove (the first compaction after a bind always runs)
    const bool skip = !retire && acc[i].n_pair_compacted == acc[i].n_pair;
    acc[i].compact_skip = skip ? 1 : 0;
    acc[i].n_live = skip ? n : 0;
    acc[i].n_pair_compacted = acc[i].n_pair;
    // The front [0, n_front) holds photons whose window was over at the last compaction: none of
    // them has converted since (no pair rate), so the holes all lie behind it, it stays in place
    // and the partition below only has to sort what lies behind it.  Retirement removes those
    // photons: then there is no front to keep.
    if (retire || acc[i].n_front > n) acc[i].n_front = retire ? 0 : n;
  }
}

__device__ __forceinline__ bool photon_leaves(const qed_species& S, const uint32_t* W, int64_t k, const RetireArgs& r) {
  return S.tau_dev[k] < 0.0 || (r.on && window_over(W[k], r.step));
}

// live photons per instance; retired photons' energy, count and spectrum bin
template <bool MIXED>
__global__ __launch_bounds__(256) void k_compact_count(const qed_instance* __restrict__ inst, InstAcc* __restrict__ acc,
                                                       const Glob* __restrict__ glob, const uint32_t* __restrict__ win,
                                                       RetireArgs r) {
  r.step = glob->step_next;
  using Real = typename std::conditional<MIXED, float, double>::type;
  __shared__ unsigned sredu[16 * 2];
  __shared__ long long s_ll[16 * 4];
  extern __shared__ unsigned s_hist[];  // n_bins + 2 with retirement on
  const int ii = blockIdx.y;
  if (acc[ii].compact_skip) return;
  const qed_species& S = inst[ii].s[2];
  const uint32_t* W = win + acc[ii].mover_off;
  const int64_t n = acc[ii].n_start[2], F = acc[ii].n_front;
  if (r.on)
    for (int b = threadIdx.x; b < r.n_bins + 2; b += blockDim.x) s_hist[b] = 0u;
  __syncthreads();
  unsigned u[2] = {0, 0};  // live, retired
  long long fe[4] = {0, 0, 0, 0};
  if (blockIdx.x == 0 && threadIdx.x == 0 && F > 0)
    atomicAdd((unsigned long long*)&acc[ii].n_live, (unsigned long long)F);  // the front stays
  for (int64_t k = F + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double tau = S.tau_dev[k];
    if (tau < 0.0) continue;
    if (r.on && window_over(W[k], r.step)) {
      const double kx = ((const Real*)S.ux_dev)[k], ky = ((const Real*)S.uy_dev)[k], kz = ((const Real*)S.uz_dev)[k];
      const double e = sqrt(kx * kx + ky * ky + kz * kz);
      long long l[4];
      fix_split(e, l);
#pragma unroll
      for (int q = 0; q < 4; ++q) fe[q] += l[q];
      ++u[1];
      const double sb = e > 0.0 ? (log(e) - r.le_min) * r.inv_dle : -1.0;  // bin of the spectrum
      const int b = !(sb >= 0.0) ? 0 : sb >= (double)r.n_bins ? r.n_bins + 1 : 1 + (int)sb;
      atomicAdd(&s_hist[b], 1u);
    } else {
      ++u[0];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    fe[q] = wave_sum_ll(fe[q]);
    if ((threadIdx.x & 63) == 0) s_ll[(threadIdx.x >> 6) * 4 + q] = fe[q];
  }
  long long* const dst[1] = {acc[ii].fx[FX_RETIRED]};
  fix_block_flush<1>(s_ll, dst);
  block_sum_u(u, sredu);
  if (threadIdx.x == 0) {
    if (u[0]) atomicAdd((unsigned long long*)&acc[ii].n_live, (unsigned long long)u[0]);
    if (u[1]) atomicAdd(&acc[ii].n_retired, (unsigned long long)u[1]);
  }
  if (r.on) {
    __syncthreads();
    unsigned long long* H = r.spec + (size_t)ii * (r.n_bins + 2);
    for (int b = threadIdx.x; b < r.n_bins + 2; b += blockDim.x)
      if (s_hist[b]) atomicAdd(&H[b], (unsigned long long)s_hist[b]);
  }
}

__global__ __launch_bounds__(256) void k_compact_movers(const qed_instance* __restrict__ inst, InstAcc* __restrict__ acc,
                                                        const Glob* __restrict__ glob, int64_t* __restrict__ movers,
                                                        const uint32_t* __restrict__ win, RetireArgs r) {
  r.step = glob->step_next;
  const int ii = blockIdx.y;
  if (acc[ii].compact_skip) return;
  const qed_species& S = inst[ii].s[2];
  const uint32_t* W = win + acc[ii].mover_off;
  const int64_t n = acc[ii].n_start[2], L = acc[ii].n_live;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // loop bounds are identical across a wave so that every lane reaches the ballot
  for (int64_t k0 = L + blockIdx.x * (int64_t)blockDim.x; k0 < n; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    const bool mv = k < n && !photon_leaves(S, W, k, r);
    const long long slot = wave_reserve(mv, (int64_t*)&acc[ii].mover_ctr);
    if (mv) movers[acc[ii].mover_off + slot] = k;
  }
}

template <bool MIXED>
__global__ __launch_bounds__(256) void k_compact_fill(const qed_instance* __restrict__ inst, InstAcc* __restrict__ acc,
                                                      const Glob* __restrict__ glob, const int64_t* __restrict__ movers,
                                                      uint32_t* __restrict__ win, void* __restrict__ rec, int rec_words,
                                                      RetireArgs r) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  r.step = glob->step_next;
  const int ii = blockIdx.y;
  if (acc[ii].compact_skip) return;
  const qed_species& S = inst[ii].s[2];
  const int64_t L = acc[ii].n_live, n = acc[ii].n_start[2], F = acc[ii].n_front;
  const long long n_movers = (long long)acc[ii].mover_ctr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool d3 = inst[ii].dims == 3;
  Real* const X = (Real*)S.x_dev;
  Real* const Y = (Real*)S.y_dev;
  Real* const Z = (Real*)S.z_dev;
  Real* const UX = (Real*)S.ux_dev;
  Real* const UY = (Real*)S.uy_dev;
  Real* const UZ = (Real*)S.uz_dev;
  uint32_t* const W = win + acc[ii].mover_off;
  uint2* const R = (uint2*)rec + acc[ii].mover_off * rec_words;
  for (int64_t k0 = F + blockIdx.x * (int64_t)blockDim.x; k0 < L; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    const bool hole = k < L && photon_leaves(S, W, k, r);
    const long long slot = wave_reserve(hole, (int64_t*)&acc[ii].hole_ctr);
    // every hole in [F, L) has a mover in [L, n); the bounds below only guard that invariant
    if (hole && slot < n_movers) {
      const int64_t src = movers[acc[ii].mover_off + slot];
      if (src < L || src >= n) continue;
      // the mover's words, all loaded before the first store (one memory round trip)
      const Real x = X[src], y = Y[src], z = d3 ? Z[src] : Real(0), ux = UX[src], uy = UY[src], uz = UZ[src];
      const double tau = S.tau_dev[src];
      const uint64_t uid = S.uid_dev[src];
      const int32_t bs = S.birth_step_dev[src];
      const uint32_t w = W[src];
      uint2 rv[8];
      for (int q = 0; q < rec_words; ++q) rv[q] = R[src * rec_words + q];
      X[k] = x;
      Y[k] = y;
      if (d3) Z[k] = z;
      UX[k] = ux;
      UY[k] = uy;
      UZ[k] = uz;
      S.tau_dev[k] = tau;
      S.uid_dev[k] = uid;
      S.birth_step_dev[k] = bs;
      W[k] = w;
      for (int q = 0; q < rec_words; ++q) R[k * rec_words + q] = rv[q];
    }
  }
}

__global__ void k_compact_finish(const qed_instance* __restrict__ inst, int n_inst, const InstAcc* __restrict__ acc) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    const qed_species& S = inst[i].s[2];
    if (S.count_dev) *S.count_dev = acc[i].n_live;
  }
}

// ---------------------------------------------------------------------------
// partition of the photons by pair window (after the compaction): the photons that can have no
// pair rate from the next step on (an empty window, or one that ended before that step) go to
// the front [0, D), the others to the back.  The photons the sweep evaluates in a step then sit
// together, and the sweep never reaches the front.  Photons of the back that
// belong to the front swap places with front photons that belong to the back (per-uid results
// do not depend on the order).
// ---------------------------------------------------------------------------

__global__ void k_part_prep(const qed_instance* __restrict__ inst, int n_inst, InstAcc* __restrict__ acc) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    const qed_species& S = inst[i].s[2];
    int64_t n = S.count_dev ? *S.count_dev : 0;
    if (n > S.capacity) n = S.capacity;
    if (n < 0) n = 0;
    acc[i].n_start[2] = n;
    acc[i].n_live = 0;  // here: photons whose window is over (the size D of the front)
    acc[i].hole_ctr = 0;
    acc[i].mover_ctr = 0;
  }
}

__global__ __launch_bounds__(256) void k_part_count(InstAcc* __restrict__ acc, const Glob* __restrict__ glob,
                                                    const uint32_t* __restrict__ win) {
  __shared__ double sred[16];
  __shared__ unsigned sredu[16];
  const int ii = blockIdx.y;
  const int64_t n = acc[ii].n_start[2], s = glob->step_next, F = acc[ii].n_front;
  const uint32_t* W = win + acc[ii].mover_off;
  double d[1] = {0.0};
  unsigned u[1] = {0};
  if (blockIdx.x == 0 && threadIdx.x == 0 && F > 0)
    atomicAdd((unsigned long long*)&acc[ii].n_live, (unsigned long long)F);  // the front: over before
  for (int64_t k = F + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    if (window_over(W[k], s)) ++u[0];
  block_sum(d, u, sred, sredu);
  if (threadIdx.x == 0 && u[0]) atomicAdd((unsigned long long*)&acc[ii].n_live, (unsigned long long)u[0]);
}

// the photons of [D, n) whose window is over, listed in the mover array.  Each block takes a
// contiguous range: it counts its movers, reserves their places with one atomic, then lists
// them in order (one contended atomic per block rather than per wave).
__global__ __launch_bounds__(256) void k_part_movers(InstAcc* __restrict__ acc, const Glob* __restrict__ glob,
                                                     const uint32_t* __restrict__ win, int64_t* __restrict__ movers) {
  __shared__ unsigned sredu[16];
  __shared__ long long s_base;
  const int ii = blockIdx.y;
  const int64_t n = acc[ii].n_start[2], D = acc[ii].n_live, s = glob->step_next;
  const uint32_t* W = win + acc[ii].mover_off;
  int64_t b0, b1;
  block_range(D, n, blockIdx.x, gridDim.x, &b0, &b1);
  if (b0 >= b1) return;  // the whole block
  unsigned u[1] = {0};
  for (int64_t k = b0 + threadIdx.x; k < b1; k += blockDim.x)
    if (window_over(W[k], s)) ++u[0];
  block_sum_u(u, sredu);
  if (threadIdx.x == 0) s_base = u[0] ? (long long)atomicAdd((unsigned long long*)&acc[ii].mover_ctr, (unsigned long long)u[0]) : 0;
  __syncthreads();
  long long run = s_base;
  int64_t* M = movers + acc[ii].mover_off;
  for (int64_t k0 = b0; k0 < b1; k0 += blockDim.x) {  // block-uniform trip count
    const int64_t k = k0 + threadIdx.x;
    const bool mv = k < b1 && window_over(W[k], s);
    unsigned tot;
    const unsigned r = block_rank(mv, sredu, &tot);
    if (mv) M[run + r] = k;
    run += tot;
  }
}

// every photon of [F, D) whose window is not over swaps with one listed by k_part_movers (the
// front [0, F) of the last compaction is in place)
template <bool MIXED>
__global__ __launch_bounds__(256) void k_part_swap(const qed_instance* __restrict__ inst, InstAcc* __restrict__ acc,
                                                   const Glob* __restrict__ glob, const int64_t* __restrict__ movers,
                                                   uint32_t* __restrict__ win, void* __restrict__ rec, int rec_words) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  const int ii = blockIdx.y;
  const qed_species& S = inst[ii].s[2];
  const int64_t n = acc[ii].n_start[2], D = acc[ii].n_live, s = glob->step_next, F = min(acc[ii].n_front, D);
  const long long n_movers = (long long)acc[ii].mover_ctr;
  uint32_t* W = win + acc[ii].mover_off;
  const bool d3 = inst[ii].dims == 3;
  Real* const X = (Real*)S.x_dev;
  Real* const Y = (Real*)S.y_dev;
  Real* const Z = (Real*)S.z_dev;
  Real* const UX = (Real*)S.ux_dev;
  Real* const UY = (Real*)S.uy_dev;
  Real* const UZ = (Real*)S.uz_dev;
  uint2* const R = (uint2*)rec + acc[ii].mover_off * rec_words;
  // a contiguous range of [F, D) per block, its holes' places reserved with one atomic
  __shared__ unsigned sredu[16];
  __shared__ long long s_base;
  int64_t b0, b1;
  block_range(F, D, blockIdx.x, gridDim.x, &b0, &b1);
  if (b0 >= b1) return;  // the whole block
  unsigned u[1] = {0};
  for (int64_t k = b0 + threadIdx.x; k < b1; k += blockDim.x)
    if (!window_over(W[k], s)) ++u[0];
  block_sum_u(u, sredu);
  if (threadIdx.x == 0) s_base = u[0] ? (long long)atomicAdd((unsigned long long*)&acc[ii].hole_ctr, (unsigned long long)u[0]) : 0;
  __syncthreads();
  long long run = s_base;
  for (int64_t k0 = b0; k0 < b1; k0 += blockDim.x) {  // block-uniform trip count
    const int64_t k = k0 + threadIdx.x;
    const bool sw = k < b1 && !window_over(W[k], s);
    unsigned tot;
    const long long slot = run + block_rank(sw, sredu, &tot);
    run += tot;
    // the two counts are equal (both are D minus the front's photons that stay); the bounds
    // below only guard that invariant
    if (sw && slot < n_movers) {
      const int64_t j = movers[acc[ii].mover_off + slot];
      if (j < D || j >= n) continue;
      // both photons' words, all loaded before the first store (one memory round trip)
      const Real xk = X[k], xj = X[j], yk = Y[k], yj = Y[j];
      const Real zk = d3 ? Z[k] : Real(0), zj = d3 ? Z[j] : Real(0);
      const Real uxk = UX[k], uxj = UX[j], uyk = UY[k], uyj = UY[j], uzk = UZ[k], uzj = UZ[j];
      const double tk = S.tau_dev[k], tj = S.tau_dev[j];
      const uint64_t ik = S.uid_dev[k], ij = S.uid_dev[j];
      const int32_t bk = S.birth_step_dev[k], bj = S.birth_step_dev[j];
      const uint32_t wk = W[k], wj = W[j];
      uint2 rk[8], rj[8];
      for (int q = 0; q < rec_words; ++q) {
        rk[q] = R[k * rec_words + q];
        rj[q] = R[j * rec_words + q];
      }
      X[k] = xj; X[j] = xk;
      Y[k] = yj; Y[j] = yk;
      if (d3) { Z[k] = zj; Z[j] = zk; }
      UX[k] = uxj; UX[j] = uxk;
      UY[k] = uyj; UY[j] = uyk;
      UZ[k] = uzj; UZ[j] = uzk;
      S.tau_dev[k] = tj; S.tau_dev[j] = tk;
      S.uid_dev[k] = ij; S.uid_dev[j] = ik;
      S.birth_step_dev[k] = bj; S.birth_step_dev[j] = bk;
      W[k] = wj; W[j] = wk;
      for (int q = 0; q < rec_words; ++q) {
        R[k * rec_words + q] = rj[q];
        R[j * rec_words + q] = rk[q];
      }
    }
  }
}

// Live masks of every instance's photon slot groups from the windows (after a window build, and
// after the partition at compaction, which moves photons across all groups): bit i of group g
// set when slot 64 g + i holds a photon whose window is not over at the next step.  One wave per
// group; grid: x strides groups, y = instance.  The groups past the photons keep their masks
// (bits of slots that no photon holds cost the sweep a read that returns zero, nothing else).
__global__ __launch_bounds__(256) void k_window_masks(const qed_instance* __restrict__ inst,
                                                      const InstAcc* __restrict__ acc, const Glob* __restrict__ glob,
                                                      const uint32_t* __restrict__ win, uint64_t* __restrict__ lmask) {
  const int ii = blockIdx.y;
  const qed_species& S = inst[ii].s[2];
  if (S.capacity == 0 || !S.count_dev) return;
  int64_t n = *S.count_dev;
  if (n > S.capacity) n = S.capacity;
  if (n < 0) n = 0;
  const int64_t ng = (n + kWinGroup - 1) / kWinGroup, step = glob->step_next;
  const uint32_t* W = win + acc[ii].mover_off;
  uint64_t* L = lmask + acc[ii].lmask_off;
  const int lane = threadIdx.x & 63;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
  // the loop bound is wave-uniform, so every lane reaches the ballot
  for (int64_t g = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); g < ng; g += wstride) {
    const int64_t k = g * kWinGroup + lane;
    const bool live = k < n && !window_over(W[k], step);
    const uint64_t m = __ballot(live);
    if (lane == 0) L[g] = m;
  }
}

// The partition's front after a compaction (after_partition), else none (the windows were just
// rebuilt)
__global__ void k_window_front(const qed_instance* __restrict__ inst, int n_inst, InstAcc* __restrict__ acc,
                               int after_partition) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    const qed_species& S = inst[i].s[2];
    int64_t n = S.count_dev ? *S.count_dev : 0;
    if (n > S.capacity) n = S.capacity;
    if (n < 0) n = 0;
    const int64_t D = after_partition ? acc[i].n_live : 0;
    acc[i].n_front = D < 0 ? 0 : (D > n ? n : D);
  }
}

// Pair windows of every photon present (after a bind, or when the step's t0, dt or tables
// change); grid: x strides photons, y = instance.
template <bool MIXED, int FK>
__global__ __launch_bounds__(256) void k_photon_windows(const qed_instance* __restrict__ inst,
                                                        const InstAcc* __restrict__ acc, uint32_t* __restrict__ win,
                                                        void* __restrict__ rec_v, double t0, double dt,
                                                        double cp_min) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  const int ii = blockIdx.y;
  const qed_species& S = inst[ii].s[2];
  if (S.capacity == 0 || !S.count_dev) return;
  const int64_t n = min(*S.count_dev, S.capacity);
  const double eps_min = pair_eps_min(inst[ii].field, cp_min);
  uint32_t* W = win + acc[ii].mover_off;
  PhotonRecT<MIXED, FK>* R = (PhotonRecT<MIXED, FK>*)rec_v + acc[ii].mover_off;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += stride) {
    const double kx = ((const Real*)S.ux_dev)[k], ky = ((const Real*)S.uy_dev)[k], kz = ((const Real*)S.uz_dev)[k];
    const double xb = ((const Real*)S.x_dev)[k], yb = ((const Real*)S.y_dev)[k];
    const int32_t bs = S.birth_step_dev[k];
    PhotonRecT<MIXED, FK> r{};
    make_photon_rec<MIXED, FK>(r, inst[ii].field, t0, dt, kx, ky, kz, xb, yb, bs);
    R[k] = r;
    // converted photons (waiting for compaction) have no window
    W[k] = S.tau_dev[k] < kTauPendingMin
               ? kWinEmpty
               : pack_window(photon_window(inst[ii].field, eps_min, cp_min, t0, dt, kx, ky, kz, xb, bs));
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

// Reciprocal factorials 1/n! as double-doubles (Dekker splits; dd / integer division with one
// exact remainder), uploaded once per device for the correctly rounded device math.
hipError_t init_crmath() {
  static unsigned long long done = 0;  // one bit per device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 64 && (done >> dev) & 1ull) return hipSuccess;
  dd f[30];
  f[0] = {1.0, 0.0};
  for (int n = 1; n < 30; ++n) {
    const double q1 = f[n - 1].hi / n;
    const double p = q1 * n, pe = std::fma(q1, (double)n, -p);
    const double rem = ((f[n - 1].hi - p) - pe) + f[n - 1].lo;
    const double q2 = rem / n;
    const double s = q1 + q2;
    f[n] = {s, q2 - (s - q1)};
  }
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_inv_fact), f, sizeof(f));
  // log table of fast_log: c_j = 1 / (centre of the j-th sub-interval of [1/2, 1)), L_j = -log c_j
  double lt[2 * kLogTab];
  for (int j = 0; j < kLogTab; ++j) {
    const double c = 1.0 / (0.5 + (j + 0.5) / (2.0 * kLogTab));
    lt[2 * j] = c;
    lt[2 * j + 1] = -std::log(c);
  }
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_logtab), lt, sizeof(lt));
  if (e == hipSuccess && dev < 64) done |= 1ull << dev;
  return e;
}
template <int FK>
static void launch_lepton_fk(const StepArgs& a, dim3 grid, dim3 block, size_t shm, hipStream_t s, bool mixed) {
#define QED_LEP(P)                                                                   \
  if (mixed) hipLaunchKernelGGL((k_lepton<FK, P, true>), grid, block, shm, s, a); \
  else hipLaunchKernelGGL((k_lepton<FK, P, false>), grid, block, shm, s, a);
  switch (a.ppt) {
    case 1: QED_LEP(1) break;
    case 2: QED_LEP(2) break;
    case 8: QED_LEP(8) break;
    default: QED_LEP(4) break;
  }
#undef QED_LEP
}
template <int FK>
static void launch_emit_events_fk(const StepArgs& a, dim3 grid, dim3 block, size_t shm, hipStream_t s, bool mixed) {
  if (mixed) hipLaunchKernelGGL((k_emit_events<FK, true>), grid, block, shm, s, a);
  else hipLaunchKernelGGL((k_emit_events<FK, false>), grid, block, shm, s, a);
}
template <int FK>
static void launch_pair_events_fk(const StepArgs& a, dim3 grid, dim3 block, hipStream_t s, bool mixed) {
  if (mixed) hipLaunchKernelGGL((k_pair_events<FK, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_pair_events<FK, false>), grid, block, 0, s, a);
}
template <int FK, int PPT>
static void launch_photon_ppt(const StepArgs& a, dim3 grid, dim3 block, size_t shm, hipStream_t s, bool mixed) {
  if (mixed) hipLaunchKernelGGL((k_photon<FK, PPT, true>), grid, block, shm, s, a);
  else hipLaunchKernelGGL((k_photon<FK, PPT, false>), grid, block, shm, s, a);
}
template <int FK>
static void launch_photon_fk(const StepArgs& a, dim3 grid, dim3 block, size_t shm, hipStream_t s, bool mixed) {
  switch (a.ppt) {
    case 1: launch_photon_ppt<FK, 1>(a, grid, block, shm, s, mixed); break;
    case 2: launch_photon_ppt<FK, 2>(a, grid, block, shm, s, mixed); break;
    case 8: launch_photon_ppt<FK, 8>(a, grid, block, shm, s, mixed); break;
    case 16: launch_photon_ppt<FK, 16>(a, grid, block, shm, s, mixed); break;
    default: launch_photon_ppt<FK, 4>(a, grid, block, shm, s, mixed); break;
  }
}

void launch_step_begin(const qed_instance* inst, int n_inst, InstAcc* acc, Glob* glob, EvCtl* evc, EvCtl* emc,
                       int64_t* base_lep, int64_t* base_ph, int chunk_lep, int chunk_ph, int advance,
                       int count_photons, hipStream_t s) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, s, inst, n_inst, acc, glob, evc, emc, base_lep, base_ph,
                     chunk_lep, chunk_ph, advance, count_photons);
}

void launch_set_step(const qed_instance* inst, int n_inst, InstAcc* acc, Glob* glob, const uint32_t* win,
                     uint64_t* lmask, int64_t step, hipStream_t s) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(256), 0, s, glob, acc, n_inst, step);
  if (n_inst > 0 && win && lmask)
    hipLaunchKernelGGL(k_window_masks, dim3(n_inst == 1 ? 2048 : 64, n_inst), dim3(256), 0, s, inst, acc, glob, win, lmask);
}

void launch_front_clear(InstAcc* acc, int n_inst, hipStream_t s) {
  if (n_inst > 0) hipLaunchKernelGGL(k_front_clear, dim3(1), dim3(256), 0, s, acc, n_inst);
}

void launch_grid_refresh(const qed_instance* inst, int n_inst, const Glob* glob, const StepConst& sc, hipStream_t s) {
  hipLaunchKernelGGL(k_grid_refresh, dim3(2048), dim3(256), 0, s, inst, n_inst, glob, sc);
}

template <int FK>
static int emit_fit_fk(size_t shm, bool mixed) {
  int n = 0;
  const hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_emit_events<FK, true>, 256, shm)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_emit_events<FK, false>, 256, shm);
  return e == hipSuccess ? n : 0;
}
int emit_blocks_per_cu(int fk, int lepton_waves, bool mixed) {
  const size_t shm = ((size_t)lepton_waves + 1) * sizeof(int);
  switch (fk) {
    case QED_FIELD_UNIFORM: return emit_fit_fk<QED_FIELD_UNIFORM>(shm, mixed);
    case QED_FIELD_LP_PULSE: return emit_fit_fk<QED_FIELD_LP_PULSE>(shm, mixed);
    case QED_FIELD_CP_WAVE: return emit_fit_fk<QED_FIELD_CP_WAVE>(shm, mixed);
    case QED_FIELD_CP_STANDING: return emit_fit_fk<QED_FIELD_CP_STANDING>(shm, mixed);
    case QED_FIELD_GRID_FDTD: return emit_fit_fk<QED_FIELD_GRID_FDTD>(shm, mixed);
    default: return emit_fit_fk<QED_FIELD_GRID_CP_STANDING>(shm, mixed);
  }
}

void launch_emit_events(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s) {
  const dim3 g(grid), b(block);
  const size_t shm = ((size_t)a.qe.grid * a.qe.waves + 1) * sizeof(int);  // prefix of the per-wave counts
  switch (fk) {
    case QED_FIELD_UNIFORM: launch_emit_events_fk<QED_FIELD_UNIFORM>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_LP_PULSE: launch_emit_events_fk<QED_FIELD_LP_PULSE>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_CP_WAVE: launch_emit_events_fk<QED_FIELD_CP_WAVE>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_CP_STANDING: launch_emit_events_fk<QED_FIELD_CP_STANDING>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_GRID_FDTD: launch_emit_events_fk<QED_FIELD_GRID_FDTD>(a, g, b, shm, s, mixed); break;
    default: launch_emit_events_fk<QED_FIELD_GRID_CP_STANDING>(a, g, b, shm, s, mixed); break;
  }
}

static size_t lepton_shm(int fk, int n_eta) {
  return (size_t)n_eta * sizeof(double) + 16 * 2 * 4 * sizeof(long long) + 16 * 3 * sizeof(unsigned) + 64 +
         (fk == QED_FIELD_GRID_FDTD ? 3 * (size_t)kDepNodes * sizeof(double) : 0);
}
template <int FK, int PPT>
static int lepton_fit_ppt(int block, size_t shm, bool mixed) {
  int n = 0;
  const hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_lepton<FK, PPT, true>, block, shm)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_lepton<FK, PPT, false>, block, shm);
  return e == hipSuccess ? n : 0;
}
template <int FK>
static int lepton_fit_fk(int ppt, int block, size_t shm, bool mixed) {
  switch (ppt) {
    case 1: return lepton_fit_ppt<FK, 1>(block, shm, mixed);
    case 2: return lepton_fit_ppt<FK, 2>(block, shm, mixed);
    case 8: return lepton_fit_ppt<FK, 8>(block, shm, mixed);
    default: return lepton_fit_ppt<FK, 4>(block, shm, mixed);
  }
}
// Blocks of the lepton sweep that fit on one CU at once (registers, LDS), for the shape given.
int lepton_blocks_per_cu(int fk, int ppt, int block, int n_eta, bool mixed) {
  const size_t shm = lepton_shm(fk, n_eta);
  switch (fk) {
    case QED_FIELD_UNIFORM: return lepton_fit_fk<QED_FIELD_UNIFORM>(ppt, block, shm, mixed);
    case QED_FIELD_LP_PULSE: return lepton_fit_fk<QED_FIELD_LP_PULSE>(ppt, block, shm, mixed);
    case QED_FIELD_CP_WAVE: return lepton_fit_fk<QED_FIELD_CP_WAVE>(ppt, block, shm, mixed);
    case QED_FIELD_CP_STANDING: return lepton_fit_fk<QED_FIELD_CP_STANDING>(ppt, block, shm, mixed);
    case QED_FIELD_GRID_FDTD: return lepton_fit_fk<QED_FIELD_GRID_FDTD>(ppt, block, shm, mixed);
    default: return lepton_fit_fk<QED_FIELD_GRID_CP_STANDING>(ppt, block, shm, mixed);
  }
}

void launch_lepton(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s) {
  const size_t shm = lepton_shm(fk, a.tb.n_eta);
  const dim3 g(grid), b(block);
  switch (fk) {
    case QED_FIELD_UNIFORM: launch_lepton_fk<QED_FIELD_UNIFORM>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_LP_PULSE: launch_lepton_fk<QED_FIELD_LP_PULSE>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_CP_WAVE: launch_lepton_fk<QED_FIELD_CP_WAVE>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_CP_STANDING: launch_lepton_fk<QED_FIELD_CP_STANDING>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_GRID_FDTD: launch_lepton_fk<QED_FIELD_GRID_FDTD>(a, g, b, shm, s, mixed); break;
    default: launch_lepton_fk<QED_FIELD_GRID_CP_STANDING>(a, g, b, shm, s, mixed); break;
  }
}

void launch_pair_events(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s) {
  const dim3 g(grid), b(block);
  switch (fk) {
    case QED_FIELD_UNIFORM: launch_pair_events_fk<QED_FIELD_UNIFORM>(a, g, b, s, mixed); break;
    case QED_FIELD_LP_PULSE: launch_pair_events_fk<QED_FIELD_LP_PULSE>(a, g, b, s, mixed); break;
    case QED_FIELD_CP_WAVE: launch_pair_events_fk<QED_FIELD_CP_WAVE>(a, g, b, s, mixed); break;
    case QED_FIELD_CP_STANDING: launch_pair_events_fk<QED_FIELD_CP_STANDING>(a, g, b, s, mixed); break;
    case QED_FIELD_GRID_FDTD: launch_pair_events_fk<QED_FIELD_GRID_FDTD>(a, g, b, s, mixed); break;
    default: launch_pair_events_fk<QED_FIELD_GRID_CP_STANDING>(a, g, b, s, mixed); break;
  }
}

// Blocks of the photon sweep that fit on one CU at once (registers, LDS), for the shape given.
template <int FK, int PPT>
static int photon_fit_ppt(int block, size_t shm, bool mixed) {
  int n = 0;
  const hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_photon<FK, PPT, true>, block, shm)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_photon<FK, PPT, false>, block, shm);
  return e == hipSuccess ? n : 0;
}
template <int FK>
static int photon_fit_fk(int ppt, int block, size_t shm, bool mixed) {
  switch (ppt) {
    case 1: return photon_fit_ppt<FK, 1>(block, shm, mixed);
    case 2: return photon_fit_ppt<FK, 2>(block, shm, mixed);
    case 8: return photon_fit_ppt<FK, 8>(block, shm, mixed);
    case 16: return photon_fit_ppt<FK, 16>(block, shm, mixed);
    default: return photon_fit_ppt<FK, 4>(block, shm, mixed);
  }
}
static size_t photon_shm(int n_cp) { return (size_t)n_cp * sizeof(double) + 16 * 3 * sizeof(unsigned) + 64; }
int photon_blocks_per_cu(int fk, int ppt, int block, int n_cp, bool mixed) {
  const size_t shm = photon_shm(n_cp);
  switch (fk) {
    case QED_FIELD_UNIFORM: return photon_fit_fk<QED_FIELD_UNIFORM>(ppt, block, shm, mixed);
    case QED_FIELD_LP_PULSE: return photon_fit_fk<QED_FIELD_LP_PULSE>(ppt, block, shm, mixed);
    case QED_FIELD_CP_WAVE: return photon_fit_fk<QED_FIELD_CP_WAVE>(ppt, block, shm, mixed);
    case QED_FIELD_CP_STANDING: return photon_fit_fk<QED_FIELD_CP_STANDING>(ppt, block, shm, mixed);
    case QED_FIELD_GRID_FDTD: return photon_fit_fk<QED_FIELD_GRID_FDTD>(ppt, block, shm, mixed);
    default: return photon_fit_fk<QED_FIELD_GRID_CP_STANDING>(ppt, block, shm, mixed);
  }
}

void launch_photon(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s) {
  const size_t shm = photon_shm(a.tb.n_cp);  // T table and block reduction
  const dim3 g(grid), b(block);
  switch (fk) {
    case QED_FIELD_UNIFORM: launch_photon_fk<QED_FIELD_UNIFORM>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_LP_PULSE: launch_photon_fk<QED_FIELD_LP_PULSE>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_CP_WAVE: launch_photon_fk<QED_FIELD_CP_WAVE>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_CP_STANDING: launch_photon_fk<QED_FIELD_CP_STANDING>(a, g, b, shm, s, mixed); break;
    case QED_FIELD_GRID_FDTD: launch_photon_fk<QED_FIELD_GRID_FDTD>(a, g, b, shm, s, mixed); break;
    default: launch_photon_fk<QED_FIELD_GRID_CP_STANDING>(a, g, b, shm, s, mixed); break;
  }
}

void launch_init_tau(const qed_instance* inst, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_init_tau, dim3(64, 3 * n_inst), dim3(256), 0, s, inst);
}

void launch_ledger(const qed_instance* inst, int n_inst, InstAcc* acc, bool mixed, hipStream_t s) {
  hipLaunchKernelGGL(k_ledger_zero, dim3(1), dim3(256), 0, s, acc, n_inst);
  if (mixed) hipLaunchKernelGGL(k_ledger<true>, dim3(128, 3 * n_inst), dim3(256), 0, s, inst, acc);
  else hipLaunchKernelGGL(k_ledger<false>, dim3(128, 3 * n_inst), dim3(256), 0, s, inst, acc);
}

void launch_photon_windows(int fk, const qed_instance* inst, int n_inst, InstAcc* acc, const Glob* glob, uint32_t* win,
                           void* rec, uint64_t* lmask, double t0, double dt, double cp_min, bool mixed, hipStream_t s) {
  const dim3 g(n_inst == 1 ? 2048 : 64, n_inst);
  constexpr int LP = QED_FIELD_LP_PULSE, GEN = QED_FIELD_UNIFORM;  // record layouts: plane wave, general
  if (fk == LP) {
    if (mixed) hipLaunchKernelGGL((k_photon_windows<true, LP>), g, dim3(256), 0, s, inst, acc, win, rec, t0, dt, cp_min);
    else hipLaunchKernelGGL((k_photon_windows<false, LP>), g, dim3(256), 0, s, inst, acc, win, rec, t0, dt, cp_min);
  } else {
    if (mixed) hipLaunchKernelGGL((k_photon_windows<true, GEN>), g, dim3(256), 0, s, inst, acc, win, rec, t0, dt, cp_min);
    else hipLaunchKernelGGL((k_photon_windows<false, GEN>), g, dim3(256), 0, s, inst, acc, win, rec, t0, dt, cp_min);
  }
  hipLaunchKernelGGL(k_window_masks, g, dim3(256), 0, s, inst, acc, glob, win, lmask);
  hipLaunchKernelGGL(k_window_front, dim3(1), dim3(256), 0, s, inst, n_inst, acc, 0);
}

void launch_compact(int fk, const qed_instance* inst, int n_inst, InstAcc* acc, const Glob* glob, int64_t* movers,
                    uint32_t* win, void* rec, uint64_t* lmask, bool mixed, const RetireSpec& rs, hipStream_t s) {
  const int rw = photon_rec_bytes(mixed, fk) / 8;
  RetireArgs r{};
  r.on = rs.on;
  r.n_bins = rs.n_bins;
  r.le_min = rs.on ? std::log(rs.e_min) : 0.0;
  r.inv_dle = rs.on ? rs.n_bins / (std::log(rs.e_max) - std::log(rs.e_min)) : 0.0;
  r.spec = rs.spec;
  r.step = 0;
  hipLaunchKernelGGL(k_compact_prep, dim3(1), dim3(256), 0, s, inst, n_inst, acc, r.on);
  // blocks per instance: enough to stream one large instance at full bandwidth; blocks past an
  // instance's photons (or of an instance with nothing to remove) return at once
  const dim3 g(n_inst == 1 ? 2048 : 256, n_inst);
  const size_t shm = r.on ? (size_t)(r.n_bins + 2) * sizeof(unsigned) : 0;
  if (mixed) hipLaunchKernelGGL(k_compact_count<true>, g, dim3(256), shm, s, inst, acc, glob, win, r);
  else hipLaunchKernelGGL(k_compact_count<false>, g, dim3(256), shm, s, inst, acc, glob, win, r);
  hipLaunchKernelGGL(k_compact_movers, g, dim3(256), 0, s, inst, acc, glob, movers, win, r);
  if (mixed) hipLaunchKernelGGL(k_compact_fill<true>, g, dim3(256), 0, s, inst, acc, glob, movers, win, rec, rw, r);
  else hipLaunchKernelGGL(k_compact_fill<false>, g, dim3(256), 0, s, inst, acc, glob, movers, win, rec, rw, r);
  hipLaunchKernelGGL(k_compact_finish, dim3(1), dim3(256), 0, s, inst, n_inst, acc);
  hipLaunchKernelGGL(k_part_prep, dim3(1), dim3(256), 0, s, inst, n_inst, acc);
  hipLaunchKernelGGL(k_part_count, g, dim3(256), 0, s, acc, glob, win);
  hipLaunchKernelGGL(k_part_movers, g, dim3(256), 0, s, acc, glob, win, movers);
  if (mixed) hipLaunchKernelGGL(k_part_swap<true>, g, dim3(256), 0, s, inst, acc, glob, movers, win, rec, rw);
  else hipLaunchKernelGGL(k_part_swap<false>, g, dim3(256), 0, s, inst, acc, glob, movers, win, rec, rw);
  hipLaunchKernelGGL(k_window_masks, g, dim3(256), 0, s, inst, acc, glob, win, lmask);
  hipLaunchKernelGGL(k_window_front, dim3(1), dim3(256), 0, s, inst, n_inst, acc, 1);
}

}  // namespace qedk
