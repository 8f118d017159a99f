// Device-side building blocks of the QED Monte-Carlo step (gfx950, wave64):
// constants, the Philox4x64-10 stream, field providers, the Boris push, table
// look-ups and wavefront-aggregated appends.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/qed.h"
#include "qed_crmath.h"

namespace qedk {

// CODATA 2018
constexpr double kPi = 3.14159265358979323846;
constexpr double kAlpha = 7.2973525693e-3;             // fine-structure constant
constexpr double kLambdaCompton = 2.42631023867e-12;   // h/(m_e c) in metres

enum : uint64_t { KIND_INIT = 0, KIND_EMIT = 1, KIND_PAIR = 2 };

// Pointers into global memory.  Pointers read from the instance table are generic to the
// compiler, which would then address them with flat instructions (which also count against the
// LDS wait counter); the cast makes their loads and stores global ones.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// Element at a 32-bit byte offset from a uniform base: the address is formed as a scalar base
// plus a zero-extended 32-bit lane offset, the form global loads and stores take directly.
template <class T>
__device__ __forceinline__ gptr<T> at_off(gptr<T> base, unsigned elem) {
  return (gptr<T>)((__attribute__((address_space(1))) char*)base + elem * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ gptr<const T> at_off(gptr<const T> base, unsigned elem) {
  return (gptr<const T>)((__attribute__((address_space(1))) const char*)base + elem * (unsigned)sizeof(T));
}

// Values that are the same in every lane (loaded from a uniform address), moved to scalar
// registers so that address arithmetic on them stays scalar.
__device__ __forceinline__ int uni32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  return (T*)(uintptr_t)uni64((int64_t)(uintptr_t)p);
}
__device__ __forceinline__ double uni_f64(double v) { return __longlong_as_double(uni64(__double_as_longlong(v))); }

// Raw buffer access: a scalar resource (base, size in bytes) plus a 32-bit lane byte offset.
// Loads at or past the size return zero and stores there are dropped, in hardware.  Word 3 of
// the resource is the gfx9-family value for untyped (raw) access.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t bufres;
constexpr int kBufWord3 = 0x00020000;
// (base and size are made explicitly uniform: a resource must live in scalar registers)
template <class P>
__device__ __forceinline__ bufres make_buf(P base, uint32_t bytes) {
  const uint64_t b = (uint64_t)uni64((int64_t)(uintptr_t)base);
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)b, (short)0, uni32((int)bytes), kBufWord3);
}
template <class T>
__device__ __forceinline__ T buf_ld(bufres r, uint32_t byte_off);
template <>
__device__ __forceinline__ double buf_ld<double>(bufres r, uint32_t o) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
}
template <>
__device__ __forceinline__ float buf_ld<float>(bufres r, uint32_t o) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
}
template <>
__device__ __forceinline__ int32_t buf_ld<int32_t>(bufres r, uint32_t o) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0);
}
// N consecutive dwords from byte offset o (128-bit pieces, then a 64- and a 32-bit tail)
template <int N>
__device__ __forceinline__ void load_dwords(bufres r, uint32_t o, uint32_t* q) {
#pragma unroll
  for (int w = 0; w + 4 <= N; w += 4) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, o + 4u * w, 0, 0);
    q[w] = v[0];
    q[w + 1] = v[1];
    q[w + 2] = v[2];
    q[w + 3] = v[3];
  }
  constexpr int w4 = N / 4 * 4;
  if constexpr (N - w4 >= 2) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, o + 4u * w4, 0, 0);
    q[w4] = v[0];
    q[w4 + 1] = v[1];
  }
  if constexpr ((N - w4) % 2 == 1) q[N - 1] = __builtin_amdgcn_raw_buffer_load_b32(r, o + 4u * (N - 1), 0, 0);
}
__device__ __forceinline__ void buf_st(bufres r, uint32_t o, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, o, 0, 0);
}
__device__ __forceinline__ void buf_st(bufres r, uint32_t o, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, o, 0, 0);
}


// u-bins of the guide tables of the cumulative rows (a power of two, so u * kGuide is exact)
constexpr int kGuide = 64;

// Device copy of the tables plus their grid constants.
struct Tabs {
  int n_eta;
  double le0, dle;             // ln eta_min, ln-spacing of the eta rows
  double idle;                 // 1 / dle (rate look-ups only; the sampling divides)
  const double* h;
  const float* h32;
  const double* g;             // quantum reduction of the radiated power, per eta row (or NULL)
  int n_chi;
  const double* lnchi_min;     // per row: ln chi_0 and ln-spacing of the columns
  const double* dlnchi;
  const double* P;             // [n_eta][n_chi]
  const uint16_t* gP;          // [n_eta][kGuide + 1]: guide of each row's inversion
  int n_cp;
  double lc0, dlc;             // ln chi_pair_min, ln-spacing of the pair rows
  double idlc;                 // 1 / dlc (rate look-up only)
  double cp_min;               // chi_pair_min
  const double* T;
  const float* T32;
  int n_f;
  const double* f;             // f grid
  const double* Pf;            // [n_cp][n_f]
  const uint16_t* gPf;         // [n_cp][kGuide + 1]
};

// Step constants derived from qed_step_params.
struct StepConst {
  double t0, dt;
  double kappa;     // lambda_L / lambda_c = m c^2 / (hbar w)
  double a_gamma;   // sqrt(3) alpha kappa / (2 pi): eq. 2 in code time
  double a_pair;    // alpha kappa: eq. 3 in code time
  double a_rr;      // (2/3) alpha kappa: classical radiated power per eta^2 in code time (eq. 9)
  uint32_t flags;
};

// Per-instance device accumulators and step scratch.
struct InstAcc {
  int64_t n_start[3];          // particles present at the start of the step (or pass)
  int64_t n_live;              // compaction: live photons
  int64_t mover_off;           // offset of this instance's photon slots in the workspace's per-photon
                               // arrays (compaction movers, photon windows)
  int64_t lmask_off;           // offset of this instance's live masks (one per kWinGroup photon slots)
  int64_t n_front;             // photons [0, n_front) have no pair rate in any later step (their window
                               // is over; set by the partition at compaction)
  int64_t ph_first;            // first photon slot of the photon sweep's chunk list (n_front rounded
                               // down to a chunk)
  unsigned long long hole_ctr, mover_ctr;
  // energy sums of the ledger as exact fixed-point words (fix_split): field work, emission and
  // pair defects, dropped energy, radiated energy, retired photons' energy, then the three species
  long long fx[9][4];
  unsigned long long n_retired;          // photons retired at compaction (pair window over)
  unsigned long long led_count[3];
  unsigned long long n_emit, n_null, n_pair, n_dropped, n_range, n_nonfinite, n_field, n_field_lepton;
  unsigned long long n_active;           // photon steps inside the photon's window (evaluated in full)
  unsigned long long n_win_reads;        // photon slot-steps whose window word was read (live bit set)
  unsigned long long n_group_reads;      // live masks read
  unsigned long long particle_steps[3];  // particles (photon slots) present at the start of each step
  unsigned long long n_pair_compacted;   // n_pair at the last compaction (~0: unknown, e.g. after bind)
  int32_t compact_skip;                  // this compaction has nothing to remove
  int32_t pad_;
};

// ---------------------------------------------------------------------------
// Exact, order-independent energy sums for the ledger.  A term v is cut into integer limbs of
// v 2^64 with weights 2^-64, 2^-32, 2^0 and 2^32 (bits below 2^-64 truncated toward zero; every
// limb carries the sign of v; |v| < 2^62), and limbs are added into 64-bit integer words.
// Integer addition is associative, so a sum does not depend on the order of its terms: not on
// the launch shape, the block schedule or the order of an event queue.  The words are
// normalised once per step (carries moved up), so each word stays far from overflow.
// ---------------------------------------------------------------------------
enum { FX_WORK = 0, FX_DEFECT_EMIT = 1, FX_DEFECT_PAIR = 2, FX_DROPPED = 3, FX_RADIATED = 4, FX_RETIRED = 5,
       FX_ENERGY = 6 };
constexpr int kFixRunning = 6;  // FX_WORK..FX_RETIRED accumulate over the run

__device__ __forceinline__ void fix_split(double v, long long l[4]) {
  v = v > 0x1p62 ? 0x1p62 : v < -0x1p62 ? -0x1p62 : v == v ? v : 0.0;  // non-finite state is counted apart
  double a = v * 0x1p64;                // exact scaling
  const double t3 = trunc(a * 0x1p-96);
  a -= t3 * 0x1p96;                     // exact: the bits of a below 2^96
  const double t2 = trunc(a * 0x1p-64);
  a -= t2 * 0x1p64;
  const double t1 = trunc(a * 0x1p-32);
  a -= t1 * 0x1p32;
  l[0] = (long long)trunc(a);
  l[1] = (long long)t1;
  l[2] = (long long)t2;
  l[3] = (long long)t3;
}

__device__ __forceinline__ void fix_atomic_add(long long* w, const long long l[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (l[k]) atomicAdd((unsigned long long*)&w[k], (unsigned long long)l[k]);
}

// carries of words 0..2 moved up: afterwards words 0..2 lie in [0, 2^32)
__device__ __forceinline__ void fix_normalise(long long* w) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const long long c = w[k] >> 32;  // floor division by 2^32
    w[k] -= (long long)((unsigned long long)c << 32);
    w[k + 1] += c;
  }
}

// Workspace-global device state.
struct Glob {
  int64_t step_cur, step_next;   // device clock: index of the running / next step
  int64_t n_chunks[2];           // chunk-list lengths: 0 leptons, 1 photons
};

// Pair-event queue of one step: the photon sweep appends (instance << 40 | slot) of every photon
// whose optical depth reached zero; the event pass converts them.  When more events occur than
// the queue holds, `overflow` is set and the event pass finds them by a sweep over the photons.
struct EvCtl {
  int64_t count;
  int32_t overflow;
  int32_t pad;
};
struct EvQueue {
  EvCtl* ctl;
  uint64_t* ent;
  int64_t cap;
};
// Emission-event queue: (instance << 41 | species << 40 | slot) and the emitter's eta.  Every wave
// of the lepton sweep owns a segment of it: wave w of block b writes its events, in slot order, from
// entry (b nw + w) seg_len on, where seg_len = per_block * ppt * 64 is the number of lepton slots the
// wave handles in the step (per_block = chunks per block), and stores their number in
// wave_cnt[b nw + w].  No atomics, and no overflow: a lepton emits at most once per step.  The queue
// holds the bound leptons plus the rounding of the chunk list and of the blocks' runs of it.
struct EmitEv {
  uint64_t key;
  double eta;
};
struct EmitQueue {
  EvCtl* ctl;
  EmitEv* ent;
  int64_t cap;
  int32_t* wave_cnt;   // events per wave of the lepton sweep (its grid x blockDim / 64 entries)
  int grid;            // lepton-sweep blocks
  int waves;           // lepton-sweep waves per block
  int ppt;             // lepton-sweep particles per thread
};
constexpr int kEvSlotBits = 40;
// state of a photon's optical depth: >= 0 live, [kTauPendingMin, 0] converting this step, -1 gone
constexpr double kTauGone = -1.0;
constexpr double kTauPendingMin = -0.5;

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
  // periodic index in [0, n): the in-range and one-off cases (almost every particle) without the
  // 64-bit remainder, which the GPU evaluates in software
  if (i >= 0 && i < n) return i;
  if (i == -1) return n - 1;
  if (i == n) return 0;
  const int64_t r = i % n;
  return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// Compact sin/cos and log for values that only set optical-depth decrements (the step decided
// by a decrement is insensitive to their last bits; momenta always use the correctly rounded
// functions).  Written out so that the kernels carry no large-argument reduction code: fewer
// instructions and registers than the general library routines.
// ---------------------------------------------------------------------------
namespace fastm {
constexpr double f2 = 1.0 / 2.0, f3 = 1.0 / 6.0, f4 = 1.0 / 24.0, f5 = 1.0 / 120.0, f6 = 1.0 / 720.0,
                 f7 = 1.0 / 5040.0, f8 = 1.0 / 40320.0, f9 = 1.0 / 362880.0, f10 = 1.0 / 3628800.0,
                 f11 = 1.0 / 39916800.0, f12 = 1.0 / 479001600.0, f13 = 1.0 / 6227020800.0,
                 f14 = 1.0 / 87178291200.0, f15 = 1.0 / 1307674368000.0, f16 = 1.0 / 20922789888000.0,
                 f17 = 1.0 / 355687428096000.0, f18 = 1.0 / 6402373705728000.0;
}  // namespace fastm

// sin and cos of x, |x| < 2^20: x = k pi/2 + r by Cody-Waite reduction (pi/2 in three parts, the
// first with 33 bits so that k times it is exact), |r| <= pi/4, Taylor polynomials to r^13 and
// r^14 in fused multiply-adds (truncation below 3e-14 and 1e-15 relative); quadrant from k mod 4.
// These values only set optical-depth decrements, where the parity bars allow 1e-10 in the
// depth; the short polynomials keep the kernels' 64-bit constants (scalar registers) few.
// Both polynomials are evaluated and the quadrant selects (no divergent branch).
__device__ __forceinline__ void fast_sincos_r(double x, double* sv, double* cv, int* q) {
  using namespace fastm;
  const double k = rint(x * kTwoOverPi);
  double r = fma(-k, kPio2A, x);
  r = fma(-k, kPio2B, r);
  r = fma(-k, kPio2C, r);
  const double r2 = r * r;
  double ps = fma(f13, r2, -f11);
  double pc = fma(f14, r2, -f12);
  ps = fma(ps, r2, f9);
  pc = fma(pc, r2, f10);
  ps = fma(ps, r2, -f7);
  pc = fma(pc, r2, -f8);
  ps = fma(ps, r2, f5);
  pc = fma(pc, r2, f6);
  ps = fma(ps, r2, -f3);
  pc = fma(pc, r2, -f4);
  *sv = fma(r * r2, ps, r);                    // r + r^3 (-1/3! + ...)
  *cv = fma(r2 * r2, -pc, fma(-0.5, r2, 1.0));  // 1 - r^2/2 + r^4 (1/4! - ...)
  *q = (int)(int64_t)k;
}
__device__ __forceinline__ void fast_sincos(double x, double* sn, double* cs) {
  double sv, cv;
  int k;
  fast_sincos_r(x, &sv, &cv, &k);
  const int q = k & 3;
  *sn = (q & 1) ? cv : sv;
  *cs = (q & 1) ? sv : cv;
  if (q == 1 || q == 2) *cs = -*cs;
  if (q & 2) *sn = -*sn;
}
// sin(x + qs pi/2): qs = 0 sin, qs = 1 cos
__device__ __forceinline__ double fast_sinq(double x, int qs) {
  double sv, cv;
  int k;
  fast_sincos_r(x, &sv, &cv, &k);
  const int q = (k + qs) & 3;
  const double v = (q & 1) ? cv : sv;
  return (q & 2) ? -v : v;
}
__device__ __forceinline__ double fast_sin(double x) { return fast_sinq(x, 0); }
__device__ __forceinline__ double fast_cos(double x) { return fast_sinq(x, 1); }

// Natural log of a finite x > 0 with a table of kLogTab reciprocals: x = m 2^e with m in
// [1/2, 1); j = the 7 mantissa bits after the leading one picks c_j ~ 1/m (the centre of the
// j-th of 128 equal sub-intervals) and L_j = -log c_j (both rounded to double, computed on the
// host); r = m c_j - 1 (one rounding, |r| <= 2^-8) and log x = e log 2 + L_j + log1p(r), the
// series of log1p to r^5 (truncation below 1e-17 absolute).  Absolute error ~1e-16: the value
// only places a look-up between table rows.  `tab` holds c_j, L_j interleaved (an LDS copy).
constexpr int kLogTab = 128;
static __constant__ double c_logtab[2 * kLogTab];  // c_j, L_j (uploaded with the device math constants)
// LDS copy of the log table for a block (every thread calls this, then a barrier follows)
__device__ __forceinline__ void stage_logtab(double* dst) {
  for (int i = threadIdx.x; i < 2 * kLogTab; i += blockDim.x) dst[i] = c_logtab[i];
}
__device__ __forceinline__ double fast_log(double x, const double* tab) {
  int e;
  const double m = frexp(x, &e);
  const int j = (int)((uint32_t)(__double_as_longlong(m) >> 45) & (kLogTab - 1));
  const double2 cl = ((const double2*)tab)[j];
  const double r = fma(m, cl.x, -1.0);
  double p = fma(1.0 / 5.0, r, -0.25);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  const double l1p = fma(r * r, p, r);
  const double ed = (double)e;
  return fma(ed, kLn2Hi, cl.y) + fma(ed, kLn2Lo, l1p);
}

// FP32 sin and cos of |x| <= 4 (phases already reduced in FP64): Cody-Waite by pi/2 in two FP32
// parts, Taylor polynomials to r^11 and r^10 in fused multiply-adds, quadrant by selection.
__device__ __forceinline__ void fast_sincosf(float x, float* sn, float* cs) {
  const float k = rintf(x * 0.636619772f);
  const float r = fmaf(-k, -4.37113883e-8f, fmaf(-k, 1.57079637f, x));
  const float r2 = r * r;
  float ps = fmaf(-2.50521084e-8f, r2, 2.75573192e-6f);
  float pc = fmaf(2.08767570e-9f, r2, -2.75573192e-7f);
  ps = fmaf(ps, r2, -1.98412698e-4f);
  pc = fmaf(pc, r2, 2.48015873e-5f);
  ps = fmaf(ps, r2, 8.33333333e-3f);
  pc = fmaf(pc, r2, -1.38888889e-3f);
  ps = fmaf(ps, r2, -1.66666667e-1f);
  pc = fmaf(pc, r2, 4.16666667e-2f);
  const float sv = fmaf(r * r2, ps, r);
  const float cv = fmaf(r2 * r2, pc, fmaf(-0.5f, r2, 1.0f));
  const int q = (int)k & 3;
  float s = (q & 1) ? cv : sv, c = (q & 1) ? sv : cv;
  if (q & 2) s = -s;
  if (q == 1 || q == 2) c = -c;
  *sn = s;
  *cs = c;
}

// Per-instance constants of a field derived once per kernel and instance (fast paths only).
struct FieldK {
  double pi_over_len;  // plane-wave pulse: pi / Psi
};
__device__ __forceinline__ FieldK field_k(const qed_field& F) {
  FieldK k;
  k.pi_over_len = F.kind == QED_FIELD_LP_PULSE ? kPi / F.p[1] : 0.0;
  return k;
}
constexpr double kInvTwoPi = 0.15915494309189533577;

// An upper bound of |E| + |B| anywhere in a field (grid kind: the standing wave its refresh
// writes; bilinear weights keep interpolated values within the node values).  Since
// chi = (eps/2)(|E + n x B|^2 - (n.E)^2)^(1/2) <= (eps/2)(|E| + |B|), photons with
// eps < 2 chi_min / bound see no pair rate (T = 0 below the table).
__device__ __forceinline__ double field_bound(const qed_field& F) {
  switch (F.kind) {
    case QED_FIELD_UNIFORM:
      return sqrt(F.p[0] * F.p[0] + F.p[1] * F.p[1] + F.p[2] * F.p[2]) +
             sqrt(F.p[3] * F.p[3] + F.p[4] * F.p[4] + F.p[5] * F.p[5]);
    case QED_FIELD_LP_PULSE:
    case QED_FIELD_CP_WAVE:
      return 2.0 * fabs(F.p[0]);
    case QED_FIELD_GRID_FDTD:  // evolving fields: no bound
      return INFINITY;
    default:  // standing waves: |E|, |B| <= 2 a each
      return 4.0 * fabs(F.p[0]);
  }
}

// Photons below this energy have no pair rate in the field: chi <= (eps / 2) field_bound, and T
// is zero below the table's chi_min (margin for the FP32 rounding of eps and chi).
__device__ __forceinline__ double pair_eps_min(const qed_field& F, double cp_min) {
  return 2.0 * cp_min / field_bound(F) * (1.0 - 1e-5);
}

// What the photon sweep reads of a photon inside its window, in one line: a copy of its stored
// direction-and-birth state (64 bytes in FP64; 32 bytes, the stored FP32 values, in the FP32-mixed
// form).  The SoA arrays of a sparse set of photons would cost a line per array.
struct __attribute__((aligned(64))) PhotonRec {
  double kx, ky, kz, xb, yb;
  int32_t bs;
  int32_t pad0;
  double pad1[2];
};
struct __attribute__((aligned(32))) PhotonRec32 {
  float kx, ky, kz, xb, yb;
  int32_t bs;
  int32_t pad[2];
};
// In the plane-wave pulse the field at a photon depends only on psi = t - x - psi0, which is
// linear in the step index along the photon's straight path: psi(n) = A + n S with
// A = t0 - x_b - psi0 + b dt n_x and S = dt (1 - n_x).  The pulse's E and B give
// chi = (eps/2)(1 - n_x)|e(psi)| = c |e(psi)|, and the decrement of eq. 3,
// a_pair chi T(chi)/eps dt, is a_pair |e| T(chi) S / 2.  So the record holds A, S and c:
// 24 bytes in FP64, 16 in the FP32-mixed form (A in FP64).
struct __attribute__((aligned(8))) PhotonRecPW {
  double A, S, c;
};
struct __attribute__((aligned(16))) PhotonRecPW32 {
  double A;
  float S, c;
};
template <bool MIXED, int FK>
using PhotonRecT = typename std::conditional<
    FK == QED_FIELD_LP_PULSE, typename std::conditional<MIXED, PhotonRecPW32, PhotonRecPW>::type,
    typename std::conditional<MIXED, PhotonRec32, PhotonRec>::type>::type;

// bytes of one record for a precision and field kind (a multiple of 8)
__host__ __device__ constexpr int photon_rec_bytes(bool mixed, int fk) {
  return fk == QED_FIELD_LP_PULSE ? (mixed ? 16 : 24) : (mixed ? 32 : 64);
}
static_assert(sizeof(PhotonRecPW) == 24 && sizeof(PhotonRecPW32) == 16 && sizeof(PhotonRec) == 64 &&
                  sizeof(PhotonRec32) == 32,
              "record sizes as photon_rec_bytes states them");

// 1 - n_x of a direction k (|k| = eps) without cancellation for photons moving along +x
__device__ __forceinline__ double one_minus_nx(double kx, double ky, double kz, double eps) {
  return kx > 0.0 ? (ky * ky + kz * kz) / (eps * (eps + kx)) : 1.0 - kx / eps;
}

// The record of a photon from its stored state (momentum k, birth position and step).
template <bool MIXED, int FK>
__device__ inline void make_photon_rec(PhotonRecT<MIXED, FK>& R, const qed_field& F, double t0, double dt,
                                       double kx, double ky, double kz, double xb, double yb, int32_t bs) {
  if constexpr (FK == QED_FIELD_LP_PULSE) {
    const double eps = sqrt(kx * kx + ky * ky + kz * kz);
    const double omn = eps > 0.0 ? one_minus_nx(kx, ky, kz, eps) : 0.0;
    const double nx = eps > 0.0 ? kx / eps : 0.0;
    const double A = (t0 - xb - F.p[2]) + (double)bs * dt * nx;
    R.A = A;
    R.S = dt * omn;
    R.c = 0.5 * eps * omn;
    (void)yb;
  } else {
    R.kx = kx;
    R.ky = ky;
    R.kz = kz;
    R.xb = xb;
    R.yb = yb;
    R.bs = bs;
  }
}

// A window is stored in 32 bits: first and last step as 16-bit fields (lo | hi << 16), saturated
// so that the stored window always holds the exact one: lo at 65535 stands for "from 65535 or
// later", hi at 65535 for "no last step".  An empty window is lo = 65535, hi = 0.  Past step
// 65535 only the windows without a last step stay open: that culls less, never wrongly.
constexpr uint32_t kWinEmpty = 0x0000FFFFu;
__device__ __forceinline__ uint32_t pack_window(int2 w) {
  if (w.x > w.y || w.y < 0) return kWinEmpty;  // empty, or over before step 0
  const uint32_t lo = (uint32_t)min(max(w.x, 0), 65535);
  const uint32_t hi = w.y >= 65535 ? 65535u : (uint32_t)w.y;
  return lo | (hi << 16);
}
__device__ __forceinline__ bool in_window(uint32_t w, int64_t n) {
  const int64_t lo = w & 0xFFFFu, hi = w >> 16;
  return lo <= hi && lo <= (n < 65535 ? n : 65535) && (hi == 65535 || n <= hi);
}
// the window has no step at or after step s (empty windows included)
__device__ __forceinline__ bool window_over(uint32_t w, int64_t s) {
  const uint32_t lo = w & 0xFFFFu, hi = w >> 16;
  return lo > hi || (hi != 65535u && (int64_t)hi < s);
}
// Photon slots are grouped by kWinGroup consecutive slots (one wave's share of a chunk).  A group's
// live mask has bit i set for every slot i of the group whose photon's window is not over at the
// next step the photon sweep runs (it may have more bits set, never fewer): the sweep reads only
// the slots whose bit is set.  Set for a new photon by the emission pass, cleared by the sweep
// once the window is over, rebuilt from the windows after a window build or a compaction.
constexpr int kWinGroup = 64;

// The steps [lo, hi] in which a photon can have a pair rate (eq. 3 needs chi >= chi_min); in
// every other step its QED step is a no-op.  Empty (lo > hi) below pair_eps_min.  In a plane
// wave along x (E_y = B_z = e for the pulse; |E| = |B| = E0 for the CP wave) a photon with
// direction n sees |E + n x B|^2 - (n.E)^2 = (1 - n_x)^2 e^2, so chi = (eps/2)(1 - n_x)|e|:
// the CP wave gives a constant chi, and in the pulse chi <= (eps/2)(1 - n_x) E0 sin^2(pi psi/Psi),
// which reaches chi_min only for psi in [psi_a, Psi - psi_a].  psi = t - x - psi0 at the photon
// grows linearly in the step index n (by dt (1 - n_x) >= 0 per step, x = x_b + (n - b) dt n_x),
// so those steps form one interval.  Allowances: (1 - n_x) e and chi as the FP32 sweep evaluates
// them (cancellation of e - n_x e, rounding of eps, E0 and the FP32 sine), and psi as either
// sweep forms it (FP64 sums; the FP32 direction n_x, ~5e-7 relative, times the photon's age).
// Other fields get no finite support.
__device__ inline int2 photon_window(const qed_field& F, double eps_min, double cp_min, double t0, double dt,
                                     double kx, double ky, double kz, double xb, int32_t bs) {
  const int2 none = make_int2(INT_MAX, INT_MIN), all = make_int2(INT_MIN, INT_MAX);
  const double eps = sqrt(kx * kx + ky * ky + kz * kz);
  if (!(eps >= eps_min)) return none;
  if (F.kind != QED_FIELD_LP_PULSE && F.kind != QED_FIELD_CP_WAVE) return all;
  // 1 - n_x without cancellation for photons moving along +x
  const double omn = one_minus_nx(kx, ky, kz, eps);
  // FP32: e - n_x e and the rounding of |a|^2 - (n.e)^2 (whose parts are up to 2 (1 - n_x) e^2)
  // add at most ~1e-7 + sqrt(1.2e-7 (1 - n_x)) to (1 - n_x); eps, E0 and sin^2 ~1e-6 relative
  const double cmax = 0.5 * eps * (omn + 1e-6 + sqrt(1e-6 * omn)) * fabs(F.p[0]) * (1.0 + 1e-5);
  if (!(cmax >= cp_min)) return none;
  if (F.kind == QED_FIELD_CP_WAVE) return all;
  const double nx = kx / eps, len = F.p[1], psi0 = F.p[2];
  const double psa = len / kPi * asin(sqrt(cp_min / cmax)) * (1.0 - 1e-9);  // sin^2 >= cp_min / cmax
  const double S = dt * (1.0 - nx);                                         // psi(n) = A + S n
  const double A = (t0 - xb - psi0) + (double)bs * dt * nx;
  const double r = 1e-6 * dt;                                               // per step of age
  const double m = 1e-9 * (fabs(t0) + fabs(xb) + fabs(psi0) + len + fabs((double)bs * dt)) + 1e-9;
  // A + S n >= psa - m - r (n - b)   and   A + S n <= len - psa + m + r (n - b)
  const double lo = (psa - m - A + r * bs) / (S + r);
  const double hi = S - r > 0.0 ? (len - psa + m - A - r * bs) / (S - r) : INFINITY;
  const double lim = 2.0e9;
  const int ilo = lo < -lim ? INT_MIN : lo > lim ? INT_MAX : (int)floor(lo) - 2;
  const int ihi = hi > lim ? INT_MAX : hi < -lim ? INT_MIN : (int)ceil(hi) + 2;
  if (!(lo <= hi + 4.0)) return none;  // also NaN
  return make_int2(ilo, ihi);
}

// First-order (cloud-in-cell) gather of the six components at (x, y): bilinear weights over the
// four nodes around the point on each component's staggered grid (Yee offsets), periodic; node
// values of type T (FP32 refreshed grid, FP64 solver grid).
template <class T>
__device__ __forceinline__ void cic_gather6(const qed_field& F, const T* base, double x, double y, double E[3],
                                            double B[3]) {
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
    gptr<const T> g = as_global(base + c * plane);
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

// Current of one macro-particle of charge Q moving in one step (dt) from (x0, y0) to (x1, y1),
// less than a cell in each direction, with z velocity vz, added to the planes J (Jx, Jy, Jz at
// the nodes of Ex, Ey, Ez): the charge-conserving split of Esirkepov for first-order shapes in
// 2-D.  With the old and new shape factors S0, S1 of the (up to) three nodes per direction the
// particle touches and D = S1 - S0: Wx = Dx (S0y + Dy/2), Wy = Dy (S0x + Dx/2),
// Wz = S0x S0y + Dx S0y/2 + S0x Dy/2 + Dx Dy/3; Jx(i+1/2, j) = -Q/(dy dt) sum_{i'<=i} Wx,
// Jy(i, j+1/2) = -Q/(dx dt) sum_{j'<=j} Wy, Jz = Q vz Wz/(dx dy).  The discrete continuity
// equation then holds node by node for the cloud-in-cell density.  FP64 atomic adds (the
// order of the sums over particles is not fixed).
// A deposit target: LDS words of a block's node box (unwrapped node indices [ox, ox + W) x
// [oy, oy + H), three planes), or, with W = 0, the grid's current planes through global atomics.
constexpr int kDepNodes = 2048;  // LDS budget of a lepton-sweep block's current box, in nodes
struct DepositSink {
  double* lds = nullptr;
  int64_t ox = 0, oy = 0;
  int W = 0, H = 0;
};

__device__ __forceinline__ void deposit_current(const qed_field& F, double Q, double dt, double x0, double y0,
                                                double x1, double y1, double vz, const DepositSink& sink = {}) {
  const double gx0 = (x0 - F.x0) / F.dx, gy0 = (y0 - F.y0) / F.dy;
  const double gx1 = (x1 - F.x0) / F.dx, gy1 = (y1 - F.y0) / F.dy;
  const double bx = floor(fmin(gx0, gx1)), by = floor(fmin(gy0, gy1));
  const int64_t I = (int64_t)bx, Jn = (int64_t)by;
  double S0x[3], S1x[3], S0y[3], S1y[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S0x[a] = fmax(0.0, 1.0 - fabs(gx0 - (bx + a)));
    S1x[a] = fmax(0.0, 1.0 - fabs(gx1 - (bx + a)));
    S0y[a] = fmax(0.0, 1.0 - fabs(gy0 - (by + a)));
    S1y[a] = fmax(0.0, 1.0 - fabs(gy1 - (by + a)));
  }
  const bool lds = sink.W > 0;
  const int64_t plane = lds ? (int64_t)sink.W * sink.H : (int64_t)F.nx * F.ny;
  const int64_t nxp = lds ? sink.W : F.nx;
  double* const Jx = lds ? sink.lds : F.fdtd_dev + 6 * plane;
  double* const Jy = Jx + plane;
  double* const Jz = Jy + plane;
  const double cx = -Q / (F.dy * dt), cy = -Q / (F.dx * dt), cz = Q * vz / (F.dx * F.dy);
  int64_t ii[3], jj[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ii[a] = lds ? I + a - sink.ox : wrap_index(I + a, F.nx);
    jj[a] = lds ? Jn + a - sink.oy : wrap_index(Jn + a, F.ny);
  }
  auto add = [&](double* w, double v) {
    if (v == 0.0) return;
    if (lds) atomicAdd(w, v);  // LDS
    else unsafeAtomicAdd(w, v);
  };
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    double run = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double dxa = S1x[a] - S0x[a], dyb = S1y[b] - S0y[b];
      run += dxa * (S0y[b] + 0.5 * dyb);
      const double wz = S0x[a] * S0y[b] + 0.5 * dxa * S0y[b] + 0.5 * S0x[a] * dyb + dxa * dyb / 3.0;
      const int64_t k = jj[b] * nxp + ii[a];
      add(Jx + k, cx * run);
      add(Jz + k, cz * wz);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double run = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double dxa = S1x[a] - S0x[a], dyb = S1y[b] - S0y[b];
      run += dyb * (S0x[a] + 0.5 * dxa);
      add(Jy + jj[b] * nxp + ii[a], cy * run);
    }
  }
}

template <int FK, bool EXACT = true>
__device__ __forceinline__ void field_at(const qed_field& F, double x, double y, double t, double E[3],
                                         double B[3], const FieldK* K = nullptr) {
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
      double s, c, d;
      if (EXACT) {
        s = cr_sin(kPi * psi / F.p[1]);
        c = cr_cos(psi + F.p[3]);
      } else {  // K: pi / Psi precomputed
        s = fast_sin(psi * K->pi_over_len);
        c = fast_cos(psi + F.p[3]);
        (void)d;
      }
      const double e = F.p[0] * s * s * c;
      E[1] = e;
      B[2] = e;
    }
  } else if (FK == QED_FIELD_CP_WAVE) {
    const double psi = t - x + F.p[1];
    double sn, cs;
    if (EXACT) cr_sincos(psi, &sn, &cs);
    else fast_sincos(psi, &sn, &cs);
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
      fast_sincos(t, &st, &ct);
      fast_sincos(x, &sx, &cx);
    }
    E[1] = 2.0 * F.p[0] * ct * cx;
    E[2] = 2.0 * F.p[0] * st * cx;
    B[1] = 2.0 * F.p[0] * ct * sx;
    B[2] = 2.0 * F.p[0] * st * sx;
  } else if (FK == QED_FIELD_GRID_CP_STANDING) {
    cic_gather6(F, (const float*)F.grid_dev, x, y, E, B);
  } else if (FK == QED_FIELD_GRID_FDTD) {
    cic_gather6(F, (const double*)F.fdtd_dev, x, y, E, B);
  }
}

// ---------------------------------------------------------------------------
// table look-ups (Sec. 3: linear interpolation in the look-up tables)
// ---------------------------------------------------------------------------

// h(eta) from an LDS copy; clamped outside [eta_min, eta_max], counting eta > eta_max.  The
// rate only feeds the optical-depth decrement, so the device library's log serves.
__device__ __forceinline__ double lookup_h(const double* sh, const double* ltab, const Tabs& tb, double eta,
                                           unsigned& range) {
  if (eta == INFINITY) {
    ++range;
    return sh[tb.n_eta - 1];
  }
  const double s = (fast_log(eta, ltab) - tb.le0) * tb.idle;
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
// g(eta) for the deterministic radiation reaction: it changes momenta, so the index uses the
// correctly rounded log (both sides of the parity contract); clamped at the table ends.
__device__ __forceinline__ double lookup_g(const double* sg, const Tabs& tb, double eta, unsigned& range) {
  const double s = (cr_log(eta) - tb.le0) / tb.dle;
  if (!(s > 0.0)) return sg[0];
  if (s >= tb.n_eta - 1) {
    ++range;
    return sg[tb.n_eta - 1];
  }
  const int i = (int)floor(s);
  const double w = s - i;
  return (1.0 - w) * sg[i] + w * sg[i + 1];
}

__device__ __forceinline__ double lookup_T(const double* sT, const double* ltab, const Tabs& tb, double chi,
                                           unsigned& range) {
  if (!(chi >= tb.cp_min)) return 0.0;  // below the table (T ~ 0) or NaN
  if (chi == INFINITY) {
    ++range;
    return sT[tb.n_cp - 1];
  }
  const double s = (fast_log(chi, ltab) - tb.lc0) * tb.idlc;
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
__device__ __forceinline__ int row_inverse(const double* __restrict__ P, int n, double u, double* frac,
                                           const uint16_t* __restrict__ guide) {
  // the answer lies between the guides of u's bin and the next (guide tables: same answer as the
  // search over the whole row, in one or two probes instead of log2 n dependent loads)
  const int g = (int)(u * kGuide);
  int lo = guide[g], hi = guide[g + 1] + 1;
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
    const int j = row_inverse(P, tb.n_chi, u, &fr, tb.gP + (size_t)r * (kGuide + 1));
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
    const int j = row_inverse(tb.Pf + (size_t)r * tb.n_f, tb.n_f, u, &fr, tb.gPf + (size_t)r * (kGuide + 1));
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

// Slots for the block's `want` lanes from one counter with one atomic per block: wave counts by
// ballot, their prefix in LDS, one atomicAdd by thread 0.  Every thread of the block must call it
// the same number of times (it synchronises); s_wave holds >= 16 entries.
__device__ inline long long block_reserve(bool want, int64_t* counter, unsigned* s_wave, long long* s_base) {
  const unsigned long long m = __ballot(want);
  const int lane = __lane_id(), wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) s_wave[wv] = (unsigned)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned tot = 0;
    for (int w = 0; w < nw; ++w) {
      const unsigned c = s_wave[w];
      s_wave[w] = tot;
      tot += c;
    }
    *s_base = tot ? (long long)atomicAdd((unsigned long long*)counter, (unsigned long long)tot) : 0;
  }
  __syncthreads();
  const long long r = want ? *s_base + s_wave[wv] + __popcll(m & ((1ull << lane) - 1ull)) : -1;
  __syncthreads();  // s_wave and s_base are reused by the next call
  return r;
}

// Rank of a wanting thread among the wanting threads of its block (in thread order), and the
// block's total in *total; every thread of the block calls it (it holds two barriers).
__device__ inline unsigned block_rank(bool want, unsigned* s_wave, unsigned* total) {
  const unsigned long long m = __ballot(want);
  const int lane = __lane_id(), wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) s_wave[wv] = (unsigned)__popcll(m);
  __syncthreads();
  unsigned before = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const unsigned c = s_wave[w];
    if (w < wv) before += c;
    tot += c;
  }
  __syncthreads();  // s_wave is rewritten by the next call
  *total = tot;
  return before + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
}

// The contiguous range [b0, b1) of [lo, hi) that block `blk` of `nblk` takes: equal shares,
// each a multiple of the block size (so that every pass of the block covers whole blocks).
__device__ __forceinline__ void block_range(int64_t lo, int64_t hi, int blk, int nblk, int64_t* b0, int64_t* b1) {
  const int64_t len = hi > lo ? hi - lo : 0;
  const int64_t per = ((len + nblk - 1) / nblk + blockDim.x - 1) / blockDim.x * blockDim.x;
  *b0 = min(hi, lo + (int64_t)blk * per);
  *b1 = min(hi, *b0 + per);
}

// wave_reserve for lanes whose counters may differ: lanes are served one key (counter) at a time.
// Every lane of the wave must call it.
__device__ inline long long wave_reserve_grouped(bool want, int key, int64_t* counter) {
  long long res = -1;
  bool left = want;
  unsigned long long mask;
  while ((mask = __ballot(left)) != 0ull) {
    const int leader = __ffsll((long long)mask) - 1;
    const int lk = __shfl(key, leader);
    const bool mine = left && key == lk;
    const long long r = wave_reserve(mine, counter);
    if (mine) {
      res = r;
      left = false;
    }
  }
  return res;
}

// Two wave_reserve_grouped calls at once (one slot from each of two counters per wanting lane):
// the leader's two atomics are both in flight before either result is used.
__device__ inline void wave_reserve2_grouped(bool want, int key, int64_t* ca, int64_t* cb, long long* ra,
                                             long long* rb) {
  *ra = *rb = -1;
  bool left = want;
  unsigned long long mask;
  while ((mask = __ballot(left)) != 0ull) {
    const int leader = __ffsll((long long)mask) - 1;
    const int lk = __shfl(key, leader);
    const bool mine = left && key == lk;
    const unsigned long long m = __ballot(mine);
    const int lane = __lane_id();
    const unsigned long long total = (unsigned long long)__popcll(m);
    long long ba = 0, bb = 0;
    if (lane == leader) {
      ba = (long long)atomicAdd((unsigned long long*)ca, total);
      bb = (long long)atomicAdd((unsigned long long*)cb, total);
    }
    ba = __shfl(ba, leader);
    bb = __shfl(bb, leader);
    if (mine) {
      const int prefix = __popcll(m & ((1ull << lane) - 1ull));
      *ra = ba + prefix;
      *rb = bb + prefix;
      left = false;
    }
  }
}

// Sets bit `bit` of the 64-bit word `word` for every lane with a word (nullptr: none), with one
// atomic per distinct word of the wave (consecutive slots share their group's word).  Every lane
// of the wave must call it.
__device__ inline void wave_or_bit(uint64_t* word, int bit) {
  bool left = word != nullptr;
  unsigned long long mask;
  while ((mask = __ballot(left)) != 0ull) {
    const int leader = __ffsll((long long)mask) - 1;
    const long long lw = __shfl((long long)(uintptr_t)word, leader);
    const bool mine = left && (long long)(uintptr_t)word == lw;
    long long v = mine ? (long long)(1ull << bit) : 0ll;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    if (__lane_id() == leader) atomicOr((unsigned long long*)(uintptr_t)lw, (unsigned long long)v);
    if (mine) left = false;
  }
}

// sums over the 64 lanes of a wave, every lane active; every lane gets the result
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ unsigned wave_sum_u(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Event statistics of the lanes of a wave added to the accumulators of each lane's instance:
// one group of atomics per instance present in the wave.  kind 0: emission, 1: pair creation.
// The energies go in as exact fixed-point limbs (fix_split), summed over the lanes as integers.
// Every lane of the wave must call it, all lanes active.
__device__ inline void add_event_stats(int kind, bool has, int ii, InstAcc* acc, double defect, double dropped_e,
                                       unsigned n_ev, unsigned n_null, unsigned n_drop) {
  long long ld[4], le[4];
  fix_split(has ? defect : 0.0, ld);
  fix_split(has ? dropped_e : 0.0, le);
  bool left = has;
  unsigned long long mask;
  while ((mask = __ballot(left)) != 0ull) {
    const int leader = __ffsll((long long)mask) - 1;
    const int lk = __shfl(ii, leader);
    const bool mine = left && ii == lk;
    long long sd[4], se[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sd[k] = wave_sum_ll(mine ? ld[k] : 0ll);
      se[k] = wave_sum_ll(mine ? le[k] : 0ll);
    }
    const unsigned sv = wave_sum_u(mine ? n_ev : 0u);
    const unsigned sn = wave_sum_u(mine ? n_null : 0u);
    const unsigned sp = wave_sum_u(mine ? n_drop : 0u);
    if (__lane_id() == leader) {
      InstAcc& A = acc[lk];
      fix_atomic_add(A.fx[kind == 0 ? FX_DEFECT_EMIT : FX_DEFECT_PAIR], sd);
      fix_atomic_add(A.fx[FX_DROPPED], se);
      if (sv) atomicAdd(kind == 0 ? &A.n_emit : &A.n_pair, (unsigned long long)sv);
      if (sn) atomicAdd(&A.n_null, (unsigned long long)sn);
      if (sp) atomicAdd(&A.n_dropped, (unsigned long long)sp);
    }
    if (mine) left = false;
  }
}

// The key shared by all of the block's lanes that have `want` set: true (and the key in *out) when
// at least one lane wants and all wanting lanes hold the same key.  Every thread of the block must
// call it; s holds 3 ints per wave.
__device__ inline bool block_uniform_key(bool want, int key, int* s, int* out) {
  const unsigned long long m = __ballot(want);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int k0 = 0;
  bool uni = true;
  if (m) {
    k0 = __shfl(key, __ffsll((long long)m) - 1);
    uni = __ballot(want && key != k0) == 0ull;
  }
  if (__lane_id() == 0) {
    s[3 * wv] = m != 0ull;
    s[3 * wv + 1] = k0;
    s[3 * wv + 2] = uni;
  }
  __syncthreads();
  bool any = false, ok = true;
  int kk = 0;
  for (int w = 0; w < nw; ++w) {
    if (!s[3 * w]) continue;
    if (!any) {
      kk = s[3 * w + 1];
      any = true;
    } else if (s[3 * w + 1] != kk) {
      ok = false;
    }
    ok = ok && s[3 * w + 2];
  }
  __syncthreads();
  *out = kk;
  return any && ok;
}

// Event statistics of one instance gathered by a block over several rounds (thread 0 holds them),
// added to the instance's accumulators with one group of atomics at flush.
struct BlockEventStats {
  long long defect[4], dropped[4];
  unsigned long long n_ev, n_null, n_drop;
  int inst;  // -1: empty
  __device__ void clear() {
    for (int k = 0; k < 4; ++k) defect[k] = dropped[k] = 0;
    n_ev = n_null = n_drop = 0;
    inst = -1;
  }
  // block-wide sums of the lanes' values (every thread calls; s_ll holds 16 * 8 words, s_u 16 * 3)
  __device__ void add(const long long ld[4], const long long le[4], unsigned ev, unsigned nul, unsigned drp,
                      long long* s_ll, unsigned* s_u) {
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    long long wd[4], we[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wd[k] = wave_sum_ll(ld[k]);
      we[k] = wave_sum_ll(le[k]);
    }
    const unsigned sv = wave_sum_u(ev), sn = wave_sum_u(nul), sp = wave_sum_u(drp);
    if (__lane_id() == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s_ll[8 * wv + k] = wd[k];
        s_ll[8 * wv + 4 + k] = we[k];
      }
      s_u[3 * wv] = sv;
      s_u[3 * wv + 1] = sn;
      s_u[3 * wv + 2] = sp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 0; w < nw; ++w) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          defect[k] += s_ll[8 * w + k];
          dropped[k] += s_ll[8 * w + 4 + k];
        }
        n_ev += s_u[3 * w];
        n_null += s_u[3 * w + 1];
        n_drop += s_u[3 * w + 2];
      }
    }
    __syncthreads();
  }
  // thread 0 only
  __device__ void flush(int kind, InstAcc* acc) {
    if (inst >= 0) {
      InstAcc& A = acc[inst];
      fix_atomic_add(A.fx[kind == 0 ? FX_DEFECT_EMIT : FX_DEFECT_PAIR], defect);
      fix_atomic_add(A.fx[FX_DROPPED], dropped);
      if (n_ev) atomicAdd(kind == 0 ? &A.n_emit : &A.n_pair, n_ev);
      if (n_null) atomicAdd(&A.n_null, n_null);
      if (n_drop) atomicAdd(&A.n_dropped, n_drop);
    }
    clear();
  }
};

// Sum of the 64 lanes' values of one group of 64 consecutive particle slots (a wave's share of
// a chunk), converted to fixed point and added by lane 0 to the wave's words in LDS (`w`, four
// words).  The butterfly order depends only on the lane positions, i.e. on the slots, so the
// group sum is the same for any launch shape.  Every lane of the wave must call it.
__device__ __forceinline__ void fix_group_add(double v, long long* w) {
  const double s = wave_sum(v);
  if (__lane_id() == 0) {
    long long l[4];
    fix_split(s, l);
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] += l[k];
  }
}

// The block's per-wave LDS words (s_w[(wave * NQ + q) * 4 + k]) summed and added by thread 0 to
// the words of dst[q], then cleared.  Every thread of the block must call it.
template <int NQ>
__device__ inline void fix_block_flush(long long* s_w, long long* const (&dst)[NQ]) {
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      long long t[4] = {0, 0, 0, 0};
      for (int v = 0; v < nw; ++v)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          t[k] += s_w[(v * NQ + q) * 4 + k];
          s_w[(v * NQ + q) * 4 + k] = 0;
        }
      fix_atomic_add(dst[q], t);
    }
  }
  __syncthreads();
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

// block-wide sums of unsigned accumulators; result valid in thread 0.  Every thread must call.
template <int NU>
__device__ inline void block_sum_u(unsigned (&u)[NU], unsigned* su) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < NU; ++a) u[a] += __shfl_down(u[a], off);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < NU; ++a) su[wave * NU + a] = u[a];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) {
#pragma unroll
      for (int a = 0; a < NU; ++a) u[a] += su[w * NU + a];
    }
  }
  __syncthreads();
}

}  // namespace qedk
