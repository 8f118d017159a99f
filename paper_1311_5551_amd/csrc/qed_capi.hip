// C ABI of libqed (declared in include/qed.h): argument checking, device memory that the
// library owns (tables, workspace), kernel launch sequencing, HIP-graph replay and the
// energy ledger.  No call here computes physics on the host; every step of the method
// runs in the kernels of qed_tables.hip, qed_step.hip and qed_mixed.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qed_device.h"
#include "qed_kernels.h"

using namespace qedk;

namespace {

thread_local std::string g_err;

qed_status fail(qed_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(QED_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

qed_status check_device(int* dev_out, int* cus_out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(QED_ERR_DEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  *dev_out = dev;
  if (cus_out) *cus_out = prop.multiProcessorCount;
  return QED_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Value of fixed-point words (weights 2^-64, 2^-32, 2^0, 2^32; see fix_split): carries moved up,
// then the integer part (exact in 128 bits) plus the fraction, rounded once per part.
double fix_value(const long long* w_in) {
  long long w[4] = {w_in[0], w_in[1], w_in[2], w_in[3]};
  for (int k = 0; k < 3; ++k) {
    const long long c = w[k] >> 32;
    w[k] -= (long long)((unsigned long long)c << 32);
    w[k + 1] += c;
  }
  const __int128 ip = ((__int128)w[3] << 32) + w[2];
  const double frac = (double)w[1] * 0x1p-32 + (double)w[0] * 0x1p-64;  // in [0, 1)
  return (double)ip + frac;
}

// device memory check: `p` must lie in a device allocation with room for `bytes`
qed_status check_dev_range(const void* p, size_t bytes, const char* what, int inst, int sp) {
  if (!p) return fail(QED_ERR_ARG, "instance %d species %d: %s is NULL", inst, sp, what);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QED_ERR_ARG, "instance %d species %d: %s is not device memory", inst, sp, what);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(QED_ERR_ARG, "instance %d species %d: %s is not device memory", inst, sp, what);
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
    const char* b = (const char*)base;
    const char* q = (const char*)p;
    if (q + bytes > b + size)
      return fail(QED_ERR_ARG, "instance %d species %d: %s holds %zu bytes past %p, capacity needs %zu", inst, sp,
                  what, (size_t)(b + size - q), p, bytes);
  } else {
    (void)hipGetLastError();
  }
  return QED_OK;
}

}  // namespace

struct qed_tables {
  qed_table_params p{};
  int device = 0;
  double *h = nullptr, *lnchi_min = nullptr, *dlnchi = nullptr, *P = nullptr, *T = nullptr, *fgrid = nullptr,
         *Pf = nullptr, *knorm = nullptr, *g = nullptr;
  float *h32 = nullptr, *T32 = nullptr;
  uint16_t *gP = nullptr, *gPf = nullptr;  // guide tables of the cumulative rows (kGuide + 1 per row)
  std::vector<double> hh, hlnchi, hdlnchi, hP, hT, hf, hPf, hk, hg;
  bool has_g = false;
};

constexpr int64_t kDefaultEventQueue = int64_t(1) << 20;

struct qed_workspace {
  int device = 0;
  int cus = 256;
  int max_inst = 0;
  int n_inst = 0;
  bool bound = false;
  qed_precision prec = QED_FP64;
  int field_kind = 0;
  bool any_grid = false;
  int64_t fdtd_work = 0;  // field-feedback kind: work items of the largest grid's solver pass (0: none)
  std::vector<qed_instance> inst;
  std::vector<double> e0;
  qed_instance* d_inst = nullptr;
  InstAcc* d_acc = nullptr;
  Glob* d_glob = nullptr;
  EvCtl* d_evc = nullptr;  // [0] pair-event queue, [1] emission queue
  uint64_t* d_evq = nullptr;
  int64_t evq_cap = 0;
  EmitEv* d_emq = nullptr;
  int64_t emq_cap = 0;
  int32_t* d_wave_cnt = nullptr;  // emission events per wave of the lepton sweep (cus * 32 waves)
  RetireSpec retire;              // retirement of photons at compaction, and its spectra
  size_t spec_len = 0;
  int64_t lep_cap = 0;            // bound lepton slots (both species, all instances)
  SortScratch sort;  // allocated by the first qed_sort that needs it
  int64_t sort_cap = 0;
  int64_t* d_base = nullptr;  // 3 * max_inst: leptons (2 per instance) then photons
  int64_t* d_movers = nullptr;
  size_t movers_len = 0;
  // pair windows of the photons (one int2 per photon slot, instances at acc.mover_off), valid
  // for the step constants and table they were computed with
  uint32_t* d_win = nullptr;
  void* d_rec = nullptr;     // one record per photon slot (PhotonRecT: photon_rec_bytes each)
  int rec_bytes = 0;
  // blocks of the lepton [0] and photon [1] sweeps resident per CU for the shape in fit_key
  // (field kind, particles per thread, block, precision, table rows)
  int fit[2] = {0, 0};
  int fit_key[2][5] = {{-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}};
  int emit_fit = 0;                         // emission-pass blocks per CU (occupancy query)
  int emit_fit_key[3] = {-1, -1, -1};       // field kind, precision, lepton-sweep waves
  size_t win_len = 0;
  uint64_t* d_lmask = nullptr;  // live masks of the photon slot groups (kWinGroup slots each), at acc.lmask_off
  size_t lmask_len = 0;
  bool win_valid = false;
  double win_t0 = 0.0, win_dt = 0.0, win_cp_min = 0.0;
  int block[2] = {256, 256}, ppt[2] = {4, 4};  // launch shapes: [0] lepton sweep, [1] photon sweep
  // kernel timing: event pairs per kernel class, reused across reads
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;
  // graph cache
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string graph_key;
};

namespace {

void free_tables(qed_tables* t) {
  if (!t) return;
  hipFree(t->h);
  hipFree(t->lnchi_min);
  hipFree(t->dlnchi);
  hipFree(t->P);
  hipFree(t->T);
  hipFree(t->fgrid);
  hipFree(t->Pf);
  hipFree(t->knorm);
  hipFree(t->g);
  hipFree(t->h32);
  hipFree(t->T32);
  hipFree(t->gP);
  hipFree(t->gPf);
  delete t;
}

qed_status check_table_params(const qed_table_params* p) {
  if (!p) return fail(QED_ERR_ARG, "table params is NULL");
  if (p->n_eta < 2 || p->n_eta > 1024) return fail(QED_ERR_ARG, "n_eta = %d outside [2, 1024]", p->n_eta);
  if (p->n_chi < 2 || p->n_chi > 1024) return fail(QED_ERR_ARG, "n_chi = %d outside [2, 1024]", p->n_chi);
  if (p->n_chi_pair < 2 || p->n_chi_pair > 1024)
    return fail(QED_ERR_ARG, "n_chi_pair = %d outside [2, 1024]", p->n_chi_pair);
  if (p->n_f < 3 || p->n_f > 1024) return fail(QED_ERR_ARG, "n_f = %d outside [3, 1024]", p->n_f);
  if (!finite_pos(p->eta_min) || !finite_pos(p->eta_max) || !(p->eta_max > p->eta_min))
    return fail(QED_ERR_ARG, "eta range [%g, %g] invalid", p->eta_min, p->eta_max);
  if (p->eta_min < 1e-8 || p->eta_max > 1e4)
    return fail(QED_ERR_ARG, "eta range [%g, %g] outside [1e-8, 1e4]", p->eta_min, p->eta_max);
  if (!finite_pos(p->chi_pair_min) || !finite_pos(p->chi_pair_max) || !(p->chi_pair_max > p->chi_pair_min))
    return fail(QED_ERR_ARG, "chi_pair range [%g, %g] invalid", p->chi_pair_min, p->chi_pair_max);
  if (p->chi_pair_min < 1e-3 || p->chi_pair_max > 1e5)
    return fail(QED_ERR_ARG, "chi_pair range [%g, %g] outside [1e-3, 1e5]", p->chi_pair_min, p->chi_pair_max);
  if (!(p->cutoff_energy_frac > 1e-15 && p->cutoff_energy_frac < 1e-2))
    return fail(QED_ERR_ARG, "cutoff_energy_frac = %g outside (1e-15, 1e-2)", p->cutoff_energy_frac);
  return QED_OK;
}

template <class T>
qed_status dalloc(T** p, size_t n) {
  HIP_TRY(hipMalloc((void**)p, n * sizeof(T)));
  return QED_OK;
}

qed_status alloc_tables(qed_tables* t) {
  const auto& p = t->p;
  qed_status st;
  if ((st = dalloc(&t->h, p.n_eta)) || (st = dalloc(&t->lnchi_min, p.n_eta)) || (st = dalloc(&t->dlnchi, p.n_eta)) ||
      (st = dalloc(&t->P, (size_t)p.n_eta * p.n_chi)) || (st = dalloc(&t->T, p.n_chi_pair)) ||
      (st = dalloc(&t->fgrid, p.n_f)) || (st = dalloc(&t->Pf, (size_t)p.n_chi_pair * p.n_f)) ||
      (st = dalloc(&t->knorm, p.n_chi_pair)) || (st = dalloc(&t->g, p.n_eta)) || (st = dalloc(&t->h32, p.n_eta)) ||
      (st = dalloc(&t->T32, p.n_chi_pair)) || (st = dalloc(&t->gP, (size_t)p.n_eta * (kGuide + 1))) ||
      (st = dalloc(&t->gPf, (size_t)p.n_chi_pair * (kGuide + 1))))
    return st;
  return QED_OK;
}

// host copies, FP32 copies of h and T, and sanity of the result
qed_status finish_tables(qed_tables* t, bool from_device) {
  const auto& p = t->p;
  if (from_device) {
    t->hh.resize(p.n_eta);
    t->hlnchi.resize(p.n_eta);
    t->hdlnchi.resize(p.n_eta);
    t->hP.resize((size_t)p.n_eta * p.n_chi);
    t->hT.resize(p.n_chi_pair);
    t->hf.resize(p.n_f);
    t->hPf.resize((size_t)p.n_chi_pair * p.n_f);
    t->hk.resize(p.n_chi_pair);
    t->hg.resize(p.n_eta);
    HIP_TRY(hipMemcpy(t->hh.data(), t->h, p.n_eta * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hg.data(), t->g, p.n_eta * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hlnchi.data(), t->lnchi_min, p.n_eta * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hdlnchi.data(), t->dlnchi, p.n_eta * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hP.data(), t->P, t->hP.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hT.data(), t->T, p.n_chi_pair * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hf.data(), t->fgrid, p.n_f * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hPf.data(), t->Pf, t->hPf.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t->hk.data(), t->knorm, p.n_chi_pair * 8, hipMemcpyDeviceToHost));
  }
  // every cumulative row must be finite, non-decreasing, in [0, 1] and end at 1
  for (int i = 0; i < p.n_eta; ++i) {
    if (!finite_pos(t->hh[i]) || !std::isfinite(t->hlnchi[i]) || !finite_pos(t->hdlnchi[i]))
      return fail(QED_ERR_STATE, "table row %d of h / chi grid is not finite", i);
    const double* P = &t->hP[(size_t)i * p.n_chi];
    for (int j = 0; j < p.n_chi; ++j)
      if (!(P[j] >= 0.0 && P[j] <= 1.0) || (j && P[j] < P[j - 1]))
        return fail(QED_ERR_STATE, "P_chi row %d is not a cumulative distribution at column %d", i, j);
    if (P[p.n_chi - 1] != 1.0) return fail(QED_ERR_STATE, "P_chi row %d does not end at 1", i);
    if (t->has_g && !(t->hg[i] > 0.0 && t->hg[i] <= 1.0 + 1e-12))
      return fail(QED_ERR_STATE, "g row %d = %g outside (0, 1]", i, t->hg[i]);
  }
  for (int k = 0; k < p.n_chi_pair; ++k) {
    if (!(t->hT[k] >= 0.0) || !std::isfinite(t->hT[k])) return fail(QED_ERR_STATE, "T row %d not finite", k);
    const double* P = &t->hPf[(size_t)k * p.n_f];
    for (int l = 0; l < p.n_f; ++l)
      if (!(P[l] >= 0.0 && P[l] <= 1.0) || (l && P[l] < P[l - 1]))
        return fail(QED_ERR_STATE, "P_f row %d is not a cumulative distribution at column %d", k, l);
    if (P[0] != 0.0 || P[p.n_f - 1] != 1.0) return fail(QED_ERR_STATE, "P_f row %d does not span [0, 1]", k);
  }
  // guide tables: for each row and u-bin g of width 1/kGuide, the largest column j <= n - 2 with
  // P[j] < g / kGuide (0 if none); the inversion of u in bin g then searches only between the
  // guides of bins g and g + 1 (an index structure over the rows, the same answer)
  auto guides = [](const std::vector<double>& P, int rows, int n, std::vector<uint16_t>& out) {
    out.assign((size_t)rows * (kGuide + 1), 0);
    for (int r = 0; r < rows; ++r) {
      const double* row = &P[(size_t)r * n];
      int j = 0;
      for (int g = 0; g <= kGuide; ++g) {
        const double v = (double)g / kGuide;
        while (j + 1 <= n - 2 && row[j + 1] < v) ++j;
        out[(size_t)r * (kGuide + 1) + g] = (uint16_t)j;
      }
    }
  };
  std::vector<uint16_t> gP, gPf;
  guides(t->hP, p.n_eta, p.n_chi, gP);
  guides(t->hPf, p.n_chi_pair, p.n_f, gPf);
  HIP_TRY(hipMemcpy(t->gP, gP.data(), gP.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t->gPf, gPf.data(), gPf.size() * 2, hipMemcpyHostToDevice));
  std::vector<float> h32(p.n_eta), T32(p.n_chi_pair);
  for (int i = 0; i < p.n_eta; ++i) h32[i] = (float)t->hh[i];
  for (int k = 0; k < p.n_chi_pair; ++k) T32[k] = (float)t->hT[k];
  HIP_TRY(hipMemcpy(t->h32, h32.data(), p.n_eta * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t->T32, T32.data(), p.n_chi_pair * 4, hipMemcpyHostToDevice));
  return QED_OK;
}

Tabs device_tabs(const qed_tables* t) {
  Tabs tb;
  const auto& p = t->p;
  tb.n_eta = p.n_eta;
  tb.le0 = std::log(p.eta_min);
  tb.dle = (std::log(p.eta_max) - tb.le0) / (p.n_eta - 1);
  tb.idle = 1.0 / tb.dle;
  tb.h = t->h;
  tb.h32 = t->h32;
  tb.g = t->has_g ? t->g : nullptr;
  tb.n_chi = p.n_chi;
  tb.lnchi_min = t->lnchi_min;
  tb.dlnchi = t->dlnchi;
  tb.P = t->P;
  tb.gP = t->gP;
  tb.n_cp = p.n_chi_pair;
  tb.lc0 = std::log(p.chi_pair_min);
  tb.cp_min = p.chi_pair_min;
  tb.dlc = (std::log(p.chi_pair_max) - tb.lc0) / (p.n_chi_pair - 1);
  tb.idlc = 1.0 / tb.dlc;
  tb.T = t->T;
  tb.T32 = t->T32;
  tb.n_f = p.n_f;
  tb.f = t->fgrid;
  tb.Pf = t->Pf;
  tb.gPf = t->gPf;
  return tb;
}

qed_status check_params(const qed_workspace* ws, const qed_step_params* p) {
  if (!p) return fail(QED_ERR_ARG, "step params is NULL");
  if (!finite_pos(p->dt)) return fail(QED_ERR_ARG, "dt = %g must be finite and positive", p->dt);
  if (!std::isfinite(p->t0)) return fail(QED_ERR_ARG, "t0 = %g must be finite", p->t0);
  if (!finite_pos(p->lambda_L)) return fail(QED_ERR_ARG, "lambda_L = %g must be finite and positive", p->lambda_L);
  if (p->flags & ~31u) return fail(QED_ERR_ARG, "unknown flag bits 0x%x", p->flags);
  if ((p->flags & (QED_RR_QUANTUM | QED_RR_CLASSICAL)) == (QED_RR_QUANTUM | QED_RR_CLASSICAL))
    return fail(QED_ERR_ARG, "QED_RR_QUANTUM and QED_RR_CLASSICAL exclude each other");
  if ((p->flags & (QED_RR_QUANTUM | QED_RR_CLASSICAL)) && (p->flags & QED_EMIT))
    return fail(QED_ERR_ARG, "deterministic radiation reaction replaces emission: drop QED_EMIT");
  if ((p->flags & QED_PAIRS) && !(p->flags & QED_PROPAGATE))
    return fail(QED_ERR_ARG, "QED_PAIRS needs QED_PROPAGATE (pairs come from stepped photons)");
  if (p->precision != QED_FP64 && p->precision != QED_FP32_MIXED)
    return fail(QED_ERR_ARG, "unknown precision %d", (int)p->precision);
  if (ws && ws->bound && p->precision != ws->prec)
    return fail(QED_ERR_STATE, "precision differs from the one the instances were bound with");
  return QED_OK;
}

StepConst step_const(const qed_step_params* p) {
  StepConst sc;
  sc.t0 = p->t0;
  sc.dt = p->dt;
  sc.kappa = p->lambda_L / kLambdaCompton;
  sc.a_gamma = std::sqrt(3.0) * kAlpha * sc.kappa / (2.0 * kPi);
  sc.a_pair = kAlpha * sc.kappa;
  sc.a_rr = 2.0 / 3.0 * kAlpha * sc.kappa;
  sc.flags = p->flags;
  return sc;
}

hipEvent_t next_event(qed_workspace* ws) {
  if (ws->ev_used == ws->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ws->ev_pool.push_back(e);
  }
  return ws->ev_pool[ws->ev_used++];
}

// records a start event for kernel class `k`; returns the slot to close with mark_end
int mark_begin(qed_workspace* ws, int k, hipStream_t s) {
  if (!ws->profiling) return -1;
  hipEvent_t a = next_event(ws), b = next_event(ws);
  if (!a || !b) return -1;
  hipEventRecord(a, s);
  ws->ev_marks.push_back({k, {a, b}});
  return (int)ws->ev_marks.size() - 1;
}

void mark_end(qed_workspace* ws, int slot, hipStream_t s) {
  if (slot >= 0) hipEventRecord(ws->ev_marks[slot].second.second, s);
}

// Persistent grid of sweep `w` (0 lepton, 1 photon): one resident round of blocks.  The chunk
// deal gives every block the same share, so blocks beyond what fits at once would only form a
// second round that starts late.  At most 2048 threads per CU (the emission queue's bound).
int sweep_grid(qed_workspace* ws, int w, int n_tab) {
  const bool mixed = ws->prec == QED_FP32_MIXED;
  const int key[5] = {ws->field_kind, ws->ppt[w], ws->block[w], (int)mixed, n_tab};
  if (std::memcmp(key, ws->fit_key[w], sizeof(key)) != 0) {
    ws->fit[w] = w ? photon_blocks_per_cu(ws->field_kind, ws->ppt[1], ws->block[1], n_tab, mixed)
                   : lepton_blocks_per_cu(ws->field_kind, ws->ppt[0], ws->block[0], n_tab, mixed);
    std::memcpy(ws->fit_key[w], key, sizeof(key));
  }
  return ws->cus * std::max(1, std::min(ws->fit[w], 2048 / ws->block[w]));
}

// Grid of the emission pass: as many blocks as fit the CUs at once (at most 4 per CU), so that a
// step with many events keeps many of their latency chains in flight; the events are dealt to
// the blocks in equal contiguous shares.
int emit_grid(qed_workspace* ws, int lepton_waves) {
  const bool mixed = ws->prec == QED_FP32_MIXED;
  const int key[3] = {ws->field_kind, (int)mixed, lepton_waves};
  if (std::memcmp(key, ws->emit_fit_key, sizeof(key)) != 0) {
    ws->emit_fit = emit_blocks_per_cu(ws->field_kind, lepton_waves, mixed);
    std::memcpy(ws->emit_fit_key, key, sizeof(key));
  }
  return ws->cus * std::max(1, std::min(ws->emit_fit, 4));
}

qed_status enqueue_step(const qed_tables* tb, qed_workspace* ws, const qed_step_params* p, hipStream_t s) {
  const int BL = ws->block[0], BP = ws->block[1];
  const StepConst sc = step_const(p);
  int m = mark_begin(ws, 0, s);
  launch_step_begin(ws->d_inst, ws->n_inst, ws->d_acc, ws->d_glob, ws->d_evc, ws->d_evc + 1, ws->d_base,
                    ws->d_base + 2 * ws->max_inst, BL * ws->ppt[0], BP * ws->ppt[1], 1,
                    (p->flags & QED_PAIRS) ? 1 : 0, s);
  if (ws->any_grid) launch_grid_refresh(ws->d_inst, ws->n_inst, ws->d_glob, sc, s);
  mark_end(ws, m, s);
  StepArgs a;
  a.inst = ws->d_inst;
  a.acc = ws->d_acc;
  a.glob = ws->d_glob;
  a.tb = device_tabs(tb);
  a.sc = sc;
  a.q.ctl = ws->d_evc;
  a.q.ent = ws->d_evq;
  a.q.cap = ws->evq_cap;
  a.qe.ctl = ws->d_evc + 1;
  a.qe.ent = ws->d_emq;
  a.qe.cap = ws->emq_cap;
  a.qe.wave_cnt = ws->d_wave_cnt;
  a.qe.grid = sweep_grid(ws, 0, a.tb.n_eta);
  a.qe.waves = BL / 64;
  a.qe.ppt = ws->ppt[0];
  a.win = ws->d_win;
  a.rec = ws->d_rec;
  a.lmask = ws->d_lmask;
  // persistent grids (sweep_grid), blocks taking runs of the chunk list.
  // The passes run in order on `stream`: the photon sweep alone saturates HBM, so running the
  // lepton passes beside it on a second stream (their data are disjoint) shares bandwidth
  // rather than adding any.
  const bool mixed = ws->prec == QED_FP32_MIXED;
  hipStream_t sl = s;
  a.base = ws->d_base;
  a.n_base = 2 * ws->n_inst;
  a.ppt = ws->ppt[0];
  m = mark_begin(ws, 1, sl);
  launch_lepton(ws->field_kind, a, a.qe.grid, BL, mixed, sl);
  mark_end(ws, m, sl);
  if (p->flags & QED_EMIT) {
    m = mark_begin(ws, 4, sl);
    launch_emit_events(ws->field_kind, a, emit_grid(ws, a.qe.grid * a.qe.waves), 256, mixed, sl);
    mark_end(ws, m, sl);
  }
  if (p->flags & QED_PAIRS) {
    // photons only change state through the pair optical depth: without pair creation their
    // position is the closed form of their birth record and no pass runs
    a.base = ws->d_base + 2 * ws->max_inst;
    a.n_base = ws->n_inst;
    a.ppt = ws->ppt[1];
    m = mark_begin(ws, 2, s);
    launch_photon(ws->field_kind, a, sweep_grid(ws, 1, a.tb.n_cp), BP, mixed, s);
    mark_end(ws, m, s);
    m = mark_begin(ws, 3, s);
    launch_pair_events(ws->field_kind, a, ws->cus, 256, mixed, s);
    mark_end(ws, m, s);
  }
  if (ws->fdtd_work) {  // field feedback: the grid advances with the current the step deposited
    m = mark_begin(ws, 5, s);
    launch_fdtd(ws->d_inst, ws->n_inst, (int)std::min<int64_t>(ws->fdtd_work, 1 << 30), p->dt, s);
    mark_end(ws, m, s);
  }
  HIP_TRY(hipGetLastError());
  return QED_OK;
}

// (Re)computes the photons' pair windows when the step constants or tables differ from those
// they were made with.  Enqueued on `s` outside any graph capture.
qed_status ensure_windows(const qed_tables* tb, qed_workspace* ws, const qed_step_params* p, hipStream_t s) {
  const double cp_min = device_tabs(tb).cp_min;
  if (ws->win_valid && ws->win_t0 == p->t0 && ws->win_dt == p->dt && ws->win_cp_min == cp_min) return QED_OK;
  launch_photon_windows(ws->field_kind, ws->d_inst, ws->n_inst, ws->d_acc, ws->d_glob, ws->d_win, ws->d_rec, ws->d_lmask,
                        p->t0, p->dt, cp_min,
                        ws->prec == QED_FP32_MIXED, s);
  HIP_TRY(hipGetLastError());
  ws->win_valid = true;
  ws->win_t0 = p->t0;
  ws->win_dt = p->dt;
  ws->win_cp_min = cp_min;
  return QED_OK;
}

static bool grid_kind(int kind) { return kind == QED_FIELD_GRID_CP_STANDING || kind == QED_FIELD_GRID_FDTD; }

// The emission queue holds every wave segment of the lepton sweep (EmitQueue): the bound lepton
// slots plus the rounding of the chunk list (a partial chunk per species list) and of the blocks'
// runs of chunks (up to one chunk per block).  Synchronises the device when it reallocates.
qed_status ensure_emit_queue(qed_workspace* ws) {
  const int64_t ch = (int64_t)ws->block[0] * ws->ppt[0];
  const int64_t grid = (int64_t)ws->cus * (2048 / ws->block[0]);  // bound of sweep_grid
  const int64_t need = std::max<int64_t>(1, ws->lep_cap + (2 * (int64_t)ws->n_inst + grid) * ch);
  if (need <= ws->emq_cap && ws->d_emq) return QED_OK;
  HIP_TRY(hipDeviceSynchronize());
  hipFree(ws->d_emq);
  ws->d_emq = nullptr;
  ws->emq_cap = 0;
  HIP_TRY(hipMalloc((void**)&ws->d_emq, (size_t)need * sizeof(EmitEv)));
  ws->emq_cap = need;
  return QED_OK;
}

void drop_graph(qed_workspace* ws) {
  if (ws->exec) hipGraphExecDestroy(ws->exec);
  if (ws->graph) hipGraphDestroy(ws->graph);
  ws->exec = nullptr;
  ws->graph = nullptr;
  ws->graph_key.clear();
}

qed_status run_ledger(qed_workspace* ws, std::vector<InstAcc>& acc, hipStream_t s) {
  launch_ledger(ws->d_inst, ws->n_inst, ws->d_acc, ws->prec == QED_FP32_MIXED, s);
  HIP_TRY(hipGetLastError());
  acc.resize(ws->n_inst);
  HIP_TRY(hipMemcpyAsync(acc.data(), ws->d_acc, ws->n_inst * sizeof(InstAcc), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return QED_OK;
}

}  // namespace

extern "C" {

const char* qed_last_error(void) { return g_err.c_str(); }

const char* qed_version(void) { return "libqed 1.0 (gfx950, Philox4x64-10, FP64 and FP32-mixed)"; }

qed_status qed_build_tables(const qed_table_params* params, qed_tables** out) {
  if (!out) return fail(QED_ERR_ARG, "out is NULL");
  *out = nullptr;
  qed_status st = check_table_params(params);
  if (st) return st;
  int dev;
  if ((st = check_device(&dev, nullptr))) return st;
  qed_tables* t = new qed_tables();
  t->p = *params;
  t->device = dev;
  if ((st = alloc_tables(t))) {
    free_tables(t);
    return st;
  }
  t->has_g = true;
  hipError_t e = launch_build_tables(t->p, t->h, t->lnchi_min, t->dlnchi, t->P, t->T, t->fgrid, t->Pf, t->knorm,
                                     t->g, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_tables(t);
    return fail(QED_ERR_HIP, "table build: %s", hipGetErrorString(e));
  }
  if ((st = finish_tables(t, true))) {
    free_tables(t);
    return st;
  }
  *out = t;
  return QED_OK;
}

qed_status qed_tables_from_host(const qed_table_params* params, const double* h, const double* lnchi_min,
                                const double* dlnchi, const double* P_chi, const double* T, const double* f_grid,
                                const double* P_f, const double* k_norm, const double* g, qed_tables** out) {
  if (!out) return fail(QED_ERR_ARG, "out is NULL");
  *out = nullptr;
  qed_status st = check_table_params(params);
  if (st) return st;
  if (!h || !lnchi_min || !dlnchi || !P_chi || !T || !f_grid || !P_f) return fail(QED_ERR_ARG, "a table array is NULL");
  int dev;
  if ((st = check_device(&dev, nullptr))) return st;
  qed_tables* t = new qed_tables();
  t->p = *params;
  t->device = dev;
  const auto& p = t->p;
  t->hh.assign(h, h + p.n_eta);
  t->hlnchi.assign(lnchi_min, lnchi_min + p.n_eta);
  t->hdlnchi.assign(dlnchi, dlnchi + p.n_eta);
  t->hP.assign(P_chi, P_chi + (size_t)p.n_eta * p.n_chi);
  t->hT.assign(T, T + p.n_chi_pair);
  t->hf.assign(f_grid, f_grid + p.n_f);
  t->hPf.assign(P_f, P_f + (size_t)p.n_chi_pair * p.n_f);
  if (k_norm) t->hk.assign(k_norm, k_norm + p.n_chi_pair);
  else t->hk.assign(p.n_chi_pair, 0.0);
  t->has_g = g != nullptr;
  if (g) t->hg.assign(g, g + p.n_eta);
  else t->hg.assign(p.n_eta, 0.0);
  auto up = [&](double* d, const std::vector<double>& v) {
    return hipMemcpy(d, v.data(), v.size() * 8, hipMemcpyHostToDevice);
  };
  if ((st = alloc_tables(t))) {
    free_tables(t);
    return st;
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(t->h, t->hh);
  if (e == hipSuccess) e = up(t->lnchi_min, t->hlnchi);
  if (e == hipSuccess) e = up(t->dlnchi, t->hdlnchi);
  if (e == hipSuccess) e = up(t->P, t->hP);
  if (e == hipSuccess) e = up(t->T, t->hT);
  if (e == hipSuccess) e = up(t->fgrid, t->hf);
  if (e == hipSuccess) e = up(t->Pf, t->hPf);
  if (e == hipSuccess) e = up(t->knorm, t->hk);
  if (e == hipSuccess) e = up(t->g, t->hg);
  if (e != hipSuccess) {
    free_tables(t);
    return fail(QED_ERR_HIP, "table upload: %s", hipGetErrorString(e));
  }
  if ((st = finish_tables(t, false))) {
    free_tables(t);
    return st;
  }
  *out = t;
  return QED_OK;
}

qed_status qed_tables_view(const qed_tables* t, qed_table_view* out) {
  if (!t || !out) return fail(QED_ERR_ARG, "NULL argument");
  out->params = t->p;
  out->h = t->hh.data();
  out->lnchi_min = t->hlnchi.data();
  out->dlnchi = t->hdlnchi.data();
  out->P_chi = t->hP.data();
  out->T = t->hT.data();
  out->f_grid = t->hf.data();
  out->P_f = t->hPf.data();
  out->k_norm = t->hk.data();
  out->g = t->has_g ? t->hg.data() : nullptr;
  return QED_OK;
}

void qed_tables_destroy(qed_tables* t) { free_tables(t); }

qed_status qed_workspace_create(int32_t max_inst, qed_workspace** out) {
  if (!out) return fail(QED_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (max_inst < 1 || max_inst > 65535 / 3) return fail(QED_ERR_ARG, "max_inst = %d outside [1, 21845]", max_inst);
  int dev, cus;
  qed_status st = check_device(&dev, &cus);
  if (st) return st;
  qed_workspace* ws = new qed_workspace();
  ws->device = dev;
  ws->cus = cus;
  ws->max_inst = max_inst;
  hipError_t e = hipMalloc((void**)&ws->d_inst, max_inst * sizeof(qed_instance));
  if (e == hipSuccess) e = hipMalloc((void**)&ws->d_acc, max_inst * sizeof(InstAcc));
  if (e == hipSuccess) e = hipMalloc((void**)&ws->d_glob, sizeof(Glob));
  if (e == hipSuccess) e = hipMalloc((void**)&ws->d_evc, 2 * sizeof(EvCtl));
  if (e == hipSuccess) e = hipMemset(ws->d_evc, 0, 2 * sizeof(EvCtl));
  if (e == hipSuccess) e = hipMalloc((void**)&ws->d_evq, (size_t)kDefaultEventQueue * sizeof(uint64_t));
  if (e == hipSuccess) ws->evq_cap = kDefaultEventQueue;
  if (e == hipSuccess) e = hipMalloc((void**)&ws->d_base, 3 * (size_t)max_inst * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc((void**)&ws->d_wave_cnt, (size_t)cus * 32 * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(ws->d_wave_cnt, 0, (size_t)cus * 32 * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(ws->d_glob, 0, sizeof(Glob));
  if (e == hipSuccess) e = hipMemset(ws->d_acc, 0, max_inst * sizeof(InstAcc));
  if (e == hipSuccess) e = init_crmath();
  if (e != hipSuccess) {
    qed_workspace_destroy(ws);
    return fail(QED_ERR_HIP, "workspace allocation: %s", hipGetErrorString(e));
  }
  *out = ws;
  return QED_OK;
}

void qed_workspace_destroy(qed_workspace* ws) {
  if (!ws) return;
  drop_graph(ws);
  for (hipEvent_t e : ws->ev_pool) hipEventDestroy(e);
  hipFree(ws->d_inst);
  hipFree(ws->d_acc);
  hipFree(ws->d_glob);
  hipFree(ws->d_evc);
  hipFree(ws->d_evq);
  hipFree(ws->d_emq);
  hipFree(ws->d_wave_cnt);
  hipFree(ws->retire.spec);
  hipFree(ws->sort.key);
  hipFree(ws->sort.dst);
  hipFree(ws->sort.hist);
  hipFree(ws->sort.stage);
  hipFree(ws->d_base);
  hipFree(ws->d_movers);
  hipFree(ws->d_win);
  hipFree(ws->d_rec);
  hipFree(ws->d_lmask);
  delete ws;
}

qed_status qed_set_kernel_launch(qed_workspace* ws, int32_t kernel, int32_t block, int32_t ppt) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  if (kernel != QED_KERNEL_LEPTON && kernel != QED_KERNEL_PHOTON)
    return fail(QED_ERR_ARG, "kernel = %d: need QED_KERNEL_LEPTON or QED_KERNEL_PHOTON", kernel);
  if (block < 64 || block > 256 || block % 64) return fail(QED_ERR_ARG, "block = %d: need 64..256, multiple of 64", block);
  if (ppt != 1 && ppt != 2 && ppt != 4 && ppt != 8 && !(ppt == 16 && kernel == QED_KERNEL_PHOTON))
    return fail(QED_ERR_ARG, "ppt = %d: need 1, 2, 4 or 8 (or 16 for the photon sweep)", ppt);
  const int k = kernel == QED_KERNEL_LEPTON ? 0 : 1;
  if (ws->block[k] != block || ws->ppt[k] != ppt) drop_graph(ws);
  ws->block[k] = block;
  ws->ppt[k] = ppt;
  if (k == 0 && ws->bound) return ensure_emit_queue(ws);
  return QED_OK;
}

qed_status qed_set_launch(qed_workspace* ws, int32_t block, int32_t ppt) {
  qed_status st = qed_set_kernel_launch(ws, QED_KERNEL_LEPTON, block, ppt);
  return st ? st : qed_set_kernel_launch(ws, QED_KERNEL_PHOTON, block, ppt);
}

qed_status qed_bind(qed_workspace* ws, const qed_instance* inst, int32_t n_inst, const qed_step_params* params) {
  if (!ws || !inst) return fail(QED_ERR_ARG, "NULL argument");
  if (n_inst < 1 || n_inst > ws->max_inst) return fail(QED_ERR_ARG, "n_inst = %d outside [1, %d]", n_inst, ws->max_inst);
  ws->bound = false;
  qed_status st = check_params(nullptr, params);
  if (st) return st;
  const bool mixed = params->precision == QED_FP32_MIXED;
  const size_t fe = mixed ? 4 : 8;
  int cur;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != ws->device) return fail(QED_ERR_STATE, "workspace belongs to device %d, current is %d", ws->device, cur);
  size_t movers = 0;
  for (int i = 0; i < n_inst; ++i) {
    const qed_instance& I = inst[i];
    if (I.dims != 2 && I.dims != 3) return fail(QED_ERR_ARG, "instance %d: dims = %d (2 or 3)", i, I.dims);
    if (!finite_pos(I.weight)) return fail(QED_ERR_ARG, "instance %d: weight must be finite and positive", i);
    const qed_field& F = I.field;
    if (F.kind < QED_FIELD_UNIFORM || F.kind > QED_FIELD_GRID_FDTD)
      return fail(QED_ERR_ARG, "instance %d: unknown field kind %d", i, F.kind);
    if (F.kind != inst[0].field.kind)
      return fail(QED_ERR_ARG, "instance %d: all bound instances must share one field kind", i);
    for (int k = 0; k < 16; ++k)
      if (!std::isfinite(F.p[k])) return fail(QED_ERR_ARG, "instance %d: field parameter %d not finite", i, k);
    if (F.kind == QED_FIELD_LP_PULSE && !finite_pos(F.p[1]))
      return fail(QED_ERR_ARG, "instance %d: pulse length must be positive", i);
    if (grid_kind(F.kind)) {
      if (F.nx < 2 || F.ny < 2 || !finite_pos(F.dx) || !finite_pos(F.dy) || !std::isfinite(F.x0) || !std::isfinite(F.y0))
        return fail(QED_ERR_ARG, "instance %d: grid shape invalid", i);
      if ((int64_t)F.nx * F.ny > ((int64_t)1 << 31)) return fail(QED_ERR_ARG, "instance %d: grid above 2^31 nodes", i);
    }
    if (F.kind == QED_FIELD_GRID_CP_STANDING &&
        (st = check_dev_range(F.grid_dev, (size_t)6 * F.nx * F.ny * 4, "grid_dev", i, -1)))
      return st;
    if (F.kind == QED_FIELD_GRID_FDTD) {
      // the deposit assumes moves below a cell per step, which the solver's Courant condition
      // (dt < 1/sqrt(1/dx^2 + 1/dy^2)) implies for particles slower than light
      if (mixed || I.dims != 2) return fail(QED_ERR_ARG, "instance %d: the field-feedback kind runs in FP64, 2-D", i);
      if (!(params->dt * std::sqrt(1.0 / (F.dx * F.dx) + 1.0 / (F.dy * F.dy)) < 1.0))
        return fail(QED_ERR_ARG, "instance %d: dt above the Yee Courant limit of the grid", i);
      if ((st = check_dev_range(F.fdtd_dev, (size_t)9 * F.nx * F.ny * 8, "fdtd_dev", i, -1))) return st;
    }
    for (int s = 0; s < 3; ++s) {
      const qed_species& S = I.s[s];
      if (S.capacity < 0 || S.capacity > ((int64_t)1 << 40)) return fail(QED_ERR_ARG, "instance %d species %d: capacity", i, s);
      if ((st = check_dev_range(S.count_dev, 8, "count_dev", i, s))) return st;
      if (S.capacity == 0) continue;
      const size_t n = (size_t)S.capacity;
      if ((st = check_dev_range(S.x_dev, n * fe, "x_dev", i, s)) || (st = check_dev_range(S.y_dev, n * fe, "y_dev", i, s)) ||
          (st = check_dev_range(S.ux_dev, n * fe, "ux_dev", i, s)) ||
          (st = check_dev_range(S.uy_dev, n * fe, "uy_dev", i, s)) ||
          (st = check_dev_range(S.uz_dev, n * fe, "uz_dev", i, s)) ||
          (st = check_dev_range(S.tau_dev, n * 8, "tau_dev", i, s)) ||
          (st = check_dev_range(S.uid_dev, n * 8, "uid_dev", i, s)))
        return st;
      if (I.dims == 3 && (st = check_dev_range(S.z_dev, n * fe, "z_dev", i, s))) return st;
      if (s == 2 && (st = check_dev_range(S.birth_step_dev, n * 4, "birth_step_dev", i, s))) return st;
      if (mixed && s < 2) {
        if ((st = check_dev_range(S.x_lo_dev, n * 4, "x_lo_dev", i, s)) ||
            (st = check_dev_range(S.y_lo_dev, n * 4, "y_lo_dev", i, s)) ||
            (st = check_dev_range(S.ux_lo_dev, n * 4, "ux_lo_dev", i, s)) ||
            (st = check_dev_range(S.uy_lo_dev, n * 4, "uy_lo_dev", i, s)) ||
            (st = check_dev_range(S.uz_lo_dev, n * 4, "uz_lo_dev", i, s)))
          return st;
        if (I.dims == 3 && (st = check_dev_range(S.z_lo_dev, n * 4, "z_lo_dev", i, s))) return st;
      }
    }
    movers += (size_t)I.s[2].capacity;
  }
  // every child needs a slot in its species: emission needs photons, pairs need both leptons
  drop_graph(ws);
  ws->inst.assign(inst, inst + n_inst);
  ws->n_inst = n_inst;
  ws->prec = params->precision;
  ws->field_kind = inst[0].field.kind;
  ws->any_grid = inst[0].field.kind == QED_FIELD_GRID_CP_STANDING;
  ws->fdtd_work = 0;
  for (int i = 0; i < n_inst; ++i)
    if (inst[i].field.kind == QED_FIELD_GRID_FDTD)
      ws->fdtd_work = std::max<int64_t>(ws->fdtd_work, (int64_t)inst[i].field.ny * ((inst[i].field.nx + 255) / 256));
  // compaction scratch: one mover index per photon slot
  std::vector<InstAcc> acc0(n_inst);
  std::memset(acc0.data(), 0, n_inst * sizeof(InstAcc));
  size_t off = 0, goff = 0;
  for (int i = 0; i < n_inst; ++i) {
    acc0[i].n_pair_compacted = ~0ull;  // the first compaction after a bind always runs
    acc0[i].mover_off = (int64_t)off;
    acc0[i].lmask_off = (int64_t)goff;  // the masks are made with the windows
    off += (size_t)inst[i].s[2].capacity;
    goff += ((size_t)inst[i].s[2].capacity + kWinGroup - 1) / kWinGroup;
  }
  if (goff > ws->lmask_len || !ws->d_lmask) {
    hipFree(ws->d_lmask);
    ws->d_lmask = nullptr;
    ws->lmask_len = 0;
    HIP_TRY(hipMalloc((void**)&ws->d_lmask, (goff ? goff : 1) * sizeof(uint64_t)));
    ws->lmask_len = goff ? goff : 1;
  }
  // no bit for a slot no photon has held yet (the window build sets those of the bound photons)
  HIP_TRY(hipMemset(ws->d_lmask, 0, ws->lmask_len * sizeof(uint64_t)));
  if (movers > ws->movers_len) {
    hipFree(ws->d_movers);
    ws->d_movers = nullptr;
    ws->movers_len = 0;
    HIP_TRY(hipMalloc((void**)&ws->d_movers, (movers ? movers : 1) * sizeof(int64_t)));
    ws->movers_len = movers;
  }
  const int rec_bytes = photon_rec_bytes(params->precision == QED_FP32_MIXED, inst[0].field.kind);
  if (movers > ws->win_len || !ws->d_win || rec_bytes > ws->rec_bytes) {
    hipFree(ws->d_win);
    hipFree(ws->d_rec);
    ws->d_win = nullptr;
    ws->d_rec = nullptr;
    ws->win_len = 0;
    ws->rec_bytes = 0;
    HIP_TRY(hipMalloc((void**)&ws->d_win, (movers ? movers : 1) * sizeof(uint32_t)));
    HIP_TRY(hipMalloc((void**)&ws->d_rec, (movers ? movers : 1) * (size_t)rec_bytes));
    ws->win_len = movers ? movers : 1;
    ws->rec_bytes = rec_bytes;
  }
  ws->win_valid = false;  // computed by the first step, which knows t0, dt and the tables
  if (ws->retire.spec) HIP_TRY(hipMemset(ws->retire.spec, 0, ws->spec_len * sizeof(unsigned long long)));
  // emission queue: the wave segments of the lepton sweep (a lepton emits at most once per step)
  int64_t leptons = 0;
  for (int i = 0; i < n_inst; ++i) leptons += inst[i].s[0].capacity + inst[i].s[1].capacity;
  ws->lep_cap = leptons;
  if ((st = ensure_emit_queue(ws))) return st;
  HIP_TRY(hipMemcpy(ws->d_inst, inst, n_inst * sizeof(qed_instance), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws->d_acc, acc0.data(), n_inst * sizeof(InstAcc), hipMemcpyHostToDevice));
  std::vector<InstAcc> acc;
  if ((st = run_ledger(ws, acc, nullptr))) return st;
  ws->e0.resize(n_inst);
  for (int i = 0; i < n_inst; ++i)
    ws->e0[i] = (fix_value(acc[i].fx[FX_ENERGY]) + fix_value(acc[i].fx[FX_ENERGY + 1]) +
                 fix_value(acc[i].fx[FX_ENERGY + 2])) * inst[i].weight;
  ws->bound = true;
  return QED_OK;
}

qed_status qed_init_optical_depth(qed_workspace* ws, qed_stream stream) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  launch_init_tau(ws->d_inst, ws->n_inst, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return QED_OK;
}

qed_status qed_set_step(qed_workspace* ws, int64_t step, qed_stream stream) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  if (step < 0 || step > ((int64_t)1 << 31)) return fail(QED_ERR_ARG, "step = %lld outside [0, 2^31]", (long long)step);
  launch_set_step(ws->d_inst, ws->n_inst, ws->d_acc, ws->d_glob, ws->d_win, ws->d_lmask, step, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return QED_OK;
}

qed_status qed_step(const qed_tables* tables, qed_workspace* ws, const qed_step_params* params, qed_stream stream) {
  if (!tables || !ws) return fail(QED_ERR_ARG, "NULL argument");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  if (tables->device != ws->device) return fail(QED_ERR_STATE, "tables and workspace are on different devices");
  qed_status st = check_params(ws, params);
  if (st) return st;
  if ((params->flags & QED_RR_QUANTUM) && !tables->has_g)
    return fail(QED_ERR_STATE, "QED_RR_QUANTUM needs tables with g (built, or supplied with g)");
  if ((st = ensure_windows(tables, ws, params, (hipStream_t)stream))) return st;
  return enqueue_step(tables, ws, params, (hipStream_t)stream);
}

qed_status qed_run(const qed_tables* tables, qed_workspace* ws, const qed_step_params* params, int64_t n_steps,
                   int32_t graph_steps, qed_stream stream) {
  if (!tables || !ws) return fail(QED_ERR_ARG, "NULL argument");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  if (tables->device != ws->device) return fail(QED_ERR_STATE, "tables and workspace are on different devices");
  qed_status st = check_params(ws, params);
  if (st) return st;
  if ((params->flags & QED_RR_QUANTUM) && !tables->has_g)
    return fail(QED_ERR_STATE, "QED_RR_QUANTUM needs tables with g (built, or supplied with g)");
  if (n_steps < 0) return fail(QED_ERR_ARG, "n_steps < 0");
  if (graph_steps < 0 || graph_steps > 100000) return fail(QED_ERR_ARG, "graph_steps = %d outside [0, 1e5]", graph_steps);
  hipStream_t s = (hipStream_t)stream;
  if (graph_steps > 0 && s == nullptr) return fail(QED_ERR_ARG, "graph replay needs a non-null stream");
  if (graph_steps > 0 && ws->profiling) return fail(QED_ERR_STATE, "kernel timing is on; graph replay cannot record it");
  if ((st = ensure_windows(tables, ws, params, s))) return st;
  int64_t done = 0;
  if (graph_steps > 0 && n_steps >= graph_steps) {
    char key[256];
    snprintf(key, sizeof(key), "%p|%a|%a|%a|%u|%d|%d|%d|%d", (const void*)tables, params->t0, params->dt,
             params->lambda_L, params->flags, (int)params->precision, ws->block[0] * 16 + ws->ppt[0],
             ws->block[1] * 16 + ws->ppt[1], graph_steps);
    if (ws->graph_key != key) {
      drop_graph(ws);
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int g = 0; g < graph_steps; ++g) {
        st = enqueue_step(tables, ws, params, s);
        if (st) {
          hipGraph_t junk = nullptr;
          hipStreamEndCapture(s, &junk);
          if (junk) hipGraphDestroy(junk);
          return st;
        }
      }
      HIP_TRY(hipStreamEndCapture(s, &ws->graph));
      HIP_TRY(hipGraphInstantiate(&ws->exec, ws->graph, nullptr, nullptr, 0));
      ws->graph_key = key;
    }
    for (; done + graph_steps <= n_steps; done += graph_steps) HIP_TRY(hipGraphLaunch(ws->exec, s));
  }
  for (; done < n_steps; ++done)
    if ((st = enqueue_step(tables, ws, params, s))) return st;
  return QED_OK;
}

qed_status qed_profile(qed_workspace* ws, int32_t enable) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  ws->profiling = enable != 0;
  ws->ev_marks.clear();
  ws->ev_used = 0;
  return QED_OK;
}

qed_status qed_sort(qed_workspace* ws, const qed_step_params* params, qed_stream stream) {
  if (!ws || !params) return fail(QED_ERR_ARG, "NULL argument");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  if (!(params->dt > 0.0) || !std::isfinite(params->dt)) return fail(QED_ERR_ARG, "dt must be positive");
  int64_t cap = 0;
  int tiles = 0;
  for (const qed_instance& I : ws->inst) {
    if (!grid_kind(I.field.kind)) continue;
    for (int s = 0; s < 3; ++s) cap = std::max<int64_t>(cap, I.s[s].capacity);
    tiles = std::max(tiles, ((I.field.nx + 7) / 8) * ((I.field.ny + 7) / 8));
  }
  if (cap == 0) return QED_OK;  // no grid instance: nothing to reorder
  if (cap >= (int64_t(1) << 32)) return fail(QED_ERR_ARG, "qed_sort handles up to 2^32 - 1 slots per species");
  HIP_TRY(hipSetDevice(ws->device));
  if (cap > ws->sort_cap || tiles > ws->sort.hist_len) {
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    hipFree(ws->sort.key);
    hipFree(ws->sort.dst);
    hipFree(ws->sort.hist);
    hipFree(ws->sort.stage);
    ws->sort = SortScratch();
    ws->sort_cap = 0;
    HIP_TRY(hipMalloc((void**)&ws->sort.key, (size_t)cap * sizeof(int32_t)));
    HIP_TRY(hipMalloc((void**)&ws->sort.dst, (size_t)cap * sizeof(uint32_t)));
    HIP_TRY(hipMalloc((void**)&ws->sort.hist, (size_t)tiles * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&ws->sort.stage, (size_t)cap * 8));
    ws->sort.hist_len = tiles;
    ws->sort_cap = cap;
  }
  const bool mixed = ws->prec == QED_FP32_MIXED;
  for (int ii = 0; ii < ws->n_inst; ++ii) {
    const qed_instance& I = ws->inst[ii];
    if (!grid_kind(I.field.kind)) continue;
    for (int s = 0; s < 3; ++s) {
      if (I.s[s].capacity == 0) continue;
      HIP_TRY(launch_sort_species(ws->d_inst, I, ii, s, ws->d_glob, params->dt, mixed, ws->sort, ws->cus * 8,
                                  (hipStream_t)stream));
    }
  }
  launch_front_clear(ws->d_acc, ws->n_inst, (hipStream_t)stream);  // the photons moved: no front
  HIP_TRY(hipGetLastError());
  ws->win_valid = false;  // the photons moved: their windows and records are set again by the next step
  return QED_OK;
}

qed_status qed_sort_static(qed_workspace* ws, const qed_step_params* params, qed_stream stream) {
  if (!ws || !params) return fail(QED_ERR_ARG, "NULL argument");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  if (!(params->dt > 0.0) || !std::isfinite(params->dt)) return fail(QED_ERR_ARG, "dt must be positive");
  int64_t cap = 0;
  int tiles = 0;
  for (const qed_instance& I : ws->inst) {
    if (!grid_kind(I.field.kind)) continue;
    for (int s = 0; s < 3; ++s) cap = std::max<int64_t>(cap, I.s[s].capacity);
    tiles = std::max(tiles, ((I.field.nx + 7) / 8) * ((I.field.ny + 7) / 8));
  }
  if (cap == 0) return QED_OK;
  if (cap > kStaticSortSlots)
    return fail(QED_ERR_ARG, "qed_sort_static handles species of up to %lld slots (capacity %lld here); use qed_sort",
                (long long)kStaticSortSlots, (long long)cap);
  if (tiles > kStaticSortTiles)
    return fail(QED_ERR_ARG, "qed_sort_static handles grids of up to %d tiles of 8 x 8 cells (%d here); use qed_sort",
                kStaticSortTiles, tiles);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != ws->device) return fail(QED_ERR_STATE, "workspace belongs to device %d, current is %d", ws->device, cur);
  SortScratch w;
  HIP_TRY(static_sort_scratch(&w));
  const bool mixed = ws->prec == QED_FP32_MIXED;
  for (int ii = 0; ii < ws->n_inst; ++ii) {
    const qed_instance& I = ws->inst[ii];
    if (!grid_kind(I.field.kind)) continue;
    for (int s = 0; s < 3; ++s) {
      if (I.s[s].capacity == 0) continue;
      HIP_TRY(launch_sort_species(ws->d_inst, I, ii, s, ws->d_glob, params->dt, mixed, w, ws->cus * 8,
                                  (hipStream_t)stream));
    }
  }
  launch_front_clear(ws->d_acc, ws->n_inst, (hipStream_t)stream);  // the photons moved: no front
  HIP_TRY(hipGetLastError());
  ws->win_valid = false;
  return QED_OK;
}

qed_status qed_set_event_queue(qed_workspace* ws, int64_t capacity) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  if (capacity < 1 || capacity > (int64_t(1) << 32))
    return fail(QED_ERR_ARG, "event queue capacity = %lld outside [1, 2^32]", (long long)capacity);
  HIP_TRY(hipSetDevice(ws->device));
  HIP_TRY(hipDeviceSynchronize());
  drop_graph(ws);
  uint64_t* q = nullptr;
  HIP_TRY(hipMalloc((void**)&q, (size_t)capacity * sizeof(uint64_t)));
  hipFree(ws->d_evq);
  ws->d_evq = q;
  ws->evq_cap = capacity;
  return QED_OK;
}

qed_status qed_profile_read(qed_workspace* ws, double* ms, int64_t* launches) {
  if (!ws || !ms || !launches) return fail(QED_ERR_ARG, "NULL argument");
  for (int k = 0; k < QED_PROFILE_CLASSES; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto& mk : ws->ev_marks) {
    HIP_TRY(hipEventSynchronize(mk.second.second));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, mk.second.first, mk.second.second));
    ms[mk.first] += t;
    launches[mk.first] += 1;
  }
  ws->ev_marks.clear();
  ws->ev_used = 0;
  return QED_OK;
}

qed_status qed_compact(qed_workspace* ws, qed_stream stream) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  launch_compact(ws->field_kind, ws->d_inst, ws->n_inst, ws->d_acc, ws->d_glob, ws->d_movers, ws->d_win, ws->d_rec,
                 ws->d_lmask, ws->prec == QED_FP32_MIXED, ws->retire, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return QED_OK;
}

qed_status qed_set_retire(qed_workspace* ws, int32_t n_bins, double eps_min, double eps_max) {
  if (!ws) return fail(QED_ERR_ARG, "workspace is NULL");
  if (n_bins == 0) {
    ws->retire.on = 0;
    return QED_OK;
  }
  if (n_bins < 1 || n_bins > 4096) return fail(QED_ERR_ARG, "n_bins = %d outside [1, 4096]", n_bins);
  if (!finite_pos(eps_min) || !finite_pos(eps_max) || !(eps_max > eps_min))
    return fail(QED_ERR_ARG, "photon energy range [%g, %g] invalid", eps_min, eps_max);
  const size_t len = (size_t)ws->max_inst * (n_bins + 2);
  HIP_TRY(hipSetDevice(ws->device));
  HIP_TRY(hipDeviceSynchronize());
  if (len > ws->spec_len || !ws->retire.spec) {
    hipFree(ws->retire.spec);
    ws->retire.spec = nullptr;
    ws->spec_len = 0;
    HIP_TRY(hipMalloc((void**)&ws->retire.spec, len * sizeof(unsigned long long)));
    ws->spec_len = len;
  }
  HIP_TRY(hipMemset(ws->retire.spec, 0, len * sizeof(unsigned long long)));
  ws->retire.on = 1;
  ws->retire.n_bins = n_bins;
  ws->retire.e_min = eps_min;
  ws->retire.e_max = eps_max;
  return QED_OK;
}

qed_status qed_retired_spectrum(qed_workspace* ws, int32_t inst, int64_t* counts, qed_stream stream) {
  if (!ws || !counts) return fail(QED_ERR_ARG, "NULL argument");
  if (!ws->retire.spec || ws->retire.n_bins < 1) return fail(QED_ERR_STATE, "retirement was never enabled");
  if (inst < 0 || inst >= ws->max_inst) return fail(QED_ERR_ARG, "instance %d outside [0, %d)", inst, ws->max_inst);
  const int nb = ws->retire.n_bins + 2;
  HIP_TRY(hipMemcpyAsync(counts, ws->retire.spec + (size_t)inst * nb, nb * sizeof(int64_t), hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return QED_OK;
}

qed_status qed_energy_ledger(qed_workspace* ws, qed_ledger* out, qed_stream stream) {
  if (!ws || !out) return fail(QED_ERR_ARG, "NULL argument");
  if (!ws->bound) return fail(QED_ERR_STATE, "no instances bound");
  std::vector<InstAcc> acc;
  qed_status st = run_ledger(ws, acc, (hipStream_t)stream);
  if (st) return st;
  bool dropped = false, nonfinite = false;
  for (int i = 0; i < ws->n_inst; ++i) {
    const double w = ws->inst[i].weight;
    const InstAcc& A = acc[i];
    qed_ledger& L = out[i];
    std::memset(&L, 0, sizeof(L));
    double tot = 0.0;
    for (int s = 0; s < 3; ++s) {
      L.energy[s] = fix_value(A.fx[FX_ENERGY + s]) * w;
      L.count[s] = (int64_t)A.led_count[s];
      tot += L.energy[s];
    }
    L.energy0 = ws->e0[i];
    L.work = fix_value(A.fx[FX_WORK]) * w;
    L.defect_emit = fix_value(A.fx[FX_DEFECT_EMIT]) * w;
    L.defect_pair = fix_value(A.fx[FX_DEFECT_PAIR]) * w;
    L.dropped_energy = fix_value(A.fx[FX_DROPPED]) * w;
    L.radiated = fix_value(A.fx[FX_RADIATED]) * w;
    L.retired_energy = fix_value(A.fx[FX_RETIRED]) * w;
    L.n_retired = (int64_t)A.n_retired;
    L.n_emit = (int64_t)A.n_emit;
    L.n_null = (int64_t)A.n_null;
    L.n_pair = (int64_t)A.n_pair;
    L.n_dropped = (int64_t)A.n_dropped;
    L.n_range = (int64_t)A.n_range;
    L.n_nonfinite = (int64_t)A.n_nonfinite;
    L.photon_steps_in_field = (int64_t)A.n_field;
    L.photon_steps_active = (int64_t)A.n_active;
    L.photon_window_reads = (int64_t)A.n_win_reads;
    L.photon_group_reads = (int64_t)A.n_group_reads;
    L.lepton_steps_in_field = (int64_t)A.n_field_lepton;
    for (int s = 0; s < 3; ++s) L.particle_steps[s] = (int64_t)A.particle_steps[s];
    const double resid = tot + L.retired_energy - L.energy0 - L.work - L.defect_emit - L.defect_pair +
                         L.dropped_energy + L.radiated;
    L.drift = L.energy0 > 0.0 ? std::fabs(resid) / L.energy0 : std::fabs(resid);
    dropped |= A.n_dropped > 0;
    nonfinite |= A.n_nonfinite > 0;
  }
  if (nonfinite) return fail(QED_ERR_NONFINITE, "a particle state became non-finite");
  if (dropped) return fail(QED_ERR_CAPACITY, "children were dropped: a species buffer was full");
  return QED_OK;
}

}  // extern "C"
