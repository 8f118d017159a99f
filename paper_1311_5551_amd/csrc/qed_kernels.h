// Kernel argument blocks and host-side launchers shared by the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qed_device.h"

namespace qedk {

struct StepArgs {
  const qed_instance* inst;   // bound instances (device)
  InstAcc* acc;               // per-instance accumulators (device)
  const Glob* glob;           // device clock and chunk-list lengths
  const int64_t* base;        // chunk-list prefix for this kernel's species list
  int n_base;                 // entries in `base`
  int ppt;                    // particles per thread in a chunk
  Tabs tb;
  StepConst sc;
  EvQueue q;                  // pair events of the step (photon passes)
  EmitQueue qe;               // emission events of the step (lepton passes)
  uint32_t* win;              // per-photon pair windows (pack_window); instance i's slots from acc[i].mover_off
  void* rec;                  // per-photon records (PhotonRecT<MIXED, FK>) for the in-window evaluation
  uint64_t* lmask;            // live masks of the photon slot groups; instance i's from acc[i].lmask_off
};

// retirement of photons at compaction (pair window over): the photon spectrum they are counted in
struct RetireSpec {
  int on = 0;
  int n_bins = 0;
  double e_min = 0.0, e_max = 0.0;      // log-spaced bins of photon energy (m c^2)
  unsigned long long* spec = nullptr;   // per instance n_bins + 2 counts (below, bins, above)
};

// scratch of the spatial sort (sized by the caller for the largest species and tile count)
struct SortScratch {
  int32_t* key = nullptr;
  uint32_t* dst = nullptr;
  uint32_t* hist = nullptr;
  int hist_len = 0;
  void* stage = nullptr;  // 8 bytes per slot
};

// the fixed scratch of qed_sort_static: up to 2^21 slots per species and 2^16 tiles of 8 x 8 cells
constexpr int64_t kStaticSortSlots = int64_t(1) << 21;
constexpr int kStaticSortTiles = 1 << 16;
constexpr size_t kStaticSortBytes = (size_t)kStaticSortSlots * 16 + (size_t)kStaticSortTiles * 4;
constexpr int kMaxDevices = 64;
// the device address of that scratch on the current device, split into the sort's arrays
hipError_t static_sort_scratch(SortScratch* out);

hipError_t init_crmath();
hipError_t launch_sort_species(const qed_instance* inst_dev, const qed_instance& inst_host, int ii, int s,
                               const Glob* glob, double dt, bool mixed, const SortScratch& w, int grid, hipStream_t st);
hipError_t launch_build_tables(const qed_table_params& p, double* h, double* lnchi_min, double* dlnchi, double* P,
                               double* T, double* fgrid, double* Pf, double* knorm, double* g, hipStream_t s);
void launch_step_begin(const qed_instance* inst, int n_inst, InstAcc* acc, Glob* glob, EvCtl* evc, EvCtl* emc,
                       int64_t* base_lep, int64_t* base_ph, int chunk_lep, int chunk_ph, int advance,
                       int count_photons, hipStream_t s);
void launch_front_clear(InstAcc* acc, int n_inst, hipStream_t s);
void launch_set_step(const qed_instance* inst, int n_inst, InstAcc* acc, Glob* glob, const uint32_t* win,
                     uint64_t* lmask, int64_t step, hipStream_t s);
void launch_grid_refresh(const qed_instance* inst, int n_inst, const Glob* glob, const StepConst& sc, hipStream_t s);
void launch_lepton(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s);
int photon_blocks_per_cu(int fk, int ppt, int block, int n_cp, bool mixed);
// blocks of 256 threads of the emission pass that fit a CU, with the prefix of `lepton_waves` counts
int emit_blocks_per_cu(int fk, int lepton_waves, bool mixed);
// one step of the field solver of every QED_FIELD_GRID_FDTD instance; max_nodes_rows: the largest
// instance's rows times its runs of 256 columns (the work items of one pass)
void launch_fdtd(const qed_instance* inst, int n_inst, int max_nodes_rows, double dt, hipStream_t s);
int lepton_blocks_per_cu(int fk, int ppt, int block, int n_eta, bool mixed);
void launch_photon(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s);
void launch_pair_events(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s);
void launch_emit_events(int fk, const StepArgs& a, int grid, int block, bool mixed, hipStream_t s);
void launch_init_tau(const qed_instance* inst, int n_inst, hipStream_t s);
void launch_ledger(const qed_instance* inst, int n_inst, InstAcc* acc, bool mixed, hipStream_t s);
void launch_compact(int fk, const qed_instance* inst, int n_inst, InstAcc* acc, const Glob* glob, int64_t* movers,
                    uint32_t* win, void* rec, uint64_t* lmask, bool mixed, const RetireSpec& rs, hipStream_t s);
void launch_photon_windows(int fk, const qed_instance* inst, int n_inst, InstAcc* acc, const Glob* glob, uint32_t* win,
                           void* rec, uint64_t* lmask, double t0, double dt, double cp_min, bool mixed, hipStream_t s);

}  // namespace qedk
