/*
 * qed.h -- C ABI of libqed: the per-particle QED Monte-Carlo emission step of
 * Ridgers et al., "Modelling gamma-ray photon emission and pair production in
 * high-intensity laser-matter interactions" (arXiv:1311.5551), on MI355X (gfx950).
 *
 * Pointers named *_dev are device memory on the device that was current when the
 * handle they are used with was created; other pointers are host memory.  Nothing
 * here takes ownership of caller memory.  Every call returns a qed_status and never
 * throws, aborts or exits; after a non-OK return qed_last_error() describes it.
 *
 * Code units (both sides of this interface):
 *   time t' = w t with w = 2 pi c / lambda_L;  length x' = w x / c;
 *   lepton momentum u = p/(m c), gamma = sqrt(1 + |u|^2);
 *   photon momentum k = p/(m c), energy |k| m c^2;
 *   fields E' = E/E_s and B' = c B/E_s (E_s the Schwinger field).
 */
#ifndef QED_H
#define QED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* qed_stream; /* a hipStream_t; NULL = the null stream */

typedef enum {
  QED_OK = 0,
  QED_ERR_ARG = -1,       /* invalid argument; nothing was enqueued */
  QED_ERR_HIP = -2,       /* HIP runtime failure; qed_last_error() has the HIP message */
  QED_ERR_CAPACITY = -3,  /* children were dropped because a species buffer was full */
  QED_ERR_NONFINITE = -4, /* a particle state became non-finite */
  QED_ERR_STATE = -5,     /* call order violated (e.g. a step before qed_bind) */
  QED_ERR_DEVICE = -6     /* the current device is not a gfx950 GPU */
} qed_status;

typedef enum { QED_FP64 = 0, QED_FP32_MIXED = 1 } qed_precision;

/* step flags */
enum {
  QED_EMIT = 1u,      /* leptons emit photons (Sec. 3: optical depth, P_chi sampling, recoil) */
  QED_PAIRS = 2u,     /* photons create pairs (Sec. 3: optical depth with T_pm, P_f sampling) */
  QED_PROPAGATE = 4u, /* photons are stepped; without it emitted photons are only recorded (Sec. 3.1) */
  /* Deterministic radiation reaction instead of emission (Sec. 2.4, eqs. 8 and 9): after the push
   * each lepton loses the energy radiated in the step, dgamma/dt = -(2/3) alpha kappa eta^2 g(eta)
   * in code time, along its momentum; no photons are made, the energy goes to the ledger's
   * `radiated`.  QED_RR_QUANTUM uses the quantum reduction g(eta) from the tables, QED_RR_CLASSICAL
   * g = 1 (the Landau-Lifshitz leading term).  Each excludes QED_EMIT and the other. */
  QED_RR_QUANTUM = 8u,
  QED_RR_CLASSICAL = 16u
};

/* field kinds; p[] parameters in code units */
enum {
  QED_FIELD_UNIFORM = 0,         /* p = {Ex, Ey, Ez, Bx, By, Bz} */
  QED_FIELD_LP_PULSE = 1,        /* p = {E0, Psi, psi0, phase}: psi = t - x - psi0,
                                    E_y = B_z = E0 sin^2(pi psi/Psi) cos(psi + phase) on 0 <= psi <= Psi */
  QED_FIELD_CP_WAVE = 2,         /* p = {E0, phase}: psi = t - x + phase, E = E0 (0, cos psi, sin psi),
                                    B = x_hat x E (Sec. 2.4 test configuration) */
  QED_FIELD_CP_STANDING = 3,     /* p = {E0}: two counter-propagating CP waves, E_y = 2E0 cos t cos x,
                                    E_z = 2E0 sin t cos x, B_y = 2E0 cos t sin x, B_z = 2E0 sin t sin x */
  QED_FIELD_GRID_CP_STANDING = 4, /* the standing wave written each step onto a 2-D Yee grid (FP32) and
                                    gathered with first-order (cloud-in-cell) weights (Sec. 3.2) */
  QED_FIELD_GRID_FDTD = 5        /* p = {Q}: field feedback (Sec. 3.2, the coupling to a PIC code): the
                                    fields of a 2-D Yee grid (FP64, fdtd_dev) gathered as above; after
                                    each step the leptons' current (charge -Q electrons, +Q positrons
                                    per macro-particle, code units, per unit length along z) is
                                    deposited with the charge-conserving split of Esirkepov for
                                    first-order shapes, and the grid advances one step of Maxwell's
                                    equations (dE/dt = curl B - J, dB/dt = -curl E; B half a step,
                                    E a full step, B half a step).  FP64 only, 2-D only. */
};

/* ---------------------------------------------------------------------------
 * Look-up tables (Sec. 3): h(eta) and T(chi) are read by linear interpolation between
 * tabulated nodes, and photon chi and pair split f are drawn by inverting the tabulated
 * cumulative probabilities P_chi(eta, chi) and P_f(f, chi).  Built on the device from
 * the integrals of Appendix A and B.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_eta;              /* rows of h and P_chi, log-spaced eta in [eta_min, eta_max]; 2..1024 */
  double eta_min, eta_max;
  int32_t n_chi;              /* columns of P_chi: log-spaced chi from chi_min(eta) to eta/2; >= 2 */
  double cutoff_energy_frac;  /* chi_min(eta): photons below it carry this share of the energy (1e-9) */
  int32_t n_chi_pair;         /* rows of T and P_f, log-spaced chi in [chi_pair_min, chi_pair_max]; 2..1024 */
  double chi_pair_min, chi_pair_max;
  int32_t n_f;                /* columns of P_f: f_l = sin^2(pi l / 2(n_f - 1)); >= 3 */
} qed_table_params;

typedef struct qed_tables qed_tables; /* opaque, immutable after creation, shareable across streams */

/* Host copies of the tables (valid until qed_tables_destroy):
 *   h[n_eta]                      h(eta_i) = int_0^{eta_i/2} F/chi dchi  (Appendix A)
 *   lnchi_min[n_eta], dlnchi[n_eta]  row grids: ln chi_ij = lnchi_min[i] + j dlnchi[i]
 *   P_chi[n_eta][n_chi]           P(eta_i, chi_ij); column 0 is the share below the cut, last is 1
 *   T[n_chi_pair]                 T_pm(chi_k) = 0.16 K_{1/3}^2(2/(3 chi_k)) / chi_k  (Appendix B)
 *   f_grid[n_f], P_f[n_chi_pair][n_f], k_norm[n_chi_pair]   cumulative p_f and its normaliser
 *   g[n_eta]                      g(eta_i) = 3 sqrt3 / (2 pi eta_i^2) int_0^{eta_i/2} F dchi, the
 *                                 quantum reduction of the radiated power (Appendix A, eq. 8) */
typedef struct {
  qed_table_params params;
  const double *h, *lnchi_min, *dlnchi, *P_chi, *T, *f_grid, *P_f, *k_norm;
  const double* g;            /* NULL for tables supplied without g */
} qed_table_view;

/* Builds all tables on the current device (FP64 quadrature of the Appendix A/B integrals) and
 * keeps device and host copies.  Synchronous.  QED_ERR_ARG on out-of-range parameters. */
qed_status qed_build_tables(const qed_table_params* params, qed_tables** out);

/* Wraps tables supplied as host arrays (e.g. published tables), laid out as in qed_table_view;
 * k_norm and g may be NULL (without g, steps with QED_RR_QUANTUM return QED_ERR_STATE).  Copies
 * them; the caller keeps its arrays. */
qed_status qed_tables_from_host(const qed_table_params* params, const double* h, const double* lnchi_min,
                                const double* dlnchi, const double* P_chi, const double* T,
                                const double* f_grid, const double* P_f, const double* k_norm,
                                const double* g, qed_tables** out);

qed_status qed_tables_view(const qed_tables* tables, qed_table_view* out);
void qed_tables_destroy(qed_tables* tables);

/* ---------------------------------------------------------------------------
 * Particles: one structure-of-arrays per species, caller-owned device memory.
 * Species order inside an instance: 0 electrons (charge -1), 1 positrons (+1), 2 photons.
 * Element type of x..uz: double in QED_FP64; float in QED_FP32_MIXED.
 * ------------------------------------------------------------------------- */
typedef struct {
  void *x_dev, *y_dev, *z_dev;      /* leptons: position; photons: position at birth.  z NULL in 2-D */
  void *ux_dev, *uy_dev, *uz_dev;   /* leptons: u; photons: k */
  float *x_lo_dev, *y_lo_dev, *z_lo_dev;    /* QED_FP32_MIXED leptons: low words of compensated */
  float *ux_lo_dev, *uy_lo_dev, *uz_lo_dev; /* position and momentum (value = hi + lo); else NULL */
  int32_t* birth_step_dev;          /* photons: step at whose start the photon sits at its birth
                                       position; it moves ballistically: x(step n) = x_b + (n - b) dt k/|k| */
  double* tau_dev;                  /* remaining optical depth (FP64 in both precisions); a photon with
                                       tau < 0 has been converted to a pair and awaits qed_compact */
  uint64_t* uid_dev;                /* particle id; keys the random stream of the particle */
  int64_t* count_dev;               /* number of particles in [0, count); device-resident, updated by the
                                       library as children are appended and photons compacted */
  int64_t capacity;                 /* length of every array above */
} qed_species;

typedef struct {
  int32_t kind;                     /* QED_FIELD_* */
  double p[16];
  float* grid_dev;                  /* GRID kinds: 6 x ny x nx floats, components Ex, Ey, Ez, Bx, By, Bz,
                                       x fastest; Yee offsets Ex(i+1/2, j), Ey(i, j+1/2), Ez(i, j),
                                       Bx(i, j+1/2), By(i+1/2, j), Bz(i+1/2, j+1/2); periodic */
  int32_t nx, ny;
  double dx, dy, x0, y0;
  double* fdtd_dev;                 /* QED_FIELD_GRID_FDTD: 9 x ny x nx doubles, caller-owned, read and
                                       written by qed_step: Ex, Ey, Ez, Bx, By, Bz at the staggered
                                       nodes above (E and B both at the start of the next step), then
                                       Jx, Jy, Jz at the nodes of Ex, Ey, Ez (zero between steps: the
                                       library clears them once the step's field update has used
                                       them; the caller passes them zeroed).  Else NULL. */
} qed_field;

typedef struct {
  qed_species s[3];
  qed_field field;
  double weight;                    /* real particles per macro-particle (children inherit it, Sec. 3.2) */
  uint64_t seed;                    /* Philox4x64-10 key = (seed, key_instance) */
  uint64_t key_instance;
  int32_t dims;                     /* 3, or 2 for x-y motion (z_dev NULL) */
} qed_instance;

typedef struct {
  double t0;          /* code time of step 0: step n runs from t0 + n dt to t0 + (n+1) dt */
  double dt;
  double lambda_L;    /* laser wavelength (m) that defines the code units */
  uint32_t flags;     /* QED_EMIT | QED_PAIRS | QED_PROPAGATE | QED_RR_QUANTUM | QED_RR_CLASSICAL */
  qed_precision precision;
} qed_step_params;

typedef struct qed_workspace qed_workspace; /* opaque: device state of bound instances */

/* Workspace for up to max_inst instances on the current device. */
qed_status qed_workspace_create(int32_t max_inst, qed_workspace** out);
void qed_workspace_destroy(qed_workspace* ws);

/* Binds instances (host array, copied; the device arrays they point to stay caller-owned and
 * must outlive all work enqueued on them), checks their shapes, allocates scratch sized to the
 * capacities, zeroes the event counters and records the initial energy.  Synchronous. */
qed_status qed_bind(qed_workspace* ws, const qed_instance* inst, int32_t n_inst,
                    const qed_step_params* params);

/* Launch shape of the sweep kernels: threads per block (64..256, multiple of 64) and particles
 * per thread (1, 2, 4 or 8; the photon sweep also 16); qed_set_launch sets both sweeps, qed_set_kernel_launch one of
 * them (kernel = QED_KERNEL_LEPTON or QED_KERNEL_PHOTON, the profile-class indices).  Takes
 * effect from the next step; drops a captured graph.  Results do not depend on the shape
 * (per-uid random streams, ledger sums in exact fixed point), except with field feedback
 * (QED_FIELD_GRID_FDTD), whose current sums over particles have no fixed order. */
#define QED_KERNEL_LEPTON 1
#define QED_KERNEL_PHOTON 2
qed_status qed_set_launch(qed_workspace* ws, int32_t block, int32_t ppt);
qed_status qed_set_kernel_launch(qed_workspace* ws, int32_t kernel, int32_t block, int32_t ppt);

/* Capacity (entries of 8 bytes, 1..2^32; default 2^20) of the per-step queue through which the
 * photon pass hands photons whose optical depth reached zero to the pair-creation pass.  A step
 * with more pair events than this finds the excess by a sweep over all photons: same results,
 * slower step.  Reallocates (synchronous); drops a captured graph. */
qed_status qed_set_event_queue(qed_workspace* ws, int64_t capacity);

/* Sec. 3: every macro-particle starts with a sampled optical depth, tau = -ln U with U from the
 * particle's stream at counter (uid, 0, INIT, 0), for every particle in [0, count) except the
 * converted photons still waiting for qed_compact (tau = -1), which stay converted.  Async. */
qed_status qed_init_optical_depth(qed_workspace* ws, qed_stream stream);

/* Sets the index of the next step (device-resident clock; graph-capturable).  Async. */
qed_status qed_set_step(qed_workspace* ws, int64_t step, qed_stream stream);

/* One Monte-Carlo step (Sec. 3; in the PIC coupling of Sec. 3.2 it follows the particle push):
 * for every lepton present at the start of the step: fields at (x^n, t^n), Boris push, eta,
 * tau -= lambda_gamma(eta) dt; on tau <= 0 sample chi from P_chi, recoil, append the photon and
 * redraw tau.  For every photon (QED_PAIRS): move at c, chi, tau -= lambda_pm(chi) dt; on
 * tau <= 0 sample f from P_f, append the pair, mark the photon dead.  Children are first stepped
 * in the next step.  Never allocates; async on `stream`; device-side conditions (full buffers,
 * non-finite state) are reported by the next qed_energy_ledger.  The first step after qed_bind,
 * and any step whose t0, dt or tables differ from the previous one's, also enqueues a pass that
 * sets every photon's pair window (the steps in which its pair rate can be non-zero) and the
 * live mask of every group of 64 photon slots (a bit per photon whose window is not over); a
 * caller capturing qed_step into its own graph should run one step before capturing.  The
 * photon pass reads only the photons whose live bit is set; the emission pass sets the bits of
 * the photons it appends and the photon pass clears those whose window is over. */
qed_status qed_step(const qed_tables* tables, qed_workspace* ws, const qed_step_params* params,
                    qed_stream stream);

/* n_steps steps; steps are replayed from a HIP graph of graph_steps steps (captured once per
 * workspace and launch shape; 0 = plain launches).  Async. */
qed_status qed_run(const qed_tables* tables, qed_workspace* ws, const qed_step_params* params,
                   int64_t n_steps, int32_t graph_steps, qed_stream stream);

/* Reorders the particles of every bound instance with a grid field (QED_FIELD_GRID_CP_STANDING,
 * QED_FIELD_GRID_FDTD)
 * by 8 x 8-cell tile of their position (photons: position at the start of the next step, using
 * params->dt), so that neighbouring particles gather from the same grid cache lines.  A counting
 * sort and a permutation of every array of each species; the order within a tile is not
 * specified, per-uid results of later steps are unchanged.  Allocates its scratch on the first
 * call that needs it (synchronising `stream`), then is async; up to 2^32 - 1 slots per species
 * (QED_ERR_ARG beyond).  Instances with analytic fields are left as they are. */
qed_status qed_sort(qed_workspace* ws, const qed_step_params* params, qed_stream stream);

/* qed_sort without allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same reordering, with its
 * scratch (tile keys, destination slots, staging, tile histogram) in a fixed array of 32.25 MB
 * that the library holds in device memory on every GPU it runs on until the process ends.
 * Species of up to 2^21 slots (capacity) and grids of up to 2^16 tiles of 8 x 8 cells; larger
 * ones return QED_ERR_ARG before anything is enqueued.  Async on `stream`; never allocates.
 * All calls on one GPU share that GPU's array: calls that overlap on one GPU (other streams,
 * other threads, other workspaces) race and must be ordered by the caller. */
qed_status qed_sort_static(qed_workspace* ws, const qed_step_params* params, qed_stream stream);

/* Removes the photons that pair creation annihilated (Sec. 3: the photon is deleted when it
 * creates a pair; tau < 0 marks it until then) from every bound photon species, by moving live
 * photons from the tail into the holes (order is not preserved).  With retirement on
 * (qed_set_retire) it also removes the photons whose pair window is over: they can never create
 * a pair again (the paper deletes photons that cannot matter for pair creation, Sec. 3.1); their
 * energy goes to the ledger's retired_energy and each is counted in its instance's photon
 * spectrum.  Then it puts the photons whose window is over in front of the others (the photon
 * sweep starts after them) and rebuilds the live masks of the groups of 64 photon slots.
 * Call it periodically (e.g. every 100 steps).  Async; graph-capturable. */
qed_status qed_compact(qed_workspace* ws, qed_stream stream);

/* Retirement of photons at compaction (see qed_compact): n_bins > 0 turns it on, with a photon
 * spectrum of n_bins log-spaced bins of photon energy |k| over [eps_min, eps_max] (m c^2) per
 * instance, plus an underflow and an overflow bin; n_bins = 0 turns it off.  Allocates and
 * zeroes the spectra (synchronous); a new qed_bind zeroes them again. */
qed_status qed_set_retire(qed_workspace* ws, int32_t n_bins, double eps_min, double eps_max);

/* The retired-photon spectrum of instance `inst`: counts[0] below eps_min, counts[1..n_bins]
 * the bins, counts[n_bins + 1] at or above eps_max.  Synchronises `stream`. */
qed_status qed_retired_spectrum(qed_workspace* ws, int32_t inst, int64_t* counts, qed_stream stream);

/* Energy account of one instance (Sec. 3.1 and Table 2), in m c^2 times the weight. */
typedef struct {
  double energy[3];       /* sum of gamma (leptons) and |k| (live photons) now */
  double energy0;         /* total at qed_bind */
  double work;            /* field work on leptons in the pushes since qed_bind */
  double defect_emit;     /* sum over emissions of gamma_after + |k| - gamma_before */
  double defect_pair;     /* sum over pair creations of gamma_- + gamma_+ - |k| */
  double dropped_energy;  /* energy of children that did not fit their buffer */
  double radiated;        /* energy removed by deterministic radiation reaction (QED_RR_*) */
  double retired_energy;  /* energy of the photons retired at compaction (qed_set_retire) */
  int64_t n_retired;      /* photons retired */
  int64_t count[3];
  int64_t n_emit, n_null, n_pair;  /* emissions, draws below the cut-off, pair creations */
  int64_t n_dropped, n_range, n_nonfinite;
  int64_t photon_steps_in_field;   /* photon steps that saw a non-zero pair rate */
  int64_t photon_steps_active;     /* photon steps evaluated in full: those inside the photon's pair
                                      window (the steps in which its pair rate can be non-zero) */
  int64_t lepton_steps_in_field;   /* lepton steps with the full push (all of them, except outside a
                                      plane-wave pulse, where the push is the field-free drift) */
  int64_t photon_window_reads;     /* photon slot-steps whose pair window was read: the slots whose
                                      live bit was set (a photon whose window is not over) */
  int64_t photon_group_reads;      /* live masks read (one 64-bit mask per group of 64 photon slots
                                      the photon sweep visits) */
  int64_t particle_steps[3];       /* particles present at the start of each step, summed over the
                                      steps since qed_bind (photons: buffer slots, incl. dead ones
                                      not yet compacted, counted in steps with QED_PAIRS, the steps
                                      in which photons are advanced) */
  double drift;           /* |sum energy + retired - energy0 - work - defects + dropped + radiated| / energy0 */
} qed_ledger;

/* Fills out[0..n_inst-1] for the bound instances.  Synchronises `stream`.  Returns
 * QED_ERR_CAPACITY or QED_ERR_NONFINITE (after filling out) if that happened since qed_bind. */
qed_status qed_energy_ledger(qed_workspace* ws, qed_ledger* out, qed_stream stream);

/* Kernel timing with HIP events recorded around each kernel of qed_step on its stream (not
 * available inside qed_run's graph replay).  qed_profile_read synchronises and writes, for the
 * QED_PROFILE_CLASSES kernel classes [0] step set-up (snapshot, grid refresh), [1] lepton
 * sweep, [2] photon sweep, [3] pair-creation pass, [4] photon-emission pass, [5] field solver
 * (QED_FIELD_GRID_FDTD), the summed durations in milliseconds and the launch counts since
 * qed_profile(ws, 1) or the previous read, and keeps timing. */
#define QED_PROFILE_CLASSES 6
qed_status qed_profile(qed_workspace* ws, int32_t enable);
qed_status qed_profile_read(qed_workspace* ws, double* ms, int64_t* launches);

/* Thread-local description of the last non-OK status. */
const char* qed_last_error(void);

/* Library build identifier. */
const char* qed_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QED_H */
