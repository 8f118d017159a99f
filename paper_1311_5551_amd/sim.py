"""Run driver: allocates caller-owned particle buffers (torch tensors on the GPU) for
one or more workloads, binds them to a libqed workspace and steps them.  PyTorch is
used only for device memory and streams; every step of the method runs in libqed.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import capi
from .workloads import Workload

SPECIES = ("electron", "positron", "photon")
DEFAULT_TABLE_PARAMS = dict(n_eta=256, eta_min=1e-4, eta_max=1e2, n_chi=256, cutoff_energy_frac=1e-9,
                            n_chi_pair=256, chi_pair_min=1e-2, chi_pair_max=1e2, n_f=256)


class Tables:
    """Device look-up tables (qed_build_tables or qed_tables_from_host)."""

    def __init__(self, handle, params: dict):
        self.handle = handle
        self.params = params

    @classmethod
    def build(cls, **overrides):
        p = dict(DEFAULT_TABLE_PARAMS)
        p.update(overrides)
        return cls(capi.qed_build_tables(capi.qed_table_params(**p)), p)

    @classmethod
    def from_arrays(cls, t: dict):
        p = dict(t["params"])
        arrs = [np.ascontiguousarray(t[k], dtype=np.float64) for k in
                ("h", "lnchi_min", "dlnchi", "P_chi", "T", "f_grid", "P_f")]
        kn = np.ascontiguousarray(t["k_norm"], dtype=np.float64) if "k_norm" in t else None
        g = np.ascontiguousarray(t["g"], dtype=np.float64) if t.get("g") is not None else None
        return cls(capi.qed_tables_from_host(capi.qed_table_params(**p), *arrs, kn, g), p)

    def view(self) -> dict:
        v = capi.qed_tables_view(self.handle)
        p = self.params
        ne, nc, npair, nf = p["n_eta"], p["n_chi"], p["n_chi_pair"], p["n_f"]
        get = lambda ptr, n: np.ctypeslib.as_array(ptr, shape=(n,)).copy()
        return dict(params=dict(p), h=get(v.h, ne), lnchi_min=get(v.lnchi_min, ne), dlnchi=get(v.dlnchi, ne),
                    P_chi=get(v.P_chi, ne * nc).reshape(ne, nc), T=get(v.T, npair), f_grid=get(v.f_grid, nf),
                    P_f=get(v.P_f, npair * nf).reshape(npair, nf), k_norm=get(v.k_norm, npair),
                    g=get(v.g, ne) if v.g else None)

    def __del__(self):
        try:
            if self.handle:
                capi.qed_tables_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Run:
    """One bound set of instances (one workload, or a batch sharing dt, t0 and flags)."""

    def __init__(self, workloads, tables: Tables, precision: int = capi.QED_FP64, capacity: dict | None = None,
                 device: str = "cuda:0", block: int = 256, ppt: int = 4, step0: int = 0,
                 draw_initial_tau: bool = True, photons=None, initial: list | None = None):
        """`initial`, if given, holds per instance a dict species -> arrays (as returned by
        species(..., live_only=False)) that replaces the workload's electrons (restart)."""
        import torch
        self.torch = torch
        if isinstance(workloads, Workload):
            workloads = [workloads]
        self.workloads = list(workloads)
        w0 = self.workloads[0]
        for w in self.workloads:
            if (w.dt, w.t0, w.flags, w.field_kind, w.dims) != (w0.dt, w0.t0, w0.flags, w0.field_kind, w0.dims):
                raise ValueError("batched workloads must share dt, t0, flags, field kind and dims")
        self.tables = tables
        self.precision = precision
        self.mixed = precision == capi.QED_FP32_MIXED
        self.dev = torch.device(device)
        torch.cuda.set_device(self.dev)
        self.stream = torch.cuda.Stream(device=self.dev)
        self.dt, self.t0, self.flags, self.dims = w0.dt, w0.t0, w0.flags, w0.dims
        self.params = capi.qed_step_params(t0=self.t0, dt=self.dt, lambda_L=1e-6, flags=self.flags,
                                           precision=precision)
        fdt = torch.float32 if self.mixed else torch.float64
        self.bufs = []
        insts = []
        for wi, w in enumerate(self.workloads):
            cap = dict(electron=4 * w.n + 1024, positron=w.n + 1024, photon=8 * w.n + 4096)
            cap.update(w.capacity or {})
            cap.update(capacity or {})
            inst = capi.qed_instance()
            b = {}
            for si, name in enumerate(SPECIES):
                n_cap = int(cap[name])
                sb = {}
                for k in ("x", "y", "z", "ux", "uy", "uz"):
                    sb[k] = None if (k == "z" and self.dims == 2) else torch.zeros(max(n_cap, 1), dtype=fdt,
                                                                                   device=self.dev)
                    if self.mixed and si < 2:
                        sb[k + "_lo"] = None if (k == "z" and self.dims == 2) else torch.zeros(
                            max(n_cap, 1), dtype=torch.float32, device=self.dev)
                sb["tau"] = torch.zeros(max(n_cap, 1), dtype=torch.float64, device=self.dev)
                sb["uid"] = torch.zeros(max(n_cap, 1), dtype=torch.int64, device=self.dev)
                sb["birth_step"] = torch.zeros(max(n_cap, 1), dtype=torch.int32, device=self.dev) if si == 2 else None
                sb["count"] = torch.zeros(1, dtype=torch.int64, device=self.dev)
                sb["capacity"] = n_cap
                b[name] = sb
                sp = inst.s[si]
                for k in ("x", "y", "z", "ux", "uy", "uz"):
                    setattr(sp, k + "_dev", _ptr(sb[k]))
                    if self.mixed and si < 2:
                        setattr(sp, k + "_lo_dev", _ptr(sb[k + "_lo"]))
                sp.birth_step_dev = _ptr(sb["birth_step"])
                sp.tau_dev = _ptr(sb["tau"])
                sp.uid_dev = _ptr(sb["uid"])
                sp.count_dev = _ptr(sb["count"])
                sp.capacity = n_cap
            if initial is not None:
                for si, name in enumerate(SPECIES):
                    if name in initial[wi] and len(initial[wi][name]["uid"]):
                        self._load(b[name], initial[wi][name], lepton=si < 2)
            else:
                self._load(b["electron"], w.electrons, lepton=True)
                if photons is not None and wi == 0:
                    self._load(b["photon"], photons, lepton=False)
            f = inst.field
            f.kind = w.field_kind
            fp = list(w.field) + [0.0] * (16 - len(w.field))
            f.p = (C.c_double * 16)(*fp)
            if w.field_kind in (capi.QED_FIELD_GRID_CP_STANDING, capi.QED_FIELD_GRID_FDTD):
                nx, ny, dx, dy, x0, y0 = w.grid
                f.nx, f.ny, f.dx, f.dy, f.x0, f.y0 = nx, ny, dx, dy, x0, y0
            if w.field_kind == capi.QED_FIELD_GRID_CP_STANDING:
                b["grid"] = torch.zeros(6 * nx * ny, dtype=torch.float32, device=self.dev)
                f.grid_dev = _ptr(b["grid"])
            elif w.field_kind == capi.QED_FIELD_GRID_FDTD:
                # the solver's planes Ex..Bz, Jx..Jz (FP64), from the workload's initial fields
                init = np.zeros((9, ny, nx)) if w.fields is None else np.asarray(w.fields, dtype=np.float64)
                if init.shape != (9, ny, nx):
                    raise ValueError("initial field planes must have shape (9, ny, nx)")
                b["fdtd"] = torch.as_tensor(np.ascontiguousarray(init).reshape(-1)).to(self.dev)
                f.fdtd_dev = _ptr(b["fdtd"])
            inst.weight = w.weight
            inst.seed = w.seed
            inst.key_instance = w.instance
            inst.dims = w.dims
            insts.append(inst)
            self.bufs.append(b)
        self.insts = insts
        torch.cuda.synchronize(self.dev)
        self.ws = capi.qed_workspace_create(len(insts))
        capi.qed_set_launch(self.ws, block, ppt)
        capi.qed_bind(self.ws, insts, self.params)
        if draw_initial_tau:
            capi.qed_init_optical_depth(self.ws, self._s())
        capi.qed_set_step(self.ws, step0, self._s())
        self.step_index = step0

    # -- helpers -----------------------------------------------------------------
    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _load(self, sb, d, lepton):
        torch = self.torch
        n = len(d["uid"])
        if n > sb["capacity"]:
            raise ValueError("initial particles exceed capacity")
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            if sb[k] is None:
                continue
            v = torch.as_tensor(np.asarray(d.get(k, np.zeros(n)), dtype=np.float64))
            if self.mixed:
                hi = v.to(torch.float32)
                sb[k][:n].copy_(hi)
                if lepton:
                    sb[k + "_lo"][:n].copy_((v - hi.to(torch.float64)).to(torch.float32))
            else:
                sb[k][:n].copy_(v)
        if "tau" in d:
            sb["tau"][:n].copy_(torch.as_tensor(np.asarray(d["tau"], dtype=np.float64)))
        sb["uid"][:n].copy_(torch.as_tensor(np.asarray(d["uid"], dtype=np.uint64).view(np.int64)))
        if sb["birth_step"] is not None and "birth_step" in d:
            sb["birth_step"][:n].copy_(torch.as_tensor(np.asarray(d["birth_step"], dtype=np.int32)))
        sb["count"].fill_(n)

    # -- the C ABI calls -----------------------------------------------------------
    def set_launch(self, block, ppt):
        capi.qed_set_launch(self.ws, block, ppt)

    def set_kernel_launch(self, kernel: int, block: int, ppt: int):
        capi.qed_set_kernel_launch(self.ws, kernel, block, ppt)

    def set_event_queue(self, capacity: int):
        capi.qed_set_event_queue(self.ws, capacity)

    def step(self, n: int = 1):
        for _ in range(n):
            capi.qed_step(self.tables.handle, self.ws, self.params, self._s())
        self.step_index += n

    def run(self, n: int, graph_steps: int = 0):
        capi.qed_run(self.tables.handle, self.ws, self.params, n, graph_steps, self._s())
        self.step_index += n

    def compact(self):
        capi.qed_compact(self.ws, self._s())

    def set_retire(self, n_bins: int, eps_min: float = 1e-3, eps_max: float = 1e4):
        """Retire photons whose pair window is over at each compaction (n_bins = 0: off)."""
        capi.qed_set_retire(self.ws, n_bins, eps_min, eps_max)
        self.retire_bins = n_bins

    def retired_spectrum(self, inst: int = 0):
        """Counts of retired photons: [below, bins..., above]."""
        return capi.qed_retired_spectrum(self.ws, inst, self.retire_bins, self._s())

    def sort(self):
        capi.qed_sort(self.ws, self.params, self._s())

    def sort_static(self):
        """qed_sort_static: the same reordering with the library's fixed scratch (no allocation)."""
        capi.qed_sort_static(self.ws, self.params, self._s())

    def fields(self, inst: int = 0):
        """The solver planes (9, ny, nx) of a field-feedback instance as they stand (Ex Ey Ez Bx By
        Bz at the start of the next step; the current planes are zero between steps)."""
        nx, ny = self.workloads[inst].grid[:2]
        self.synchronize()
        return self.bufs[inst]["fdtd"].cpu().numpy().reshape(9, ny, nx)

    def ledger(self):
        st, led = capi.qed_energy_ledger(self.ws, len(self.insts), self._s())
        for d in led:
            d["status"] = capi.STATUS_NAMES[st]
        return led

    def profile(self, enable: bool = True):
        capi.qed_profile(self.ws, enable)

    def profile_read(self):
        """(ms, launches) per kernel class: [set-up, lepton sweep, photon sweep, pair events, emission events]."""
        return capi.qed_profile_read(self.ws)

    def synchronize(self):
        self.stream.synchronize()

    # -- read-back ---------------------------------------------------------------------
    def count(self, inst: int = 0, species: str = "photon") -> int:
        self.stream.synchronize()
        return min(int(self.bufs[inst][species]["count"].item()), self.bufs[inst][species]["capacity"])

    def species(self, inst: int = 0, name: str = "electron", live_only: bool = True) -> dict:
        """Host copy of one species: x, y, (z), ux, uy, uz as FP64 (hi + lo in the mixed form),
        tau, uid (uint64) and, for photons, birth_step."""
        self.stream.synchronize()
        sb = self.bufs[inst][name]
        n = self.count(inst, name)
        out = {}
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            if sb[k] is None:
                continue
            v = sb[k][:n].double()
            if (k + "_lo") in sb and sb[k + "_lo"] is not None:
                v = v + sb[k + "_lo"][:n].double()
            out[k] = v.cpu().numpy()
        out["tau"] = sb["tau"][:n].cpu().numpy()
        out["uid"] = sb["uid"][:n].cpu().numpy().view(np.uint64)
        if sb["birth_step"] is not None:
            out["birth_step"] = sb["birth_step"][:n].cpu().numpy()
        if live_only and name == "photon":
            keep = ~(out["tau"] < 0)
            out = {k: v[keep] for k, v in out.items()}
        return out

    def state(self) -> list:
        """Full particle state of every instance (restartable with Run(..., initial=...,
        draw_initial_tau=False, step0=step_index)); with the counter-based generator this is
        the whole state of the run."""
        return [{name: self.species(i, name, live_only=False) for name in SPECIES} for i in range(len(self.insts))]

    def close(self):
        if getattr(self, "ws", None):
            capi.qed_workspace_destroy(self.ws)
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
