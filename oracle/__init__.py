"""Python access to the FP64 CPU oracle (test infrastructure only).

Only tests/, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it.

Functions mirror the paper's objects: F(eta, chi), h, g (Appendix A), T_pm,
p_f, k (Appendix B), the look-up tables of Sec. 3, Philox4x64-10, and the
Monte-Carlo step of Sec. 3 run over whole particle families.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None

FLAG_EMIT = 1
FLAG_PAIRS = 2
FLAG_PROPAGATE = 4
FLAG_RR_QUANTUM = 8      # continuous radiation reaction, power P_c g(eta) (eqs. 8, 9, Appendix A)
FLAG_RR_CLASSICAL = 16   # continuous radiation reaction, classical power (g = 1)

FIELD_UNIFORM = 0
FIELD_LP_PULSE = 1
FIELD_CP_WAVE = 2
FIELD_CP_STANDING = 3
FIELD_GRID_CP_STANDING = 4
FIELD_GRID_FDTD = 5      # p = {Q}: Yee grid advanced by Maxwell's equations with the leptons' current

SPECIES = ("electron", "positron", "photon")


class _TableParams(C.Structure):
    _fields_ = [("n_eta", C.c_int32), ("eta_min", C.c_double), ("eta_max", C.c_double),
                ("n_chi", C.c_int32), ("cutoff_energy_frac", C.c_double),
                ("n_chi_pair", C.c_int32), ("chi_pair_min", C.c_double), ("chi_pair_max", C.c_double),
                ("n_f", C.c_int32)]


class _Config(C.Structure):
    _fields_ = [("field_kind", C.c_int32), ("field", C.c_double * 16),
                ("grid_nx", C.c_int32), ("grid_ny", C.c_int32),
                ("grid_dx", C.c_double), ("grid_dy", C.c_double),
                ("grid_x0", C.c_double), ("grid_y0", C.c_double),
                ("dims", C.c_int32), ("dt", C.c_double), ("t0", C.c_double),
                ("step0", C.c_int64), ("n_steps", C.c_int64),
                ("seed", C.c_uint64), ("instance", C.c_uint64), ("flags", C.c_uint32),
                ("draw_initial_tau", C.c_int32), ("lambda_L", C.c_double)]


class _Tables(C.Structure):
    _fields_ = [("n_eta", C.c_int32), ("eta_min", C.c_double), ("eta_max", C.c_double),
                ("h", C.POINTER(C.c_double)),
                ("n_chi", C.c_int32), ("lnchi_min", C.POINTER(C.c_double)),
                ("dlnchi", C.POINTER(C.c_double)), ("P_chi", C.POINTER(C.c_double)),
                ("n_chi_pair", C.c_int32), ("chi_pair_min", C.c_double), ("chi_pair_max", C.c_double),
                ("T", C.POINTER(C.c_double)), ("n_f", C.c_int32),
                ("f_grid", C.POINTER(C.c_double)), ("P_f", C.POINTER(C.c_double)),
                ("g", C.POINTER(C.c_double))]


_DP = C.POINTER(C.c_double)


class _Species(C.Structure):
    _fields_ = [("x", _DP), ("y", _DP), ("z", _DP), ("ux", _DP), ("uy", _DP), ("uz", _DP),
                ("tau", _DP), ("margin", _DP), ("uid", C.POINTER(C.c_uint64)),
                ("birth", C.POINTER(C.c_int64)), ("family", C.POINTER(C.c_int64)),
                ("count", C.c_int64), ("capacity", C.c_int64)]


class _Ledger(C.Structure):
    _fields_ = [("energy0", C.c_double * 3), ("energy", C.c_double * 3), ("count", C.c_int64 * 3),
                ("work", C.c_double), ("defect_emit", C.c_double), ("defect_pair", C.c_double),
                ("n_emit", C.c_int64), ("n_null", C.c_int64), ("n_pair", C.c_int64),
                ("n_range", C.c_int64), ("n_nonfinite", C.c_int64), ("particle_steps", C.c_int64),
                ("radiated", C.c_double)]


def lib():
    """Load oracle/liboracle.so, compiling it first if it has not been built."""
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        for name in ("oracle_bessel_k", "oracle_bessel_k_tail"):
            getattr(L, name).argtypes = [C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        for name in ("oracle_F", "oracle_energy_below", "oracle_cutoff_chi", "oracle_pf"):
            getattr(L, name).argtypes = [C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        for name in ("oracle_h", "oracle_g", "oracle_T", "oracle_pair_k", "oracle_cr_exp", "oracle_cr_log",
                     "oracle_cr_sin", "oracle_cr_cos"):
            getattr(L, name).argtypes = [C.c_double]
            getattr(L, name).restype = C.c_double
        for name in ("oracle_number_cumulative", "oracle_pf_cumulative"):
            getattr(L, name).argtypes = [C.c_double, _DP, C.c_int, _DP]
            getattr(L, name).restype = None
        L.oracle_philox.argtypes = [C.POINTER(C.c_uint64)] * 3
        L.oracle_philox.restype = None
        L.oracle_gauss_legendre.argtypes = [C.c_int, _DP, _DP]
        L.oracle_build_tables.argtypes = [C.POINTER(_TableParams)] + [_DP] * 9
        L.oracle_build_tables.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(_Config), C.POINTER(_Tables), C.POINTER(_Species),
                                 C.POINTER(_Species), C.POINTER(_Ledger)]
        L.oracle_fields.argtypes = [C.POINTER(_Config)] + [C.c_double] * 4 + [_DP, _DP]
        L.oracle_fields.restype = None
        L.oracle_grid_gather.argtypes = [C.POINTER(_Config), C.c_int, _DP, C.c_double, C.c_double]
        L.oracle_grid_gather.restype = C.c_double
        for name in ("oracle_eta", "oracle_chi"):
            getattr(L, name).argtypes = [C.POINTER(_Config)] + [C.c_double] * 7
            getattr(L, name).restype = C.c_double
        L.oracle_run.restype = C.c_int
        L.oracle_run_pic.argtypes = [C.POINTER(_Config), C.POINTER(_Tables), C.POINTER(_Species),
                                     C.POINTER(_Species), C.POINTER(_Ledger), _DP]
        L.oracle_run_pic.restype = C.c_int
        L.oracle_deposit.argtypes = [C.POINTER(_Config)] + [C.c_double] * 6 + [_DP]
        L.oracle_deposit.restype = None
        L.oracle_fdtd_step.argtypes = [C.POINTER(_Config), _DP]
        L.oracle_fdtd_step.restype = None
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        _LIB = L
    return _LIB


def _vec(fn, *args):
    b = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64) for a in args])
    out = np.empty(b[0].shape)
    for idx in np.ndindex(out.shape):
        out[idx] = fn(*[float(x[idx]) for x in b])
    return out if out.shape else float(out)


# ---- special functions -------------------------------------------------------
def bessel_k(nu, y):
    return _vec(lib().oracle_bessel_k, nu, y)


def bessel_k_tail(nu, y):
    """int_y^inf K_nu(t) dt"""
    return _vec(lib().oracle_bessel_k_tail, nu, y)


def F(eta, chi):
    """Quantum synchrotron function (Appendix A)."""
    return _vec(lib().oracle_F, eta, chi)


def h(eta):
    return _vec(lib().oracle_h, eta)


def g(eta):
    return _vec(lib().oracle_g, eta)


def energy_below(eta, chi):
    """int_0^chi F(eta, chi') dchi'"""
    return _vec(lib().oracle_energy_below, eta, chi)


def cutoff_chi(eta, frac=1e-9):
    return _vec(lib().oracle_cutoff_chi, eta, frac)


def T(chi):
    """Pair emissivity T_pm(chi) (Appendix B)."""
    return _vec(lib().oracle_T, chi)


def pair_k(chi):
    return _vec(lib().oracle_pair_k, chi)


def pf(f, chi):
    """Normalised pair energy-split density p_f(f, chi) (Appendix B)."""
    return _vec(lib().oracle_pf, f, chi)


def gauss_legendre(n):
    x = np.empty(n)
    w = np.empty(n)
    lib().oracle_gauss_legendre(n, x.ctypes.data_as(_DP), w.ctypes.data_as(_DP))
    return x, w


def philox(counter, key):
    """One Philox4x64-10 block for a 4-word counter and a 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.empty(4, dtype=np.uint64)
    P = C.POINTER(C.c_uint64)
    lib().oracle_philox(c.ctypes.data_as(P), k.ctypes.data_as(P), o.ctypes.data_as(P))
    return o


def number_cumulative(eta, chi):
    """int_0^chi F(eta, chi')/chi' dchi' at ascending chi (Appendix A)."""
    c = np.ascontiguousarray(chi, dtype=np.float64)
    out = np.empty_like(c)
    lib().oracle_number_cumulative(float(eta), c.ctypes.data_as(_DP), len(c), out.ctypes.data_as(_DP))
    return out


def pf_cumulative(chi, f):
    """int_0^f p_f(f', chi) df' at ascending f in [0, 1] (Appendix B, normalised)."""
    a = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(a)
    lib().oracle_pf_cumulative(float(chi), a.ctypes.data_as(_DP), len(a), out.ctypes.data_as(_DP))
    return out


# ---- tables ------------------------------------------------------------------
DEFAULT_TABLE_PARAMS = dict(n_eta=256, eta_min=1e-4, eta_max=1e2, n_chi=256, cutoff_energy_frac=1e-9,
                            n_chi_pair=256, chi_pair_min=1e-2, chi_pair_max=1e2, n_f=256)


def build_tables(**overrides) -> dict:
    """The look-up tables of Sec. 3 (h, T_pm, P_chi, P_f) and g(eta) of Appendix A as numpy arrays."""
    p = dict(DEFAULT_TABLE_PARAMS)
    p.update(overrides)
    tp = _TableParams(**p)
    ne, nc, npair, nf = p["n_eta"], p["n_chi"], p["n_chi_pair"], p["n_f"]
    t = dict(params=p,
             h=np.empty(ne), lnchi_min=np.empty(ne), dlnchi=np.empty(ne), P_chi=np.empty((ne, nc)),
             T=np.empty(npair), f_grid=np.empty(nf), P_f=np.empty((npair, nf)), k_norm=np.empty(npair),
             g=np.empty(ne))
    rc = lib().oracle_build_tables(C.byref(tp), *[t[k].ctypes.data_as(_DP) for k in
                                                  ("h", "lnchi_min", "dlnchi", "P_chi", "T", "f_grid",
                                                   "P_f", "k_norm", "g")])
    if rc != 0:
        raise ValueError("oracle_build_tables rejected its parameters")
    return t


# ---- Monte-Carlo run -----------------------------------------------------------
@dataclass
class RunConfig:
    field_kind: int
    field: tuple
    dt: float
    n_steps: int
    t0: float = 0.0
    step0: int = 0
    seed: int = 1
    instance: int = 0
    flags: int = FLAG_EMIT | FLAG_PAIRS | FLAG_PROPAGATE
    dims: int = 3
    draw_initial_tau: bool = True
    lambda_L: float = 1e-6
    grid: tuple = (0, 0, 0.0, 0.0, 0.0, 0.0)  # nx, ny, dx, dy, x0, y0


def _species_in(d):
    if d is None:
        return _Species(count=0, capacity=0), []
    keep = []

    def arr(name, dtype=np.float64):
        a = d.get(name)
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a

    n = len(d["uid"])
    s = _Species(count=n, capacity=n)
    for name in ("x", "y", "z", "ux", "uy", "uz", "tau"):
        a = arr(name)
        if a is not None:
            setattr(s, name, a.ctypes.data_as(_DP))
    u = arr("uid", np.uint64)
    s.uid = u.ctypes.data_as(C.POINTER(C.c_uint64))
    b = arr("birth_step", np.int64)
    if b is not None:
        s.birth = b.ctypes.data_as(C.POINTER(C.c_int64))
    return s, keep


def _config(cfg: RunConfig) -> _Config:
    conf = _Config()
    conf.field_kind = cfg.field_kind
    fp = list(cfg.field) + [0.0] * (16 - len(cfg.field))
    conf.field = (C.c_double * 16)(*fp)
    conf.grid_nx, conf.grid_ny, conf.grid_dx, conf.grid_dy, conf.grid_x0, conf.grid_y0 = cfg.grid
    conf.dims = cfg.dims
    conf.dt = cfg.dt
    conf.t0 = cfg.t0
    conf.step0 = cfg.step0
    conf.n_steps = cfg.n_steps
    conf.seed = cfg.seed
    conf.instance = cfg.instance
    conf.flags = cfg.flags
    conf.draw_initial_tau = 1 if cfg.draw_initial_tau else 0
    conf.lambda_L = cfg.lambda_L
    return conf


def fields(cfg: RunConfig, x, y, z, t):
    """E and B (code units) that the step of `cfg` sees at the points (x, y, z) and times t
    (broadcast); arrays of shape (..., 3)."""
    conf = _config(cfg)
    b = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64) for a in (x, y, z, t)])
    E = np.empty(b[0].shape + (3,))
    B = np.empty(b[0].shape + (3,))
    e3, b3 = np.empty(3), np.empty(3)
    for idx in np.ndindex(b[0].shape):
        lib().oracle_fields(C.byref(conf), *[float(a[idx]) for a in b], e3.ctypes.data_as(_DP),
                            b3.ctypes.data_as(_DP))
        E[idx] = e3
        B[idx] = b3
    return E, B


def grid_gather(cfg: RunConfig, comp: int, nodes, x, y):
    """First-order gather of component `comp` (0..5: Ex, Ey, Ez, Bx, By, Bz) of the grid of `cfg`
    from the node values `nodes` (ny x nx, that component's staggered grid) at (x, y)."""
    conf = _config(cfg)
    n = np.ascontiguousarray(nodes, dtype=np.float64)
    assert n.shape == (cfg.grid[1], cfg.grid[0])
    return _vec(lambda a, b: lib().oracle_grid_gather(C.byref(conf), int(comp), n.ctypes.data_as(_DP), a, b), x, y)


def eta(cfg: RunConfig, x, y, z, t, ux, uy, uz):
    """eta of a lepton with momentum u at (x, y, z, t) in the fields of `cfg` (eq. 1)."""
    conf = _config(cfg)
    return _vec(lambda *a: lib().oracle_eta(C.byref(conf), *a), x, y, z, t, ux, uy, uz)


def chi(cfg: RunConfig, x, y, z, t, kx, ky, kz):
    """chi of a photon with momentum k at (x, y, z, t) in the fields of `cfg` (eq. 1)."""
    conf = _config(cfg)
    return _vec(lambda *a: lib().oracle_chi(C.byref(conf), *a), x, y, z, t, kx, ky, kz)


def deposit(cfg: RunConfig, Q, x0, y0, x1, y1, vz, J=None):
    """The current planes (3, ny, nx: Jx, Jy, Jz) of one macro-particle of charge Q moving in one
    step of cfg.dt from (x0, y0) to (x1, y1) with z velocity vz, added to J (zeros if None)."""
    conf = _config(cfg)
    nx, ny = cfg.grid[0], cfg.grid[1]
    out = np.zeros((3, ny, nx)) if J is None else np.ascontiguousarray(J, dtype=np.float64).copy()
    lib().oracle_deposit(C.byref(conf), float(Q), float(x0), float(y0), float(x1), float(y1), float(vz),
                         out.ctypes.data_as(_DP))
    return out


def fdtd_step(cfg: RunConfig, F):
    """One step of the Yee solver on the nine planes F (9, ny, nx: Ex Ey Ez Bx By Bz Jx Jy Jz);
    returns the advanced planes (the current planes unchanged)."""
    conf = _config(cfg)
    out = np.ascontiguousarray(F, dtype=np.float64).copy()
    assert out.shape == (9, cfg.grid[1], cfg.grid[0])
    lib().oracle_fdtd_step(C.byref(conf), out.ctypes.data_as(_DP))
    return out


def run(cfg: RunConfig, tables: dict, electrons=None, positrons=None, photons=None, capacity=None, fields=None):
    """Advance every family rooted at the given particles; return (species dict, ledger dict).

    With ``cfg.field_kind == FIELD_GRID_FDTD`` the run couples the particles to the grid
    (field feedback): ``fields`` holds the nine planes (9, ny, nx) at the start, and the planes
    at the end are returned in the ledger as ``fields``.

    Each species input is a dict of arrays x, y, z, ux, uy, uz, uid (and tau when
    ``cfg.draw_initial_tau`` is False; photons may carry ``birth_step``).  Outputs hold
    the live particles of each species, family by family; photons report the position
    where they were born and ``birth_step``, the step at whose start they sat there
    (their position at the start of step n is x + (n - birth_step) dt k/|k|).  Also
    ``margin``: the smallest |tau| a particle
    showed after a decrement (small values flag threshold straddles), and ``family``:
    the index, in input order, of the particle the family grew from.
    """
    L = lib()
    p = tables["params"]
    tab = _Tables(n_eta=p["n_eta"], eta_min=p["eta_min"], eta_max=p["eta_max"],
                  h=tables["h"].ctypes.data_as(_DP), n_chi=p["n_chi"],
                  lnchi_min=tables["lnchi_min"].ctypes.data_as(_DP),
                  dlnchi=tables["dlnchi"].ctypes.data_as(_DP),
                  P_chi=tables["P_chi"].ctypes.data_as(_DP), n_chi_pair=p["n_chi_pair"],
                  chi_pair_min=p["chi_pair_min"], chi_pair_max=p["chi_pair_max"],
                  T=tables["T"].ctypes.data_as(_DP), n_f=p["n_f"],
                  f_grid=tables["f_grid"].ctypes.data_as(_DP), P_f=tables["P_f"].ctypes.data_as(_DP))
    g_arr = None
    if tables.get("g") is not None:
        g_arr = np.ascontiguousarray(tables["g"], dtype=np.float64)  # held for the call
        tab.g = g_arr.ctypes.data_as(_DP)
    conf = _config(cfg)

    ins = (_Species * 3)()
    keep = []
    for i, d in enumerate((electrons, positrons, photons)):
        s, k = _species_in(d)
        ins[i] = s
        keep += k
    n_in = sum(int(ins[i].count) for i in range(3))
    cap = capacity if capacity is not None else [max(16, 4 * n_in)] * 3

    for attempt in range(2):
        outs = (_Species * 3)()
        bufs = []
        for i in range(3):
            b = {k: np.empty(cap[i]) for k in ("x", "y", "z", "ux", "uy", "uz", "tau", "margin")}
            b["uid"] = np.empty(cap[i], dtype=np.uint64)
            b["family"] = np.empty(cap[i], dtype=np.int64)
            b["birth_step"] = np.empty(cap[i], dtype=np.int64)
            bufs.append(b)
            o = _Species(count=0, capacity=cap[i])
            for k in ("x", "y", "z", "ux", "uy", "uz", "tau", "margin"):
                setattr(o, k, b[k].ctypes.data_as(_DP))
            o.uid = b["uid"].ctypes.data_as(C.POINTER(C.c_uint64))
            o.family = b["family"].ctypes.data_as(C.POINTER(C.c_int64))
            o.birth = b["birth_step"].ctypes.data_as(C.POINTER(C.c_int64))
            outs[i] = o
        led = _Ledger()
        if cfg.field_kind == FIELD_GRID_FDTD:
            F = np.ascontiguousarray(fields, dtype=np.float64).copy()  # a fresh copy for each attempt
            assert F.shape == (9, cfg.grid[1], cfg.grid[0])
            rc = L.oracle_run_pic(C.byref(conf), C.byref(tab), ins, outs, C.byref(led), F.ctypes.data_as(_DP))
        else:
            rc = L.oracle_run(C.byref(conf), C.byref(tab), ins, outs, C.byref(led))
        if rc == 0:
            break
        if rc == -2:
            raise ValueError("oracle_run: inconsistent flags (radiation reaction without its table, or "
                             "field feedback outside 2-D or with radiation reaction)")
        # outputs did not fit: retry with the sizes the oracle reported (same result, deterministic)
        cap = [int(outs[i].count) + 1 for i in range(3)]
    else:
        raise RuntimeError("oracle output sizing failed")

    res = {}
    for i, name in enumerate(SPECIES):
        n = int(outs[i].count)
        res[name] = {k: v[:n].copy() for k, v in bufs[i].items()}
        if cfg.dims == 2:
            res[name].pop("z")
    ledger = dict(energy0=list(led.energy0), energy=list(led.energy), count=list(led.count),
                  work=led.work, defect_emit=led.defect_emit, defect_pair=led.defect_pair,
                  radiated=led.radiated,
                  n_emit=led.n_emit, n_null=led.n_null, n_pair=led.n_pair, n_range=led.n_range,
                  n_nonfinite=led.n_nonfinite, particle_steps=led.particle_steps)
    if cfg.field_kind == FIELD_GRID_FDTD:
        ledger["fields"] = F
    return res, ledger


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the following oracle runs (results do not depend on it)."""
    lib().oracle_set_threads(int(n))
