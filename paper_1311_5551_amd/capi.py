"""Thin ctypes binding of libqed (include/qed.h): structures and functions with the
same names as the C ABI.  Argument marshalling only; all computation runs in the
library's HIP kernels.  Importing this module loads paper_1311_5551_amd/libqed.so
and fails loudly if it has not been built."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqed.so")

QED_OK, QED_ERR_ARG, QED_ERR_HIP, QED_ERR_CAPACITY, QED_ERR_NONFINITE, QED_ERR_STATE, QED_ERR_DEVICE = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "QED_OK", -1: "QED_ERR_ARG", -2: "QED_ERR_HIP", -3: "QED_ERR_CAPACITY",
                -4: "QED_ERR_NONFINITE", -5: "QED_ERR_STATE", -6: "QED_ERR_DEVICE"}
QED_FP64, QED_FP32_MIXED = 0, 1
QED_EMIT, QED_PAIRS, QED_PROPAGATE = 1, 2, 4
QED_RR_QUANTUM, QED_RR_CLASSICAL = 8, 16
QED_PROFILE_CLASSES = 6
QED_KERNEL_LEPTON, QED_KERNEL_PHOTON = 1, 2
QED_FIELD_UNIFORM, QED_FIELD_LP_PULSE, QED_FIELD_CP_WAVE, QED_FIELD_CP_STANDING, QED_FIELD_GRID_CP_STANDING = \
    0, 1, 2, 3, 4
QED_FIELD_GRID_FDTD = 5

_vp = C.c_void_p
_DP = C.POINTER(C.c_double)


class qed_table_params(C.Structure):
    _fields_ = [("n_eta", C.c_int32), ("eta_min", C.c_double), ("eta_max", C.c_double),
                ("n_chi", C.c_int32), ("cutoff_energy_frac", C.c_double),
                ("n_chi_pair", C.c_int32), ("chi_pair_min", C.c_double), ("chi_pair_max", C.c_double),
                ("n_f", C.c_int32)]


class qed_table_view(C.Structure):
    _fields_ = [("params", qed_table_params), ("h", _DP), ("lnchi_min", _DP), ("dlnchi", _DP), ("P_chi", _DP),
                ("T", _DP), ("f_grid", _DP), ("P_f", _DP), ("k_norm", _DP), ("g", _DP)]


class qed_species(C.Structure):
    _fields_ = [("x_dev", _vp), ("y_dev", _vp), ("z_dev", _vp), ("ux_dev", _vp), ("uy_dev", _vp), ("uz_dev", _vp),
                ("x_lo_dev", _vp), ("y_lo_dev", _vp), ("z_lo_dev", _vp),
                ("ux_lo_dev", _vp), ("uy_lo_dev", _vp), ("uz_lo_dev", _vp),
                ("birth_step_dev", _vp), ("tau_dev", _vp), ("uid_dev", _vp), ("count_dev", _vp),
                ("capacity", C.c_int64)]


class qed_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_double * 16), ("grid_dev", _vp), ("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("x0", C.c_double), ("y0", C.c_double), ("fdtd_dev", _vp)]


class qed_instance(C.Structure):
    _fields_ = [("s", qed_species * 3), ("field", qed_field), ("weight", C.c_double), ("seed", C.c_uint64),
                ("key_instance", C.c_uint64), ("dims", C.c_int32)]


class qed_step_params(C.Structure):
    _fields_ = [("t0", C.c_double), ("dt", C.c_double), ("lambda_L", C.c_double), ("flags", C.c_uint32),
                ("precision", C.c_int32)]


class qed_ledger(C.Structure):
    _fields_ = [("energy", C.c_double * 3), ("energy0", C.c_double), ("work", C.c_double),
                ("defect_emit", C.c_double), ("defect_pair", C.c_double), ("dropped_energy", C.c_double),
                ("radiated", C.c_double), ("retired_energy", C.c_double), ("n_retired", C.c_int64),
                ("count", C.c_int64 * 3), ("n_emit", C.c_int64), ("n_null", C.c_int64), ("n_pair", C.c_int64),
                ("n_dropped", C.c_int64), ("n_range", C.c_int64), ("n_nonfinite", C.c_int64),
                ("photon_steps_in_field", C.c_int64), ("photon_steps_active", C.c_int64),
                ("lepton_steps_in_field", C.c_int64), ("photon_window_reads", C.c_int64),
                ("photon_group_reads", C.c_int64),
                ("particle_steps", C.c_int64 * 3), ("drift", C.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["energy"] = list(self.energy)
        d["count"] = list(self.count)
        d["particle_steps"] = list(self.particle_steps)
        return d


# name -> (restype, argtypes)
_SIGNATURES = {
    "qed_build_tables": (C.c_int, [C.POINTER(qed_table_params), C.POINTER(_vp)]),
    "qed_tables_from_host": (C.c_int, [C.POINTER(qed_table_params)] + [_DP] * 9 + [C.POINTER(_vp)]),
    "qed_tables_view": (C.c_int, [_vp, C.POINTER(qed_table_view)]),
    "qed_tables_destroy": (None, [_vp]),
    "qed_workspace_create": (C.c_int, [C.c_int32, C.POINTER(_vp)]),
    "qed_workspace_destroy": (None, [_vp]),
    "qed_bind": (C.c_int, [_vp, C.POINTER(qed_instance), C.c_int32, C.POINTER(qed_step_params)]),
    "qed_set_launch": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "qed_set_event_queue": (C.c_int, [_vp, C.c_int64]),
    "qed_set_kernel_launch": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32]),
    "qed_init_optical_depth": (C.c_int, [_vp, _vp]),
    "qed_set_step": (C.c_int, [_vp, C.c_int64, _vp]),
    "qed_step": (C.c_int, [_vp, _vp, C.POINTER(qed_step_params), _vp]),
    "qed_run": (C.c_int, [_vp, _vp, C.POINTER(qed_step_params), C.c_int64, C.c_int32, _vp]),
    "qed_compact": (C.c_int, [_vp, _vp]),
    "qed_sort": (C.c_int, [_vp, C.POINTER(qed_step_params), _vp]),
    "qed_sort_static": (C.c_int, [_vp, C.POINTER(qed_step_params), _vp]),
    "qed_energy_ledger": (C.c_int, [_vp, C.POINTER(qed_ledger), _vp]),
    "qed_set_retire": (C.c_int, [_vp, C.c_int32, C.c_double, C.c_double]),
    "qed_retired_spectrum": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int64), _vp]),
    "qed_profile": (C.c_int, [_vp, C.c_int32]),
    "qed_profile_read": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "qed_last_error": (C.c_char_p, []),
    "qed_version": (C.c_char_p, []),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libqed.so is not built (%s); run paper_1311_5551_amd/build.py" % LIB_PATH)
        # torch ships its own HIP runtime with the same soname as the system one; loading torch
        # first makes libqed bind to that copy, so the process holds a single HIP runtime
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class QEDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status, allow=()):
    if status != QED_OK and status not in allow:
        raise QEDError(status, lib().qed_last_error().decode())
    return status


# --- functions with the C names ---------------------------------------------
def qed_build_tables(params: qed_table_params):
    h = _vp()
    check(lib().qed_build_tables(C.byref(params), C.byref(h)))
    return h


def qed_tables_from_host(params, h, lnchi_min, dlnchi, P_chi, T, f_grid, P_f, k_norm=None, g=None):
    out = _vp()
    arrs = [h, lnchi_min, dlnchi, P_chi, T, f_grid, P_f]
    ptrs = [a.ctypes.data_as(_DP) for a in arrs] + [a.ctypes.data_as(_DP) if a is not None else None
                                                    for a in (k_norm, g)]
    check(lib().qed_tables_from_host(C.byref(params), *ptrs, C.byref(out)))
    return out


def qed_tables_view(tables) -> qed_table_view:
    v = qed_table_view()
    check(lib().qed_tables_view(tables, C.byref(v)))
    return v


def qed_tables_destroy(tables):
    lib().qed_tables_destroy(tables)


def qed_workspace_create(max_inst: int):
    ws = _vp()
    check(lib().qed_workspace_create(max_inst, C.byref(ws)))
    return ws


def qed_workspace_destroy(ws):
    lib().qed_workspace_destroy(ws)


def qed_bind(ws, insts, params: qed_step_params):
    arr = (qed_instance * len(insts))(*insts)
    return check(lib().qed_bind(ws, arr, len(insts), C.byref(params)))


def qed_set_launch(ws, block: int, ppt: int):
    return check(lib().qed_set_launch(ws, block, ppt))


def qed_set_kernel_launch(ws, kernel: int, block: int, ppt: int):
    return check(lib().qed_set_kernel_launch(ws, kernel, block, ppt))


def qed_set_event_queue(ws, capacity: int):
    return check(lib().qed_set_event_queue(ws, capacity))


def qed_init_optical_depth(ws, stream=None):
    return check(lib().qed_init_optical_depth(ws, stream))


def qed_set_step(ws, step: int, stream=None):
    return check(lib().qed_set_step(ws, step, stream))


def qed_step(tables, ws, params: qed_step_params, stream=None):
    return check(lib().qed_step(tables, ws, C.byref(params), stream))


def qed_run(tables, ws, params: qed_step_params, n_steps: int, graph_steps: int = 0, stream=None):
    return check(lib().qed_run(tables, ws, C.byref(params), n_steps, graph_steps, stream))


def qed_sort(ws, params: qed_step_params, stream=None):
    return check(lib().qed_sort(ws, C.byref(params), stream))


def qed_sort_static(ws, params: qed_step_params, stream=None):
    return check(lib().qed_sort_static(ws, C.byref(params), stream))


def qed_set_retire(ws, n_bins: int, eps_min: float, eps_max: float):
    return check(lib().qed_set_retire(ws, n_bins, eps_min, eps_max))


def qed_retired_spectrum(ws, inst: int, n_bins: int, stream=None):
    out = (C.c_int64 * (n_bins + 2))()
    check(lib().qed_retired_spectrum(ws, inst, out, stream))
    return list(out)


def qed_compact(ws, stream=None):
    return check(lib().qed_compact(ws, stream))


def qed_energy_ledger(ws, n_inst: int, stream=None, allow=(QED_ERR_CAPACITY, QED_ERR_NONFINITE)):
    out = (qed_ledger * n_inst)()
    st = check(lib().qed_energy_ledger(ws, out, stream), allow=allow)
    return st, [o.as_dict() for o in out]


def qed_profile(ws, enable: bool):
    return check(lib().qed_profile(ws, 1 if enable else 0))


def qed_profile_read(ws):
    ms = (C.c_double * QED_PROFILE_CLASSES)()
    n = (C.c_int64 * QED_PROFILE_CLASSES)()
    check(lib().qed_profile_read(ws, ms, n))
    return list(ms), list(n)


def qed_version() -> str:
    return lib().qed_version().decode()
