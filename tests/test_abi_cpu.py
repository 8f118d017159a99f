"""CPU checks of the C ABI: the library loads, exports every function include/qed.h
declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qed.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qed_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1311_5551_amd import capi
    return capi.lib()


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("qed_build_tables", "qed_step", "qed_compact", "qed_energy_ledger"):
        assert n in names


def test_every_declared_function_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_arguments_rejected_before_any_device_work(lib):
    from paper_1311_5551_amd import capi
    out = C.c_void_p()
    assert lib.qed_build_tables(None, C.byref(out)) == capi.QED_ERR_ARG
    assert b"NULL" in lib.qed_last_error()
    bad = capi.qed_table_params(n_eta=1, eta_min=1e-4, eta_max=1e2, n_chi=16, cutoff_energy_frac=1e-9,
                                n_chi_pair=16, chi_pair_min=1e-2, chi_pair_max=1e2, n_f=16)
    assert lib.qed_build_tables(C.byref(bad), C.byref(out)) == capi.QED_ERR_ARG
    bad = capi.qed_table_params(n_eta=16, eta_min=1e2, eta_max=1e-4, n_chi=16, cutoff_energy_frac=1e-9,
                                n_chi_pair=16, chi_pair_min=1e-2, chi_pair_max=1e2, n_f=16)
    assert lib.qed_build_tables(C.byref(bad), C.byref(out)) == capi.QED_ERR_ARG
    assert lib.qed_workspace_create(0, C.byref(out)) == capi.QED_ERR_ARG
    assert lib.qed_set_launch(None, 256, 4) == capi.QED_ERR_ARG
    assert lib.qed_set_event_queue(None, 1024) == capi.QED_ERR_ARG
    assert lib.qed_set_kernel_launch(None, capi.QED_KERNEL_PHOTON, 256, 4) == capi.QED_ERR_ARG
    assert lib.qed_step(None, None, None, None) == capi.QED_ERR_ARG
    assert lib.qed_compact(None, None) == capi.QED_ERR_ARG
    assert lib.qed_energy_ledger(None, None, None) == capi.QED_ERR_ARG
    assert lib.qed_bind(None, None, 0, None) == capi.QED_ERR_ARG
    assert b"gfx950" in lib.qed_version()


def test_struct_layouts_match_the_header(tmp_path):
    # compile the header with the host C compiler and compare sizes and field offsets with the
    # ctypes mirrors used by the Python binding
    from paper_1311_5551_amd import capi
    structs = {"qed_table_params": capi.qed_table_params, "qed_table_view": capi.qed_table_view,
               "qed_species": capi.qed_species, "qed_field": capi.qed_field,
               "qed_instance": capi.qed_instance, "qed_step_params": capi.qed_step_params,
               "qed_ledger": capi.qed_ledger}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qed.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(cls, f).offset, (name, f)
