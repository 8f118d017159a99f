"""The HIP path against the paper's own ensemble results (Sec. 4, Table 2): the uniform-B test
problems 1 and 3 run through the C ABI with GPU-built tables, at the paper's electron count
for test 3 and a tenth of it for test 1; energy per initial electron in electrons, photons
and positrons against Table 2, and the ledger closing on the per-event defects.  Then the
electron and photon spectra of test 1 against the direct solution of the kinetic equations
(eqs. 6-7), as the paper checks its own Monte-Carlo (Figs. 2-4)."""
import os

import numpy as np
import pytest

from paper_1311_5551_amd import workloads as W
from paper_1311_5551_amd.sim import Run, Tables

from parity import record

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def table2():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "table2_energy.txt")):
        if line.startswith("#") or not line.strip():
            continue
        test, comp, _, end = line.split()
        rows[(int(test), comp)] = float(end)
    return rows


@pytest.fixture(scope="module")
def gpu_tables():
    return Tables.build()


@pytest.mark.parametrize("test,n,tol", [(1, 1_000_000, 0.03), (3, 1_000_000, 0.04)])
def test_table2_energy_partition_on_gpu(test, n, tol, gpu_tables):
    # dt = 0.3 Delta t_QED (the paper's dt is not stated; its Fig. 6 puts the dt error there at ~3%)
    ref = table2()
    w = W.paper_test(test, n, 0.3)
    r = Run(w, gpu_tables)
    r.step(w.n_steps)
    led = r.ledger()[0]
    assert led["status"] == "QED_OK"
    e = [v / n for v in led["energy"]]
    assert e[0] == pytest.approx(ref[(test, "electron")], rel=tol)
    assert e[2] == pytest.approx(ref[(test, "photon")], rel=tol)
    if test == 1:
        assert 0.2 < e[1] < 0.7                       # paper 0.4, from ~1e-3 pairs per electron
        assert 0 < (led["defect_emit"] + led["defect_pair"]) / n < 0.01   # paper 0.001
    else:
        assert e[1] == pytest.approx(ref[(test, "positron")], rel=0.1)
        assert 0 < (led["defect_emit"] + led["defect_pair"]) / n < 0.05   # paper 0.006
    # no field work in a static B: the books close on the defects alone
    assert led["drift"] < 1e-12
    assert abs(led["work"]) < 1e-9 * led["energy0"]


def _coarse_bins(edges, lo, per_bin=6):
    """Coarse bins made of whole solver cells: every per_bin-th cell edge from the first at or above lo."""
    first = int(np.searchsorted(edges, lo))
    b = edges[first::per_bin]
    return b if b[-1] == edges[-1] else np.append(b, edges[-1])


def _coarse(edges, fine, bins):
    """The solver's cell contents summed over the coarse bins (bins are cell edges)."""
    i = np.searchsorted(edges, bins)
    return np.array([fine[i[k]:i[k + 1]].sum() for k in range(len(bins) - 1)])


@pytest.mark.parametrize("test,b,t_fs", [(1, 1e-3, 1.0), (3, 9e-3, 0.1)])
def test_spectra_match_master_equation_on_gpu(test, b, t_fs, gpu_tables):
    # paper tests 1 and 3 with pairs at dt = 0.05 Delta t_QED, 1e6 electrons through the C ABI:
    # the electron, photon (and for test 3 positron) spectra at t0 against the direct solution of
    # eqs. 6-7 (Figs. 2 and 4)
    from oracle import master as M
    n = 1_000_000
    w = W.paper_test(test, n, 0.05)
    w.capacity = dict(electron=n + 400_000, positron=400_000, photon=16 * n)
    r = Run(w, gpu_tables)
    r.step(w.n_steps)
    led = r.ledger()[0]
    assert led["status"] == "QED_OK"
    s = M.solve(b, 1000.0, W.fs_to_code(t_fs), cells_per_e=20, pairs=True)
    e = r.species(0, "electron")
    pos = r.species(0, "positron")
    ph = r.species(0, "photon")
    energy = lambda d: np.sqrt(1.0 + d["ux"] ** 2 + d["uy"] ** 2 + d["uz"] ** 2)
    eps = np.sqrt(ph["ux"] ** 2 + ph["uy"] ** 2 + ph["uz"] ** 2)
    cases = [("electron", energy(e), s.electron, 30.0), ("photon", eps, s.photon, 3.0)]
    if test == 3:
        cases.append(("positron", energy(pos), s.positron, 3.0))
    rec = {}
    for name, vals, fine, lo in cases:
        bins = _coarse_bins(s.edges, lo)
        mc = np.histogram(vals, bins=bins)[0] / n
        me = _coarse(s.edges, fine, bins)
        sig = np.sqrt(np.maximum(me, 1e-12) / n)
        # bins holding >= 1e-4 of the particles (the far tail is the scheme's numerical diffusion)
        dev = np.where(me >= 1e-4, np.abs(mc - me) / (4.0 * sig + 0.05 * me), 0.0)
        rec[name] = {"mc": mc.tolist(), "master": me.tolist(), "worst": float(dev.max())}
        assert dev.max() < 1.0, (name, mc, me)
    record("spectra_vs_master_test%d" % test, rec)
    # and the energies: the direct solution is the dt -> 0 limit, the run has dt = 0.05 Delta t_QED
    assert led["energy"][0] / n == pytest.approx(s.energy("electron"), rel=0.015)
    assert led["energy"][2] / n == pytest.approx(s.energy("photon"), rel=0.015)
    if test == 3:
        assert led["energy"][1] / n == pytest.approx(s.energy("positron"), rel=0.03)
