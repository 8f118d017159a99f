"""The HIP path against the paper's own ensemble results (Sec. 4, Table 2): the uniform-B test
problems 1 and 3 run through the C ABI with GPU-built tables, at the paper's electron count
for test 3 and a tenth of it for test 1; energy per initial electron in electrons, photons
and positrons against Table 2, and the ledger closing on the per-event defects."""
import os

import pytest

from paper_1311_5551_amd import workloads as W
from paper_1311_5551_amd.sim import Run, Tables

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
