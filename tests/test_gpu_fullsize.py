"""Per-uid parity at the full sizes of the collision and grid workloads, run the way the bench
runs them, against the oracle on a subset of the particle families.

Every particle's random stream is keyed by its uid and the step (Sec. 3 with Philox4x64-10), so
the families grown from a subset of the initial electrons are the same in the full run as in an
oracle run of that subset alone.  Every particle of the oracle's families must exist in the full
GPU run with the same state (the strict FP64 bars of the parity tests); a family in which the two
sides took different decisions shows up as a missing uid or a different state.  The full runs
reach the paths small runs never take: photon chunk lists far above 8192 chunks (the sweep's
multi-run deal), lepton sweeps whose blocks take several chunks, the partition and the live masks
over ~1e8 photon slots, graph replay with compaction, and the grid sort."""
import numpy as np
import pytest

import oracle
from paper_1311_5551_amd import capi, workloads as W
from paper_1311_5551_amd.sim import Run, Tables

from parity import E_TOL, STRADDLE, TAU_TOL, U_CAP, U_FRAC, U_TOL, X_TOL, compare_species, record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shared_tables(oracle_tables):
    return Tables.from_arrays(oracle_tables)


def _subset_of_gpu(g, uids):
    """The GPU particles whose uid is among `uids`."""
    keep = np.isin(g["uid"], uids)
    return {k: v[keep] for k, v in g.items()}


def _check_subset(run, o_res, label):
    """Every oracle particle found in the GPU run with the same state (flagged threshold straddles
    excepted)."""
    flagged = set()
    for s in o_res.values():
        flagged |= set(int(f) for f in s["family"][s["margin"] < STRADDLE])
    summary = {"flagged_families": len(flagged)}
    for name in ("electron", "positron", "photon"):
        o = o_res[name]
        g = _subset_of_gpu(run.species(0, name), o["uid"])
        rep = compare_species(g, o, photon=name == "photon")
        fam = o["family"][rep["ib"]]
        ok = np.array([int(f) not in flagged for f in fam], dtype=bool)
        missing_fam = set(int(f) for f in o["family"][np.isin(o["uid"], rep["only_oracle"])])
        ue, ee, xe, te = rep["u_err"], rep["e_err"], rep["x_err"], rep["tau_err"]
        hard = ((ee > E_TOL) | (ue > U_CAP) | (xe > X_TOL) | (te > TAU_TOL)) & ok
        summary[name] = dict(oracle=int(len(o["uid"])), matched=int(len(rep["ia"])),
                             missing_on_gpu=int(len(rep["only_oracle"])), u_err_max=float(ue.max(initial=0.0)),
                             tau_err_max=float(te.max(initial=0.0)), hard_fail=int(hard.sum()),
                             frac_within_u_tol=float(np.mean(ue[ok] <= U_TOL)) if ok.any() else 1.0)
        assert not hard.any(), (name, summary[name])
        assert summary[name]["frac_within_u_tol"] >= U_FRAC, (name, summary[name])
        assert missing_fam <= flagged, (name, sorted(missing_fam - flagged)[:10])
    record("fullsize_" + label, summary)
    return summary


def test_collision_full_size_against_oracle_families(shared_tables, oracle_tables):
    # configuration 2 at its full size, stepped the way the bench steps it: HIP graphs of 100 steps,
    # compaction (and the window partition) every 100 steps, all 20000 steps; the lepton sweep at
    # 256 x 1 (~3900 chunks over 2048 blocks, so blocks take two chunks) and the photon sweep at
    # 256 x 4 (~95 000 chunks at the end)
    n_fam = 1000
    w = W.collision_config2()
    r = Run(w, shared_tables)
    r.set_kernel_launch(capi.QED_KERNEL_LEPTON, 256, 1)
    r.set_kernel_launch(capi.QED_KERNEL_PHOTON, 256, 4)
    for _ in range(w.n_steps // 100):
        r.run(100, graph_steps=100)
        r.compact()
    led = r.ledger()[0]
    print("[fullsize] collision: GPU run done, %d photons" % led["count"][2], flush=True)
    assert led["status"] == "QED_OK"
    assert led["count"][2] > 8192 * 1024 and led["n_pair"] > 0
    assert led["drift"] < 1e-12
    sub = W.subset(w, range(n_fam))
    cfg = oracle.RunConfig(field_kind=sub.field_kind, field=sub.field, dt=sub.dt, n_steps=sub.n_steps,
                           flags=sub.flags, seed=sub.seed, instance=sub.instance)
    o_res, o_led = oracle.run(cfg, oracle_tables, electrons=sub.electrons, capacity=[4 * n_fam, 2 * n_fam, 200 * n_fam])
    print("[fullsize] collision: oracle done", flush=True)
    assert o_led["n_emit"] > 50 * n_fam
    s = _check_subset(r, o_res, "collision_1e6")
    assert s["photon"]["matched"] > 0.99 * s["photon"]["oracle"]


def test_grid_full_size_against_oracle_families(shared_tables, oracle_tables):
    # configuration 3 at its full size: 1.6e7 electrons on the 4096 x 2048 Yee grid, sorted by tile
    # every 10 steps as the bench does, for the 91 steps to four times the population; the oracle
    # evaluates the grid nodes on demand for the first 2000 electrons' families
    n_fam = 2000
    w = W.grid_config3()
    n = w.n
    w.capacity = dict(electron=int(1.2 * n) + 4096, positron=n // 50 + 4096, photon=int(3.5 * n) + 4096)
    w.n_steps = 91
    r = Run(w, shared_tables)
    for k in range(w.n_steps):
        if k % 10 == 0:
            r.sort()
        r.step(1)
    led = r.ledger()[0]
    assert led["status"] == "QED_OK"
    assert sum(led["count"]) > 3.5 * n
    sub = W.subset(w, range(n_fam))
    cfg = oracle.RunConfig(field_kind=sub.field_kind, field=sub.field, dt=sub.dt, n_steps=sub.n_steps,
                           flags=sub.flags, seed=sub.seed, instance=sub.instance, dims=2, grid=sub.grid)
    o_res, o_led = oracle.run(cfg, oracle_tables, electrons=sub.electrons)
    assert o_led["n_emit"] > n_fam
    _check_subset(r, o_res, "grid_1.6e7")
