"""GPU tests of the library's mechanics around the step: edge cases (empty and ragged
species, full buffers, non-finite state, eta above the table), argument checking,
compaction, HIP-graph replay, batched instances, restarts and the FP32-mixed form."""
import math

import numpy as np
import pytest

import oracle
from paper_1311_5551_amd import autotune, capi, workloads as W
from paper_1311_5551_amd.sim import Run, Tables

from parity import compare_species, oracle_run, record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shared_tables(oracle_tables):
    return Tables.from_arrays(oracle_tables)


def _states_equal(ra, rb, ia=0, ib=0, species=("electron", "positron", "photon")):
    """Bitwise equality of two runs' particles, matched by uid."""
    for name in species:
        a, b = ra.species(ia, name), rb.species(ib, name)
        assert len(a["uid"]) == len(b["uid"]), name
        oa, ob = np.argsort(a["uid"]), np.argsort(b["uid"])
        for k in a:
            np.testing.assert_array_equal(a[k][oa], b[k][ob], err_msg="%s.%s" % (name, k))


@pytest.mark.parametrize("n,ppt", [(0, 4), (1, 1), (63, 2), (65, 8), (257, 4), (1025, 8)])
def test_empty_and_ragged_counts(n, ppt, shared_tables, oracle_tables):
    w = W.uniform_b(n, 1000.0, 1e-3, 0.15, 40, W.FLAG_EMIT)
    r = Run(w, shared_tables, ppt=ppt)
    r.step(w.n_steps)
    led = r.ledger()[0]
    assert led["status"] == "QED_OK"
    o_res, o_led = oracle_run(w, oracle_tables)
    assert led["n_emit"] == o_led["n_emit"] and led["count"] == o_led["count"]
    for name in ("electron", "photon"):
        rep = compare_species(r.species(0, name), o_res[name], photon=name == "photon")
        assert rep["matched"] == len(o_res[name]["uid"]) == rep["n_gpu"]
        assert (rep["e_err"] <= 1e-12).all()


def test_capacity_overflow_is_reported_and_accounted(shared_tables, oracle_tables):
    n = 4000
    w = W.uniform_b(n, 1000.0, 1e-3, 0.15, 1, W.FLAG_EMIT)
    o_res, o_led = oracle_run(w, oracle_tables)
    cap = o_led["n_emit"] // 2
    r = Run(w, shared_tables, capacity=dict(photon=cap))
    r.step(1)
    led = r.ledger()[0]
    assert led["status"] == "QED_ERR_CAPACITY"
    assert led["n_dropped"] == o_led["n_emit"] - cap
    assert led["count"][2] == cap
    # the dropped photons' energy is booked, so the ledger still closes
    assert led["drift"] < 1e-12
    assert led["dropped_energy"] > 0


def test_nonfinite_state_is_reported(shared_tables):
    w = W.uniform_b(100, 1000.0, 1e-3, 0.15, 3, W.FLAG_EMIT)
    w.electrons["ux"][7] = float("nan")
    r = Run(w, shared_tables)
    r.step(3)
    led = r.ledger()[0]
    assert led["status"] == "QED_ERR_NONFINITE"
    assert led["n_nonfinite"] >= 1
    e = r.species(0, "electron")
    assert np.isfinite(e["ux"][e["uid"] != 7]).all()


def test_eta_above_table_is_clamped_and_counted(shared_tables, oracle_tables):
    # gamma = 2e5 in B' = 1e-3: eta = 200 > eta_max = 100
    w = W.uniform_b(200, 2e5, 1e-3, 1e-3, 5, W.FLAG_EMIT)
    r = Run(w, shared_tables)
    r.step(5)
    led = r.ledger()[0]
    o_res, o_led = oracle_run(w, oracle_tables)
    assert led["n_range"] == o_led["n_range"] > 0
    rep = compare_species(r.species(0, "electron"), o_res["electron"])
    assert (rep["e_err"] <= 1e-12).all()


def test_invalid_arguments_are_rejected(shared_tables):
    w = W.uniform_b(10, 1000.0, 1e-3, 0.15, 3, W.FLAG_EMIT)
    r = Run(w, shared_tables)
    bad = capi.qed_step_params(t0=0.0, dt=-1.0, lambda_L=1e-6, flags=1, precision=0)
    with pytest.raises(capi.QEDError) as e:
        capi.qed_step(shared_tables.handle, r.ws, bad, r._s())
    assert e.value.status == capi.QED_ERR_ARG
    bad = capi.qed_step_params(t0=0.0, dt=0.1, lambda_L=1e-6, flags=capi.QED_PAIRS, precision=0)
    with pytest.raises(capi.QEDError):
        capi.qed_step(shared_tables.handle, r.ws, bad, r._s())
    bad = capi.qed_step_params(t0=0.0, dt=0.1, lambda_L=1e-6, flags=1, precision=1)
    with pytest.raises(capi.QEDError) as e:
        capi.qed_step(shared_tables.handle, r.ws, bad, r._s())
    assert e.value.status == capi.QED_ERR_STATE
    with pytest.raises(capi.QEDError):
        capi.qed_set_launch(r.ws, 100, 4)
    with pytest.raises(capi.QEDError):
        capi.qed_set_launch(r.ws, 256, 3)
    # a host pointer, and a capacity larger than the allocation, are refused at bind
    inst = capi.qed_instance.from_buffer_copy(r.insts[0])
    host = np.zeros(16)
    inst.s[0].x_dev = host.ctypes.data
    with pytest.raises(capi.QEDError) as e:
        capi.qed_bind(r.ws, [inst], r.params)
    assert e.value.status == capi.QED_ERR_ARG
    inst = capi.qed_instance.from_buffer_copy(r.insts[0])
    inst.s[2].capacity = inst.s[2].capacity * 1000 + 10 ** 8
    with pytest.raises(capi.QEDError) as e:
        capi.qed_bind(r.ws, [inst], r.params)
    assert e.value.status == capi.QED_ERR_ARG
    tp = capi.qed_table_params(n_eta=1, eta_min=1e-4, eta_max=1e2, n_chi=16, cutoff_energy_frac=1e-9,
                               n_chi_pair=16, chi_pair_min=1e-2, chi_pair_max=1e2, n_f=16)
    with pytest.raises(capi.QEDError):
        capi.qed_build_tables(tp)


def _collision_run(tables, n=3000, steps=2600, seed=21, **kw):
    w = W.collision(n, n_steps=steps, meet_step=steps // 2, seed=seed)
    return w, Run(w, tables, **kw)


def test_compaction_preserves_live_photons(shared_tables):
    w, ra = _collision_run(shared_tables)
    _, rb = _collision_run(shared_tables)
    ra.step(1800)
    rb.step(1800)
    before = ra.species(0, "photon", live_only=True)
    n_slots = ra.count(0, "photon")
    ra.compact()
    after = ra.species(0, "photon", live_only=False)
    assert (after["tau"] >= 0).all()
    assert len(after["uid"]) == len(before["uid"]) < n_slots
    oa, ob = np.argsort(after["uid"]), np.argsort(before["uid"])
    for k in before:
        np.testing.assert_array_equal(after[k][oa], before[k][ob])
    # stepping on from the compacted buffer changes nothing per uid
    ra.step(800)
    rb.step(800)
    _states_equal(ra, rb)


def test_graph_replay_matches_plain_launches(shared_tables):
    # plain launches vs steps replayed from a captured HIP graph, with eager work in between
    w, ra = _collision_run(shared_tables, n=2000)
    _, rb = _collision_run(shared_tables, n=2000)
    ra.step(2600)
    for chunk in (600, 600, 600, 800):
        rb.run(chunk, graph_steps=50)
        rb.ledger()  # eager work and a synchronisation between replays
    _states_equal(ra, rb)
    la, lb = ra.ledger()[0], rb.ledger()[0]
    for k in ("n_emit", "n_null", "n_pair", "count"):
        assert la[k] == lb[k]


@pytest.mark.parametrize("precision", [capi.QED_FP64, capi.QED_FP32_MIXED])
@pytest.mark.parametrize("compact", [False, True])
def test_batched_instances_equal_single_runs(compact, precision, shared_tables):
    # compact=True: the batched run compacts every 100 steps, which also partitions each
    # instance's photons and rebuilds its live masks; the single runs never compact.  Both
    # precisions: the FP32-mixed batched form of configuration 5 equals its single runs bit for bit
    ws = [W.collision(n, a0=a0, gamma_mean=g0, n_steps=2400, meet_step=1200, seed=1, instance=i, uid0=0)
          for i, (n, a0, g0) in enumerate([(1000, 200.0, 2000.0), (17, 450.0, 800.0), (3001, 60.0, 4500.0),
                                           (1, 300.0, 1500.0), (650, 120.0, 3000.0)])]
    rb = Run(ws, shared_tables, precision=precision)
    if compact:
        for _ in range(24):
            rb.step(100)
            rb.compact()
        assert sum(l["photon_group_reads"] for l in rb.ledger()) > 0
    else:
        rb.step(2400)
    for i, w in enumerate(ws):
        rs = Run(w, shared_tables, precision=precision)
        rs.step(2400)
        _states_equal(rb, rs, ia=i, ib=0)
        lb, ls = rb.ledger()[i], rs.ledger()[0]
        assert lb["n_emit"] == ls["n_emit"] and lb["n_pair"] == ls["n_pair"]


def test_event_queue_overflow_falls_back_to_sweep(shared_tables):
    # a one-entry pair-event queue overflows on most steps with pairs; the sweep that then finds
    # the converting photons gives the same particles as the queue
    w, ra = _collision_run(shared_tables, n=2000)
    _, rb = _collision_run(shared_tables, n=2000)
    rb.set_event_queue(1)
    ra.step(2600)
    rb.step(2600)
    la, lb = ra.ledger()[0], rb.ledger()[0]
    assert la["n_pair"] == lb["n_pair"] > 5
    _states_equal(ra, rb)
    with pytest.raises(capi.QEDError):
        rb.set_event_queue(0)


def test_autotuned_shapes_leave_particles_unchanged(shared_tables):
    # the tuner's trial steps run with every candidate shape; per-uid results equal a run with the
    # default shape, and each sweep gets a shape
    w, ra = _collision_run(shared_tables, n=2000)
    _, rb = _collision_run(shared_tables, n=2000)
    ra.step(1500)
    rb.step(1500)
    res = autotune.tune(rb, steps_per_trial=3, rounds=1, min_particles=10)
    assert res["lepton"] is not None and res["photon"] is not None
    assert len(res["trials"]) == len(autotune.CANDIDATES)
    ra.step(rb.step_index - ra.step_index)
    rb.step(300)
    ra.step(300)
    _states_equal(ra, rb)


def test_spatial_sort_reorders_without_changing_particles(shared_tables):
    # grid workload: sorting by tile keeps every particle (per uid, bit for bit) and the steps
    # after it give the same particles as steps without sorting
    def make():
        w = W.grid_config3(n=3000, nx=256, ny=64, n_steps=200, seed=2)
        w.capacity = dict(electron=20 * w.n, positron=20 * w.n, photon=100 * w.n)
        return w, Run(w, shared_tables)
    _, ra = make()
    _, rb = make()
    ra.step(100)
    rb.step(100)
    before = {name: rb.species(0, name) for name in ("electron", "positron", "photon")}
    rb.sort()
    for name, b in before.items():
        a = rb.species(0, name)
        assert len(a["uid"]) == len(b["uid"])
        oa, ob = np.argsort(a["uid"]), np.argsort(b["uid"])
        for k in b:
            np.testing.assert_array_equal(a[k][oa], b[k][ob], err_msg="%s.%s" % (name, k))
    # the sort moved electrons into tile order: cell-row keys are non-decreasing in slot order
    e = rb.species(0, "electron")
    tile = (np.floor(e["y"] / (2 * np.pi / 128)).astype(np.int64) % 64 // 8) * 32 + \
        (np.floor(e["x"] / (2 * np.pi / 128)).astype(np.int64) % 256 // 8)
    assert np.all(np.diff(tile) >= 0)
    for _ in range(10):
        ra.step(10)
        rb.step(10)
        rb.sort()
    _states_equal(ra, rb)
    assert ra.ledger()[0]["status"] == rb.ledger()[0]["status"] == "QED_OK"


def test_restart_from_saved_state_is_exact(shared_tables):
    w, ra = _collision_run(shared_tables, n=1500)
    ra.step(2600)
    _, rb = _collision_run(shared_tables, n=1500)
    rb.step(1300)
    st = rb.state()
    rc = Run(w, shared_tables, initial=st, draw_initial_tau=False, step0=1300)
    rc.step(1300)
    _states_equal(ra, rc)


def _spectrum(ph, bins):
    eps = np.sqrt(ph["ux"] ** 2 + ph["uy"] ** 2 + ph["uz"] ** 2)
    return np.histogram(eps, bins=bins)[0]


def test_fp32_mixed_against_fp64(gpu_tables_default):
    # precision form of the collision: per-bin photon spectrum error, mean energy loss, pair
    # yield, and ledger closure, against the FP64 form (same random streams)
    t = gpu_tables_default
    n, steps = 100000, 2600
    w = W.collision(n, n_steps=steps, meet_step=steps // 2, seed=31)
    r64 = Run(w, t)
    r32 = Run(w, t, precision=capi.QED_FP32_MIXED)
    r64.step(steps)
    r32.step(steps)
    l64, l32 = r64.ledger()[0], r32.ledger()[0]
    bins = np.logspace(-3, 4, 65)
    s64, s32 = _spectrum(r64.species(0, "photon"), bins), _spectrum(r32.species(0, "photon"), bins)
    sel = s64 >= 10000
    rel = np.abs(s32[sel] - s64[sel]) / s64[sel]
    g0 = l64["energy0"] / n
    loss64 = g0 - l64["energy"][0] / n
    loss32 = g0 - l32["energy"][0] / n
    rec = dict(bins_used=int(sel.sum()), spectrum_rel_err_max=float(rel.max()),
               energy_loss_rel_err=abs(loss32 - loss64) / loss64,
               pair_yield_64=l64["n_pair"] / n, pair_yield_32=l32["n_pair"] / n,
               photons_64=l64["count"][2], photons_32=l32["count"][2], drift_32=l32["drift"], drift_64=l64["drift"])
    record("fp32_mixed_vs_fp64", rec)
    assert l32["status"] == "QED_OK" and l64["status"] == "QED_OK"
    assert sel.sum() >= 10
    assert rel.max() <= 1e-3
    assert rec["energy_loss_rel_err"] <= 1e-3
    assert l32["drift"] <= 1e-9


@pytest.fixture(scope="module")
def gpu_tables_default():
    return Tables.build()


def test_radiation_reaction_flags(oracle_tables):
    # the quantum drag needs g; the classical one does not; either excludes stochastic emission
    t_nog = Tables.from_arrays({k: v for k, v in oracle_tables.items() if k != "g"})
    assert t_nog.view()["g"] is None
    r = Run(W.uniform_b(16, 100.0, 1e-3, 0.01, 2, capi.QED_RR_QUANTUM), t_nog)
    with pytest.raises(capi.QEDError) as e:
        r.step(1)
    assert e.value.status == capi.QED_ERR_STATE
    r.close()
    r = Run(W.uniform_b(16, 100.0, 1e-3, 0.01, 2, capi.QED_RR_CLASSICAL), t_nog)
    r.step(2)
    led = r.ledger()[0]
    assert led["status"] == "QED_OK" and led["radiated"] > 0
    r.close()
    for flags in (capi.QED_EMIT | capi.QED_RR_QUANTUM, capi.QED_RR_QUANTUM | capi.QED_RR_CLASSICAL):
        with pytest.raises(capi.QEDError) as e:
            Run(W.uniform_b(16, 100.0, 1e-3, 0.01, 2, flags), t_nog)
        assert e.value.status == capi.QED_ERR_ARG


def test_radiation_reaction_fp32_mixed(shared_tables):
    # FP32-mixed drag against the FP64 one (same tables): per-lepton gamma and the mean loss
    w = W.collision(20000, a0=200.0, n_steps=2600, meet_step=1300, seed=5, flags=capi.QED_RR_QUANTUM)
    w.capacity = dict(electron=w.n + 1024, positron=1024, photon=1024)
    r64 = Run(w, shared_tables)
    r32 = Run(w, shared_tables, precision=capi.QED_FP32_MIXED)
    r64.step(w.n_steps)
    r32.step(w.n_steps)
    l64, l32 = r64.ledger()[0], r32.ledger()[0]
    a, b = r64.species(0, "electron"), r32.species(0, "electron")
    oa, ob = np.argsort(a["uid"]), np.argsort(b["uid"])
    ga = np.sqrt(1 + a["ux"][oa] ** 2 + a["uy"][oa] ** 2 + a["uz"][oa] ** 2)
    gb = np.sqrt(1 + b["ux"][ob] ** 2 + b["uy"][ob] ** 2 + b["uz"][ob] ** 2)
    rel = np.abs(gb - ga) / ga
    rec = dict(gamma_rel_p50=float(np.median(rel)), gamma_rel_max=float(rel.max()),
               radiated_rel=abs(l32["radiated"] - l64["radiated"]) / l64["radiated"], drift_32=l32["drift"])
    record("rr_fp32_mixed_vs_fp64", rec)
    assert l32["status"] == "QED_OK"
    assert l64["radiated"] > 0.05 * l64["energy0"]
    # FP32 push increments round at ~6e-8 each; over 1300 in-pulse steps the walk stays ~1e-6
    assert rec["gamma_rel_max"] < 4e-5
    assert rec["radiated_rel"] < 1e-7
    assert l32["drift"] < 1e-9


def test_init_optical_depth_keeps_converted_photons(shared_tables):
    # a second qed_init_optical_depth in the middle of a run redraws the live particles' depths
    # and leaves the photons converted since the last compaction converted
    w, r = _collision_run(shared_tables, n=1500)
    r.step(1800)
    before = r.species(0, "photon", live_only=False)
    gone = before["tau"] < 0
    assert gone.any()
    capi.qed_init_optical_depth(r.ws, r._s())
    after = r.species(0, "photon", live_only=False)
    np.testing.assert_array_equal(after["tau"] < 0, gone)
    assert (after["tau"][~gone] > 0).all()
    r.step(10)
    assert r.ledger()[0]["status"] == "QED_OK"


@pytest.mark.parametrize("flags", [W.FLAG_EMIT | W.FLAG_PAIRS | W.FLAG_PROPAGATE, capi.QED_RR_QUANTUM])
def test_ledger_is_independent_of_launch_shape(flags, shared_tables):
    # every energy sum of the ledger is an exact fixed-point sum, so runs whose sweeps have
    # different launch shapes (hence other blocks, waves and atomic orders) give bit-identical
    # ledgers as well as identical particles
    shapes = [((64, 1), (64, 1)), ((256, 8), (256, 16)), ((128, 2), (192, 4))]
    leds, runs = [], []
    for (bl, pl), (bp, pp) in shapes:
        w = W.collision(2000, n_steps=2600, meet_step=1300, seed=21, flags=flags)
        if flags == capi.QED_RR_QUANTUM:
            w.capacity = dict(electron=w.n + 1024, positron=1024, photon=1024)
        r = Run(w, shared_tables)
        r.set_kernel_launch(capi.QED_KERNEL_LEPTON, bl, pl)
        r.set_kernel_launch(capi.QED_KERNEL_PHOTON, bp, pp)
        for _ in range(26):
            r.step(100)
            r.compact()
        leds.append(r.ledger()[0])
        runs.append(r)
    assert leds[0]["status"] == "QED_OK"
    keys = ("energy", "energy0", "work", "defect_emit", "defect_pair", "dropped_energy", "radiated", "drift",
            "count", "n_emit", "n_null", "n_pair")
    for l in leds[1:]:
        for k in keys:
            assert l[k] == leds[0][k], k
    if flags == capi.QED_RR_QUANTUM:
        assert leds[0]["radiated"] > 0
    else:
        assert leds[0]["n_pair"] > 0 and leds[0]["defect_emit"] != 0.0
    for r in runs[1:]:
        _states_equal(runs[0], r)


def _photon_energies(ph):
    return np.sqrt(ph["ux"] ** 2 + ph["uy"] ** 2 + ph["uz"] ** 2)


def _ensemble_errors(g, o, n_electrons, bins=np.logspace(-3, 4, 65), min_count=10000):
    """Ensemble errors of an FP32-mixed run against the FP64 oracle on the same random streams.

    The two sides reproduce almost every particle per uid; the rest belong to families in which
    FP32 rounding moved an event by a step, after which the family is a different Monte-Carlo
    realisation.  Those particles make sampling noise, not a precision bias, so each error is
    returned with the 3-sigma noise that the particles not reproduced per uid can make: a bin's
    photons, and the electrons whose final energy differs."""
    eg, eo = _photon_energies(g["photon"]), _photon_energies(o["photon"])
    hg, ho = np.histogram(eg, bins)[0], np.histogram(eo, bins)[0]
    ug = np.histogram(eg[~np.isin(g["photon"]["uid"], o["photon"]["uid"])], bins)[0]
    uo = np.histogram(eo[~np.isin(o["photon"]["uid"], g["photon"]["uid"])], bins)[0]
    sel = ho >= min_count
    spec_rel = np.abs(hg[sel] - ho[sel]) / ho[sel]
    spec_noise = 3.0 * np.sqrt(ug[sel] + uo[sel]) / ho[sel]
    ge = np.sqrt(1 + g["electron"]["ux"] ** 2 + g["electron"]["uy"] ** 2 + g["electron"]["uz"] ** 2)
    oe = np.sqrt(1 + o["electron"]["ux"] ** 2 + o["electron"]["uy"] ** 2 + o["electron"]["uz"] ** 2)
    common, ig, io = np.intersect1d(g["electron"]["uid"], o["electron"]["uid"], return_indices=True)
    differs = np.abs(ge[ig] - oe[io]) > 1e-3 * oe[io]  # FP32 rounding alone moves gamma by ~1e-5
    n_div = int(differs.sum()) + (len(ge) - len(common)) + (len(oe) - len(common))
    loss_noise = 3.0 * np.std(oe) * np.sqrt(2.0 * n_div) / n_electrons
    return dict(bins_used=int(sel.sum()), spectrum_rel_err_max=float(spec_rel.max()) if sel.any() else 0.0,
                spectrum_excess_max=float(np.max(spec_rel - spec_noise)) if sel.any() else 0.0,
                electrons_diverged=n_div, loss_noise=float(loss_noise))


def test_fp32_mixed_against_fp64_oracle(shared_tables, oracle_tables):
    # configuration 4 (the precision form of the collision) against the FP64 oracle on the same
    # electrons and random streams: per-bin photon spectrum (64 log bins on [1e-3, 1e4]), mean
    # energy loss of the electrons, pair yield, the fraction of oracle particles reproduced per uid,
    # and the ledger closure.  The oracle's tables are loaded, so only precision separates them.
    n, steps = 10000, 2600
    w = W.collision(n, n_steps=steps, meet_step=steps // 2, seed=31)
    r32 = Run(w, shared_tables, precision=capi.QED_FP32_MIXED)
    for _ in range(steps // 100):
        r32.step(100)
        r32.compact()
    l32 = r32.ledger()[0]
    print("[fp32 vs oracle] GPU run done; oracle on %d electrons x %d steps" % (n, steps), flush=True)
    o_res, o_led = oracle_run(w, oracle_tables, capacity=[4 * n, 2 * n, 200 * n])
    print("[fp32 vs oracle] oracle done", flush=True)
    assert l32["status"] == "QED_OK"
    g = {name: r32.species(0, name) for name in ("electron", "positron", "photon")}
    from scipy import stats
    p_ks = stats.ks_2samp(_photon_energies(g["photon"]), _photon_energies(o_res["photon"])).pvalue
    g0 = o_led["energy0"][0] / n
    loss_o = g0 - o_led["energy"][0] / n
    loss_g = l32["energy0"] / n - l32["energy"][0] / n
    uid_match = {name: float(np.mean(np.isin(o_res[name]["uid"], g[name]["uid"]))) for name in g}
    rec = _ensemble_errors(g, o_res, n)
    rec.update(ks_p=float(p_ks), energy_loss_oracle=loss_o, energy_loss_rel_err=abs(loss_g - loss_o) / loss_o,
               pair_yield_oracle=o_led["n_pair"] / n, pair_yield_fp32=l32["n_pair"] / n,
               photons_oracle=len(o_res["photon"]["uid"]), photons_fp32=len(g["photon"]["uid"]),
               uid_reproduced=uid_match, drift_32=l32["drift"])
    record("fp32_mixed_vs_oracle", rec)
    assert rec["bins_used"] >= 10
    assert rec["spectrum_excess_max"] <= 1e-3          # per bin: 1e-3 beyond the diverged families' noise
    assert p_ks > 0.01
    assert rec["energy_loss_rel_err"] <= 1e-3 + rec["loss_noise"] / loss_o
    assert abs(l32["n_pair"] - o_led["n_pair"]) <= 0.05 * o_led["n_pair"] + 3
    assert uid_match["photon"] > 0.99
    assert l32["drift"] <= 1e-9


def _c5_like_instances(n_steps=2400):
    # a spread of configuration 5's instance parameters: counts, a0 and gamma0 from its ranges
    return [W.collision(nn, a0=a0, gamma_mean=g0, n_steps=n_steps, meet_step=n_steps // 2, seed=1, instance=i)
            for i, (nn, a0, g0) in enumerate([(1000, 480.0, 600.0), (2500, 60.0, 4800.0), (1, 250.0, 2000.0),
                                              (1800, 300.0, 1200.0), (700, 150.0, 3500.0)])]


@pytest.mark.parametrize("precision", [capi.QED_FP64, capi.QED_FP32_MIXED])
def test_batched_instances_against_oracle(precision, shared_tables, oracle_tables):
    # configuration 5's batched form (several instances of uneven sizes in one launch, compaction
    # every 100 steps) against the oracle instance by instance: FP64 per uid at the strict bars,
    # FP32-mixed by the ensemble bars of the precision form
    ws = _c5_like_instances()
    rb = Run(ws, shared_tables, precision=precision)
    for _ in range(ws[0].n_steps // 100):
        rb.step(100)
        rb.compact()
    leds = rb.ledger()
    summary = {}
    for i, w in enumerate(ws):
        o_res, o_led = oracle_run(w, oracle_tables, capacity=[4 * w.n + 64, 2 * w.n + 64, 300 * w.n + 1024])
        print("[batched vs oracle] instance %d: oracle done" % i, flush=True)
        assert leds[i]["status"] == "QED_OK"
        if precision == capi.QED_FP64:
            for name in ("electron", "positron", "photon"):
                rep = compare_species(rb.species(i, name), o_res[name], photon=name == "photon")
                flagged = (o_res[name]["margin"] < 1e-9).any()
                assert flagged or (len(rep["only_gpu"]) == 0 and len(rep["only_oracle"]) == 0), (i, name)
                assert (rep["u_err"] <= 1e-10).all() and (rep["e_err"] <= 1e-12).all(), (i, name)
                assert (rep["tau_err"] <= 1e-10).all(), (i, name)
                summary["%d_%s_u_err_max" % (i, name)] = float(rep["u_err"].max(initial=0.0))
            assert leds[i]["n_emit"] == o_led["n_emit"] and leds[i]["n_pair"] == o_led["n_pair"]
        else:
            # mean electron energy at the end (the pulse may still be on the beam, so the mean loss
            # can be small or of either sign; the energy is the well-defined ensemble number)
            e_o, e_g = o_led["energy"][0] / w.n, leds[i]["energy"][0] / w.n
            loss_o = o_led["energy0"][0] / w.n - e_o
            loss_g = leds[i]["energy0"] / w.n - e_g
            g = {name: rb.species(i, name) for name in ("electron", "positron", "photon")}
            ph_match = float(np.mean(np.isin(o_res["photon"]["uid"], g["photon"]["uid"])))
            ens = _ensemble_errors(g, o_res, w.n, min_count=1000)
            summary[i] = dict(energy_rel_err=abs(e_g - e_o) / e_o, loss_oracle=loss_o, loss_fp32=loss_g,
                              loss_noise=ens["loss_noise"] / e_o,
                              spectrum_rel_err_max=ens["spectrum_rel_err_max"],
                              spectrum_excess_max=ens["spectrum_excess_max"],
                              photons=(leds[i]["count"][2], o_led["count"][2]),
                              pairs=(leds[i]["n_pair"], o_led["n_pair"]), uid_reproduced=ph_match)
            if w.n >= 500:
                assert summary[i]["energy_rel_err"] <= 1e-3 + summary[i]["loss_noise"], (i, summary[i])
                assert summary[i]["spectrum_excess_max"] <= 1e-3, (i, summary[i])
                assert ph_match > 0.98, (i, summary[i])
            assert leds[i]["drift"] <= 1e-9
    record("batched_vs_oracle_%s" % ("fp64" if precision == capi.QED_FP64 else "fp32"), summary)
