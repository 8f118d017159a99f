"""Helpers shared by the GPU parity tests: run a workload on the GPU (through the C ABI)
and on the oracle (CPU), match particles by uid and compare them.

Both sides evaluate exp, log, sin and cos correctly rounded wherever a result reaches a
momentum or a sampled chi, and order the FP64 operations of the step the same way, so with
the oracle's tables loaded into the library the momenta agree to the last bit.  What may
differ is the optical depth: the kernels decrement it with the device library's log and
trigonometry, so tau differs by a few ulp per decrement and an event can move by one step
when tau lands within rounding of zero (a threshold straddle).  Bars:
  momenta    max_c |du_c| / max(|u|, 1)  <= 1e-12 for >= 99% of particles, every particle
             within U_CAP, and |d gamma| / gamma <= E_TOL for all
  positions  |dx| / max(|x|, 1)          <= 1e-10
  tau        |dtau|                      <= 1e-10  (sums of O(1) decrements)
A particle whose family showed |tau| < 1e-9 after some decrement is a flagged threshold
straddle: the two sides may legitimately decide its event differently.  With tables built
on the GPU the bars widen (see the end-to-end constants in test_gpu_parity.py).
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle

OUT_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")


def record(name, data):
    """Append a measurement to gpurun_out/parity_records.jsonl (read back from the GPU machine)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    with open(os.path.join(OUT_DIR, "parity_records.jsonl"), "a") as f:
        f.write(json.dumps({"name": name, "data": data}, default=float) + "\n")

U_TOL = 1e-12
U_FRAC = 0.99
U_CAP = 1e-10
E_TOL = 1e-12
X_TOL = 1e-10
TAU_TOL = 1e-10
STRADDLE = 1e-9


def oracle_run(w, tables, electrons=None, photons=None, capacity=None):
    cfg = oracle.RunConfig(field_kind=w.field_kind, field=w.field, dt=w.dt, n_steps=w.n_steps, flags=w.flags,
                           seed=w.seed, instance=w.instance, dims=w.dims, grid=w.grid, t0=w.t0)
    return oracle.run(cfg, tables, electrons=electrons if electrons is not None else w.electrons, photons=photons,
                      capacity=capacity)


def match(a_uid, b_uid):
    """Index arrays (ia, ib) of common uids, plus uids only in a and only in b."""
    a_uid = np.asarray(a_uid, dtype=np.uint64)
    b_uid = np.asarray(b_uid, dtype=np.uint64)
    assert len(np.unique(a_uid)) == len(a_uid), "duplicate uids"
    assert len(np.unique(b_uid)) == len(b_uid), "duplicate uids"
    common, ia, ib = np.intersect1d(a_uid, b_uid, assume_unique=True, return_indices=True)
    only_a = np.setdiff1d(a_uid, common, assume_unique=True)
    only_b = np.setdiff1d(b_uid, common, assume_unique=True)
    return ia, ib, only_a, only_b


def rel_err_u(g, o, ia, ib):
    ug = np.stack([g["ux"][ia], g["uy"][ia], g["uz"][ia]])
    uo = np.stack([o["ux"][ib], o["uy"][ib], o["uz"][ib]])
    scale = np.maximum(np.sqrt((uo * uo).sum(0)), 1.0)
    return np.abs(ug - uo).max(0) / scale


def rel_err_energy(g, o, ia, ib, photon):
    """|d gamma| / gamma for leptons, |d |k|| / |k| for photons (rotation-invariant)."""
    ug = np.stack([g["ux"][ia], g["uy"][ia], g["uz"][ia]])
    uo = np.stack([o["ux"][ib], o["uy"][ib], o["uz"][ib]])
    if photon:
        eg, eo = np.sqrt((ug * ug).sum(0)), np.sqrt((uo * uo).sum(0))
    else:
        eg, eo = np.sqrt(1 + (ug * ug).sum(0)), np.sqrt(1 + (uo * uo).sum(0))
    return np.abs(eg - eo) / eo


def compare_species(g, o, photon=False, check_tau=True):
    """Per-uid comparison of one species; returns a report dict."""
    ia, ib, only_g, only_o = match(g["uid"], o["uid"])
    rep = {"n_gpu": len(g["uid"]), "n_oracle": len(o["uid"]), "matched": len(ia),
           "only_gpu": only_g, "only_oracle": only_o, "ia": ia, "ib": ib}
    if len(ia) == 0:
        rep.update(u_err=np.zeros(0), e_err=np.zeros(0), x_err=np.zeros(0), tau_err=np.zeros(0))
        return rep
    rep["u_err"] = rel_err_u(g, o, ia, ib)
    rep["e_err"] = rel_err_energy(g, o, ia, ib, photon)
    xe = []
    for k in ("x", "y", "z"):
        if k in o and k in g:
            xe.append(np.abs(g[k][ia] - o[k][ib]) / np.maximum(np.abs(o[k][ib]), 1.0))
    rep["x_err"] = np.max(np.stack(xe), axis=0)
    rep["tau_err"] = np.abs(g["tau"][ia] - o["tau"][ib]) if check_tau else np.zeros(len(ia))
    return rep


def _is_photon(d):
    return "birth_step" in d


def straddle_uids(o_all):
    """uids (any species) whose oracle margin flags a possible threshold straddle."""
    out = []
    for s in o_all.values():
        if "margin" in s:
            out.append(s["uid"][s["margin"] < STRADDLE])
    return np.concatenate(out) if out else np.zeros(0, dtype=np.uint64)
