"""Launch-shape autotuner for the two sweep kernels (lepton sweep, photon sweep).

Each candidate shape (threads per block, particles per thread) is applied to both sweeps and
timed over real steps of a bound run with the library's kernel timing; the time of each kernel
is normalised by the particles it processed in those steps, so a population that grows while
tuning biases no candidate (candidates are also visited in alternating order over the rounds).
The fastest shape per kernel is then applied with qed_set_kernel_launch.  The trial steps
advance the run: per-uid results do not depend on the launch shape (only the order of the
ledger's floating-point sums does), so tuning on the run itself changes no particle.

Results can be kept in a JSON cache keyed by device, precision, field kind, instance count and
the population's size class.
"""
from __future__ import annotations

import json
import math
import os

from . import capi

BLOCKS = (64, 128, 256)
PPTS = (1, 2, 4, 8, 16)  # 16 for the photon sweep only (the lepton sweep then runs 8)
CANDIDATES = tuple((b, p) for b in BLOCKS for p in PPTS)
LEPTON_MAX_PPT = 8
KERNELS = {"lepton": capi.QED_KERNEL_LEPTON, "photon": capi.QED_KERNEL_PHOTON}


def _slots(leds):
    lep = sum(l["particle_steps"][0] + l["particle_steps"][1] for l in leds)
    ph = sum(l["particle_steps"][2] for l in leds)
    return lep, ph


def tune(run, steps_per_trial: int = 10, rounds: int = 2, candidates=CANDIDATES, min_particles: int = 100_000):
    """Times every candidate on `run` (a sim.Run) and applies the fastest shape per kernel.

    Returns {"lepton": {...}, "photon": {...}, "times": {...}, "trials": [...]}: per kernel the
    chosen block, ppt and its time per million particle-steps (ns), or None when the kernel saw
    fewer than `min_particles` particles per step (its shape is then left as it was)."""
    per = {c: {"lepton": [], "photon": []} for c in candidates}
    trials = []
    for r in range(rounds):
        order = list(candidates) if r % 2 == 0 else list(reversed(candidates))
        for (b, p) in order:
            run.set_kernel_launch(capi.QED_KERNEL_LEPTON, b, min(p, LEPTON_MAX_PPT))
            run.set_kernel_launch(capi.QED_KERNEL_PHOTON, b, p)
            run.step(1)
            l0 = _slots(run.ledger())
            run.profile(True)
            run.step(steps_per_trial)
            ms, n = run.profile_read()
            run.profile(False)
            l1 = _slots(run.ledger())
            d_lep, d_ph = l1[0] - l0[0], l1[1] - l0[1]
            rec = {"block": b, "ppt": p, "round": r, "lepton_ms": ms[1], "photon_ms": ms[2],
                   "lepton_particles": d_lep, "photon_particles": d_ph}
            trials.append(rec)
            if d_lep >= min_particles * steps_per_trial and p <= LEPTON_MAX_PPT:
                per[(b, p)]["lepton"].append(ms[1] * 1e6 / d_lep * 1e6)
            if d_ph >= min_particles * steps_per_trial:
                per[(b, p)]["photon"].append(ms[2] * 1e6 / d_ph * 1e6)
    out = {"trials": trials, "times": {name: {"%d/%d" % c: min(v[name]) for c, v in per.items() if v[name]}
                                       for name in KERNELS},
           "particles_per_step": {"lepton": sum(t["lepton_particles"] for t in trials) / (len(trials) * steps_per_trial),
                                  "photon": sum(t["photon_particles"] for t in trials) / (len(trials) * steps_per_trial)}}
    for name, kid in KERNELS.items():
        scored = [(t, c) for c, t in out["times"][name].items()]
        if not scored:
            out[name] = None
            continue
        best_t, c = min(scored)
        b, p = (int(x) for x in c.split("/"))
        run.set_kernel_launch(kid, b, p)
        out[name] = {"block": b, "ppt": p, "ns_per_million_particle_steps": best_t}
    return out


def combine(results, weighted: bool = True):
    """One choice per kernel from several tune() results taken at different points of a run: the
    shape with the smallest sum over the points of (time per particle) x (particles per step at
    that point), i.e. the smallest estimated time of a run sampled at those points (weighted=False:
    plain sum of the per-particle times)."""
    out = {"trials": [t for r in results for t in r["trials"]], "times": {}}
    for name in KERNELS:
        timed = [r for r in results if r["times"][name]]
        keys = set.intersection(*[set(r["times"][name]) for r in timed]) if timed else set()
        wt = lambda r: r.get("particles_per_step", {}).get(name, 1.0) if weighted else 1.0
        tot = {k: sum(r["times"][name][k] * wt(r) for r in timed) for k in keys}
        out["times"][name] = tot
        if not tot:
            out[name] = None
            continue
        c = min(tot, key=tot.get)
        b, p = (int(x) for x in c.split("/"))
        out[name] = {"block": b, "ppt": p, "score": tot[c]}
    return out


def apply(run, result: dict):
    """Applies the shapes of a tune() result (or a cached one) to `run`."""
    for name, kid in KERNELS.items():
        r = result.get(name)
        if r:
            run.set_kernel_launch(kid, r["block"], r["ppt"])


def cache_key(device_name: str, precision: int, field_kind: int, n_inst: int, particles: int) -> str:
    size_class = int(math.log2(max(particles, 1)))
    return "%s|prec%d|field%d|inst%d|2^%d" % (device_name, precision, field_kind, n_inst, size_class)


def cache_load(path: str, key: str):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(key)


def cache_store(path: str, key: str, result: dict):
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = {k: v for k, v in result.items() if k != "trials"}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
