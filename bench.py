#!/usr/bin/env python3
"""Throughput of the QED Monte-Carlo step (push + emission + pairs) on one MI355X.

Workload (main line): the head-on collision of 1e6 electrons (gamma ~ N(2000, 10%),
sigma = 2 um) with a linearly polarised a0 = 200, lambda = 1 um, 30 fs sin^2 pulse,
dt = lambda/(200 c), a 20000-step schedule whose pulse peak meets the beam centre at step
10000; photon emission and pair creation on, dead photons compacted every 100 steps, FP64.

Timed window: when `warmup + steps` is shorter than the schedule, the run is advanced
untimed to `meet - steps/2 - warmup`, then `warmup` untimed steps run, then exactly `steps`
timed steps centred on the collision (the steps where the pulse drives emission and pairs).
Otherwise the window is steps [warmup, warmup + steps) of the schedule.

value = evaluated particle-steps per second of the timed window: every electron and positron
present at the start of a step (each is pushed), plus every photon step evaluated in full (a
photon inside its pair window: the steps in which its pair rate can be non-zero).  Photon slots
outside their window, whose position is the closed form of their birth record, are not counted;
their count is reported apart (`photon_slot_steps`).

Also on the same JSON line: the roofline of the dominant kernel (algorithmic bytes per launch /
its mean HIP-event duration over the same window, against 8 TB/s), and the FP64 oracle timed on
the host cores over a bounded sample of the same workload.  `detail` holds the other forms
(FP32-mixed, batched instances, the 2-D grid workload, the uniform-field workload) and the
value of the whole 20000-step schedule.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (push+QED MC) FP64 vs FP32-mixed vs batched; % HBM peak"
HBM_PEAK_GBS = 8000.0
SCHEDULE = 20000   # steps of the collision schedule
MEET = 10000       # step at which the pulse peak meets the beam centre


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_bytes(form, kind, led0, led1, grid=False, pulse=True):
    """Algorithmic HBM bytes of one kernel class between two ledgers.

    Lepton sweep, per lepton step in 3-D: with the full push 56 B read (x, u, tau) + 56 B
    written in FP64 (FP32-mixed: the stored words of position and momentum, 4 B each, plus the
    FP64 tau); outside the plane-wave pulse (field-free drift) x and u read, x written: 72 B in
    FP64; + 16 B per queued emission event.  2-D grid workload: 48 + 48 B per step (x, y, u, tau).
    Photon sweep: 8 B per live mask of a group of 64 slots that was read, and 4 B per slot
    whose pair window was read (its live bit was set); per photon inside its window what its record holds: in the
    plane-wave pulse the phase at step 0, its rate per step and the chi scale (24 B in FP64, 16 B
    in FP32-mixed), in a general field the momentum, the birth position and the birth step (44 B
    in FP64, 24 B in FP32-mixed); + 16 B (tau read and written) for the photons that see a
    non-zero pair rate; + 8 B per queued pair event.  The event passes (separate classes) read the event's particle and write
    the children."""
    d = lambda k, i=None: (led1[k][i] - led0[k][i]) if i is not None else (led1[k] - led0[k])
    if kind == "lepton":
        steps = d("particle_steps", 0) + d("particle_steps", 1)
        full = d("lepton_steps_in_field")
        if grid:
            per_full = per_drift = 96
        elif form == "fp64":
            per_full, per_drift = 112, 72
        else:
            per_full, per_drift = LEPTON_BYTES_FP32
        return full * per_full + (steps - full) * per_drift + (d("n_emit") + d("n_null")) * 16
    if pulse:
        rec = 24 if form == "fp64" else 16
    else:
        rec = 44 if form == "fp64" else 24
    return (d("photon_window_reads") * 4 + d("photon_group_reads") * 8 + d("photon_steps_active") * rec
            + d("photon_steps_in_field") * 16 + d("n_pair") * 8)


# FP32-mixed lepton bytes per step (full push, drift); set from the stored layout below
LEPTON_BYTES_FP32 = (112, 60)


def source_hash():
    h = hashlib.sha1()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1311_5551_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1311_5551_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(kernel, form):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel sources with the same bench window (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, form))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash() or d.get("bench_window") != WINDOW_KEY.get(form):
        return None
    return d.get("bytes_per_launch")


WINDOW_KEY = {}


def tune_launch(form, args, tables):
    """Autotuned sweep launch shapes for a form: the tuner runs on a separate run of the same
    collision (tune_scale times the electrons; the best shape depends on the population size, so
    full size by default), at points of the timed window, and each kernel gets the shape with the
    smallest population-weighted sum of its per-particle times over the points, an estimate of
    its total time in the window."""
    from paper_1311_5551_amd import autotune, capi, workloads as W
    from paper_1311_5551_amd.sim import Run
    prec = capi.QED_FP64 if form == "fp64" else capi.QED_FP32_MIXED
    w = W.collision_config2(n=max(int(args.electrons * args.tune_scale), 1000), n_steps=SCHEDULE)
    run = Run(w, tables, precision=prec)
    points = [int(x) for x in args.tune_at.split(",")]
    log("%s: autotuning launch shapes on a %d-electron replica at steps %s" % (form, w.n, points))
    results = []
    for p in points:
        while run.step_index < p:
            n = min(args.compact_every - run.step_index % args.compact_every, p - run.step_index)
            run.run(n, graph_steps=n if n == args.compact_every else 0)
            if run.step_index % args.compact_every == 0:
                run.compact()
        results.append(autotune.tune(run, steps_per_trial=6, rounds=2, min_particles=1000))
    res = autotune.combine(results)
    autotune.apply(run, res)
    run.close()
    log("%s: tuned lepton %s photon %s" % (form, res["lepton"], res["photon"]))
    return res


TUNED_CACHE = os.path.join(ROOT, "paper_1311_5551_amd", "tuned_launch.json")


def tuned_launch(form, args, tables):
    """Cached tuned shapes for (device, form, collision workload size, kernel sources), else a
    fresh tuning whose result is written to gpurun_out/tuned_launch.json (the tuner's output
    file; the package's cache holds its entries)."""
    import torch
    from paper_1311_5551_amd import autotune, capi
    prec = capi.QED_FP64 if form == "fp64" else capi.QED_FP32_MIXED
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = autotune.cache_key(arch, prec, 1, 1, args.electrons) + "|src" + source_hash()
    if args.tune == "auto":
        hit = autotune.cache_load(TUNED_CACHE, key)
        if hit:
            log("%s: cached launch shapes %s" % (form, {k: hit[k] for k in ("lepton", "photon")}))
            return hit
    res = tune_launch(form, args, tables)
    out = os.path.join(ROOT, "gpurun_out", "tuned_launch.json")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    autotune.cache_store(out, key, res)
    return res


def size_grid(w, tables, args, probe_n=100_000):
    """Steps until the grid workload's population reaches 4x the initial electrons, and buffer
    capacities, from a probe run of the first `probe_n` electrons (uniformly spread over the
    grid, so their yields per electron are those of the full run)."""
    from paper_1311_5551_amd import capi, workloads as W
    from paper_1311_5551_amd.sim import Run
    p = W.subset(w, range(min(w.n, probe_n)))
    p.capacity = dict(electron=20 * p.n + 4096, positron=20 * p.n + 4096, photon=40 * p.n + 4096)
    run = Run(p, tables, precision=capi.QED_FP64)
    log("grid: probe run of %d electrons to find the 4x step" % p.n)
    k = 0
    while k < 2000:
        run.step(1)
        k += 1
        led = run.ledger()[0]
        if led["status"] != "QED_OK":
            raise RuntimeError("grid probe run: %s" % led["status"])
        if sum(led["count"]) >= 4 * p.n:
            break
    run.close()
    y = [c / p.n for c in led["count"]]
    w.capacity = dict(electron=int(1.3 * y[0] * w.n) + 4096, positron=int(1.3 * y[1] * w.n) + 4096,
                      photon=int(1.3 * y[2] * w.n) + 4096)
    log("grid: %d steps, yields per electron %s" % (k, [round(v, 3) for v in y]))
    return k


def size_batched(ws, tables, args, last_step, probe_n=256):
    """Buffer capacities of the batched instances from a probe run: the first `probe_n`
    electrons of every instance (the same families as in the full run) through the schedule up
    to `last_step`, retiring photons at each compaction as the full run does; each species gets
    1.3x the largest population per initial electron the probe held (photons: just before a
    compaction) plus a margin.  Family sizes scatter widely at the strongest fields, so the
    probe takes 256 electrons per instance and the margin is 1.5x plus four standard errors of the
    probe's per-electron mean (counted as if families were independent Poisson sources)."""
    from paper_1311_5551_amd import capi, workloads as W
    from paper_1311_5551_amd.sim import Run
    probe = []
    for w in ws:
        p = W.subset(w, range(min(w.n, probe_n)))
        p.capacity = dict(electron=2000 * p.n + 4096, positron=2000 * p.n + 4096, photon=4000 * p.n + 8192)
        probe.append(p)
    run = Run(probe, tables, precision=capi.QED_FP32_MIXED)
    if args.batched_retire:
        run.set_retire(RETIRE_BINS, RETIRE_EMIN, RETIRE_EMAX)
    log("batched: sizing buffers from a %d-electron probe run" % sum(p.n for p in probe))
    step = 0
    peak = [[0, 0, 0] for _ in probe]
    while step < last_step:
        n = min(args.compact_every - step % args.compact_every, last_step - step)
        run.run(n, graph_steps=n if n == args.compact_every else 0)
        step += n
        if step % args.compact_every == 0:
            for pk, l in zip(peak, run.ledger()):
                for s_ in range(3):
                    pk[s_] = max(pk[s_], l["count"][s_])
            run.compact()
    led = run.ledger()
    run.close()
    if any(l["status"] != "QED_OK" for l in led):
        raise RuntimeError("batched probe run: %s" % sorted(set(l["status"] for l in led)))
    for w, p, l, pk in zip(ws, probe, led, peak):
        y = [max(pk[s_], l["count"][s_]) / p.n for s_ in range(3)]
        cap = [int(1.5 * y[s_] * w.n + 4.0 * w.n * math.sqrt(max(y[s_], 1.0) / p.n)) for s_ in range(3)]
        w.capacity = dict(electron=cap[0] + 4096, positron=cap[1] + 4096, photon=cap[2] + 16384)
    tot = [sum(w.capacity[k] for w in ws) for k in ("electron", "positron", "photon")]
    log("batched: capacities %d electrons, %d positrons, %d photons" % tuple(tot))


# photon spectrum of the retired photons (batched form)
RETIRE_BINS, RETIRE_EMIN, RETIRE_EMAX = 64, 1e-3, 1e4


def window(total, warmup, steps, meet):
    """(first untimed step, first timed step) of a window of `steps` steps after `warmup` untimed
    ones: centred on `meet` when the schedule is longer than warmup + steps."""
    if warmup + steps >= total:
        return 0, warmup
    s0 = min(max(meet - steps // 2, warmup), total - steps)
    return s0 - warmup, s0


def _aggregate(leds):
    out = {"particle_steps": [0, 0, 0], "count": [0, 0, 0]}
    for k in ("n_emit", "n_null", "n_pair", "photon_steps_in_field", "photon_steps_active", "lepton_steps_in_field",
              "photon_window_reads", "photon_group_reads"):
        out[k] = sum(l[k] for l in leds)
    for i in range(3):
        out["particle_steps"][i] = sum(l["particle_steps"][i] for l in leds)
        out["count"][i] = sum(l["count"][i] for l in leds)
    return out


def evaluated_steps(a0, a1):
    """Evaluated particle-steps between two aggregated ledgers: lepton steps plus photon steps
    inside the photon's pair window."""
    return (a1["particle_steps"][0] - a0["particle_steps"][0] + a1["particle_steps"][1] - a0["particle_steps"][1]
            + a1["photon_steps_active"] - a0["photon_steps_active"])


def run_form(form, args, tables, tuned):
    import torch
    from paper_1311_5551_amd import autotune, capi, workloads as W
    from paper_1311_5551_amd.sim import Run

    graphs = form not in ("grid", "feedback") and not args.no_graphs
    if form == "feedback":
        w = W.feedback_config(n=args.grid_electrons)
        total = size_grid(w, tables, args)
        ws, pre, s0, steps = [w], 0, 0, total
        workload = ("feedback_cp_standing_a500: %d electrons at rest, uniform over a periodic 4096x2048 FP64 Yee grid "
                    "(dx = lambda/128) that starts with the standing wave of two CP lasers a0=500 and is advanced "
                    "by Maxwell's equations with the leptons' current each step (field feedback, plasma density "
                    "1e-3 n_c), charge-conserving deposition, first-order gather, 2D3V, FP64, dt=lambda/400c, steps "
                    "0..%d (until the population reaches 4x), particles sorted by 8x8-cell tile every %d steps"
                    % (w.n, total, args.grid_sort_every))
    elif form == "grid":
        w = W.grid_config3(n=args.grid_electrons)
        total = size_grid(w, tables, args)
        ws, pre, s0, steps = [w], 0, 0, total
        workload = ("grid_cp_standing_a500: %d electrons at rest, uniform over a periodic 4096x2048 FP32 Yee grid "
                    "(dx = lambda/128), standing wave of two CP lasers a0=500 refreshed analytically each step, "
                    "first-order gather, 2D3V, FP64 particles, dt=lambda/400c, steps 0..%d (until the population "
                    "reaches 4x), particles sorted by 8x8-cell tile every %d steps"
                    % (w.n, total, args.grid_sort_every))
    elif form == "uniform":
        w = W.uniform_b_config1()
        total = w.n_steps
        ws, pre, s0, steps = [w], 0, 0, total
        workload = ("uniform_b_1e4: 10000 electrons gamma0=1000 perpendicular to a uniform B (eta0=1), dt=0.01 "
                    "gyro-periods, steps 0..%d, photons recorded (not propagated), FP64, hipGraph replay of "
                    "100-step graphs" % total)
    elif form == "batched":
        ws = W.batched_config5(n_steps=SCHEDULE, n_scale=args.batched_scale)
        pre, s0 = window(SCHEDULE, args.batched_warmup, args.batched_window, MEET)
        steps = min(args.batched_window, SCHEDULE - s0)
        size_batched(ws, tables, args, s0 + steps)
        total = s0 + steps
        workload = ("batched_collisions: 256 instances, N_i=floor(%s10^U(3,6)) (total %d electrons), a0~U(50,500), "
                    "gamma0 log-U[500,5000], FP32-mixed, dt=lambda/200c, steps %d..%d of %d (window centred on the "
                    "collisions at step %d; %d untimed steps before), hipGraph replay of %d-step graphs, "
                    "compaction every %d%s"
                    % ("" if args.batched_scale == 1.0 else "%g*" % args.batched_scale, sum(w.n for w in ws), s0,
                       s0 + steps, SCHEDULE, MEET, s0, args.compact_every, args.compact_every,
                       " retiring the photons whose pair window is over" if args.batched_retire else ""))
    else:
        w = W.collision_config2(n=args.electrons, n_steps=SCHEDULE)
        ws = [w]
        pre, s0 = window(SCHEDULE, args.warmup, args.steps, MEET)
        steps = min(args.steps, SCHEDULE - s0)
        total = s0 + steps
        workload = ("collision_lp_a200: %d electrons gamma~N(2000,10%%) sigma 2um vs LP a0=200 lambda 1um 30fs "
                    "sin^2, dt=lambda/200c, timed steps %d..%d of %d (the pulse meets the beam at step %d; steps "
                    "0..%d untimed), emission+pairs, compaction every %d"
                    % (w.n, s0, s0 + steps, SCHEDULE, MEET, s0, args.compact_every))
    WINDOW_KEY[form] = "%d..%d" % (s0, s0 + steps)
    prec = capi.QED_FP64 if form in ("fp64", "grid", "uniform", "feedback") else capi.QED_FP32_MIXED
    compact = form not in ("uniform",)

    def make_run():
        r = Run(ws, tables, precision=prec, block=args.block, ppt=args.ppt)
        if tuned is not None:
            autotune.apply(r, tuned)
        if form == "batched" and args.batched_retire:
            r.set_retire(RETIRE_BINS, RETIRE_EMIN, RETIRE_EMAX)
        return r

    def advance(run, step, k, graph):
        """k steps from `step`: graph replay of whole compaction periods, compaction between them."""
        done = 0
        while done < k:
            n = min(args.compact_every - step % args.compact_every, k - done)
            if graph:
                run.run(n, graph_steps=n if n == args.compact_every else 0)
            else:
                for i in range(n):
                    if form in ("grid", "feedback") and (done + i) % args.grid_sort_every == 0:
                        run.sort()  # tile order for the grid gathers, inside the timed region
                    run.step(1)
            step += n
            done += n
            if compact and step % args.compact_every == 0:
                run.compact()
            if done % 2000 < n and done < k:
                log("%s: step %d" % (form, step))
        return step

    res = dict(form=form, workload=workload, n_inst=len(ws), window=[s0, s0 + steps])
    # the whole schedule once (collision forms): evaluated particle-steps per second over all steps
    if form in ("fp64", "fp32") and args.full_run:
        log("%s: whole schedule (%d steps)" % (form, SCHEDULE))
        run = make_run()
        led0 = _aggregate(run.ledger())
        run.synchronize()
        t0 = time.perf_counter()
        advance(run, 0, SCHEDULE, graphs)
        run.synchronize()
        t1 = time.perf_counter()
        led1 = _aggregate(run.ledger())
        ev = evaluated_steps(led0, led1)
        res["whole_schedule"] = {"steps": SCHEDULE, "seconds": t1 - t0, "evaluated_particle_steps": int(ev),
                                 "value": ev / (t1 - t0),
                                 "photon_slot_steps": int(led1["particle_steps"][2] - led0["particle_steps"][2])}
        run.close()
        del run
        torch.cuda.empty_cache()

    log("%s: allocating and binding (%s)" % (form, workload[:60]))
    run = make_run()
    if pre:
        log("%s: %d untimed steps to the window" % (form, pre))
    step = advance(run, 0, pre, graphs)
    warm = s0 - pre
    log("%s: %d warmup steps" % (form, warm))
    step = advance(run, step, warm, graphs)
    led0 = run.ledger()
    run.synchronize()
    log("%s: timing steps %d..%d" % (form, s0, s0 + steps))
    t0 = time.perf_counter()
    step = advance(run, step, steps, graphs)
    run.synchronize()
    t1 = time.perf_counter()
    led1 = run.ledger()
    run.close()
    del run
    torch.cuda.empty_cache()
    # kernel times: HIP events around every kernel class on the run's stream, over the same
    # steps replayed eagerly from the same initial state (graph replay records no per-kernel
    # events, and the event records would add launch gaps to the timed run)
    log("%s: kernel timing pass (HIP events, steps %d..%d, eager)" % (form, s0, s0 + steps))
    run = make_run()
    step = advance(run, 0, s0, graphs)
    lk0 = _aggregate(run.ledger())
    run.profile(True)
    step = advance(run, step, steps, False)
    ms, launches = run.profile_read()
    run.profile(False)
    lk1 = _aggregate(run.ledger())
    run.close()
    del run
    torch.cuda.empty_cache()

    agg0, agg1 = _aggregate(led0), _aggregate(led1)
    ev = evaluated_steps(agg0, agg1)
    status = sorted(set(l["status"] for l in led1))
    d = lambda k: int(agg1[k] - agg0[k])
    res.update(seconds=t1 - t0, steps=steps, evaluated_particle_steps=int(ev), value=ev / (t1 - t0),
               ms_per_step=1e3 * (t1 - t0) / steps,
               lepton_steps=int(agg1["particle_steps"][0] + agg1["particle_steps"][1]
                                - agg0["particle_steps"][0] - agg0["particle_steps"][1]),
               photon_slot_steps=int(agg1["particle_steps"][2] - agg0["particle_steps"][2]),
               kernel_ms=dict(setup=ms[0], lepton=ms[1], photon=ms[2], pair_events=ms[3], emit_events=ms[4],
                              field_solver=ms[5]),
               launches=dict(setup=launches[0], lepton=launches[1], photon=launches[2], pair_events=launches[3],
                             emit_events=launches[4], field_solver=launches[5]),
               photons_end=int(agg1["count"][2]), pairs=d("n_pair"), emissions=d("n_emit"),
               drift_max=max(l["drift"] for l in led1),
               photon_steps_in_field=d("photon_steps_in_field"), photon_steps_active=d("photon_steps_active"),
               lepton_steps_in_field=d("lepton_steps_in_field"), photon_window_reads=d("photon_window_reads"),
               photon_group_reads=d("photon_group_reads"),
               dropped=int(sum(l["n_dropped"] for l in led1)), status=status,
               overflowed=[dict(instance=i, dropped=int(l["n_dropped"]), count=[int(c) for c in l["count"]])
                           for i, l in enumerate(led1) if l["n_dropped"] > 0][:16],
               photons_retired=int(sum(l["n_retired"] for l in led1)),
               launch={k: (tuned.get(k) if tuned else None) for k in ("lepton", "photon")},
               kernel_timing="HIP events per kernel class on the run's stream over the same steps replayed eagerly "
                             "from the same initial state" + (" (the timed run replays captured HIP graphs)"
                                                               if graphs else ""))
    # the kernel that takes the most time in the window bounds the step
    kind = "photon" if ms[2] >= ms[1] else "lepton"
    byts = kernel_bytes("fp64" if prec == capi.QED_FP64 else "fp32", kind, lk0, lk1, grid=form in ("grid", "feedback"),
                        pulse=form not in ("grid", "uniform", "feedback"))
    n_l = launches[2] if kind == "photon" else launches[1]
    avg_s = (ms[2] if kind == "photon" else ms[1]) / max(n_l, 1) * 1e-3
    achieved = byts / max(n_l, 1) / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = measured_traffic(kind, form)
    res["roofline"] = {"kernel": "k_%s (%s)" % (kind, form), "bound": "hbm",
                       "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                       "traffic": traffic, "algorithmic_bytes_per_launch": byts / max(n_l, 1),
                       "mean_launch_us": avg_s * 1e6}
    if form == "feedback" and launches[5]:
        # the Yee solver's three passes per step (B half, E, B half): 9 + 15 + 9 planes of nx x ny
        # FP64 words read or written; one fused pass would need 15 (read E, B, J; write E, B, J)
        nx, ny = ws[0].grid[:2]
        plane = nx * ny * 8
        per_step_s = ms[5] / launches[5] * 1e-3
        res["field_solver"] = {"us_per_step": per_step_s * 1e6, "bytes_per_step": 33 * plane,
                               "min_bytes_per_step": 15 * plane,
                               "achieved_GBs": 33 * plane / per_step_s / 1e9,
                               "frac": 33 * plane / per_step_s / 1e9 / HBM_PEAK_GBS}
    if form in ("fp64", "fp32") and res["emissions"] == 0 and res["lepton_steps_in_field"] == 0:
        log("%s: WARNING: the timed window has no in-field step: it measures a field-free drift" % form)
        res["note"] = "no in-field step in the timed window: a field-free drift, not the QED step"
    return res


def cpu_baseline(args):
    """The FP64 oracle on the host cores over the first `families` electrons of the collision
    workload (their whole families, all 20000 steps)."""
    import oracle
    from paper_1311_5551_amd import workloads as W
    tables = oracle.build_tables()
    w = W.subset(W.collision_config2(n=args.electrons), range(args.cpu_families))
    cfg = oracle.RunConfig(field_kind=w.field_kind, field=w.field, dt=w.dt, n_steps=w.n_steps, flags=w.flags,
                           seed=w.seed, instance=w.instance)
    threads = oracle.num_threads()
    log("cpu baseline: oracle on %d families x %d steps, %d threads" % (w.n, w.n_steps, threads))
    t0 = time.perf_counter()
    _, led = oracle.run(cfg, tables, electrons=w.electrons)
    t1 = time.perf_counter()
    # the same on one core, over a smaller share of the families
    w1 = W.subset(W.collision_config2(n=args.electrons), range(args.cpu_families_1core))
    log("cpu baseline: oracle on %d families x %d steps, 1 thread" % (w1.n, w1.n_steps))
    oracle.set_threads(1)
    try:
        t2 = time.perf_counter()
        _, led1 = oracle.run(cfg, tables, electrons=w1.electrons)
        t3 = time.perf_counter()
    finally:
        oracle.set_threads(threads)
    return {"value": led["particle_steps"] / (t1 - t0), "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d electrons of the 1e6-electron collision and all their descendants, all 20000 steps "
                      "(%d particle-steps, %.1f s; the oracle evaluates every live particle in every step, so every "
                      "one of its particle-steps is an evaluated one); oracle tables built beforehand"
                      % (w.n, led["particle_steps"], t1 - t0),
            "one_core": {"value": led1["particle_steps"] / (t3 - t2), "unit": "particle-steps/s", "cores": 1,
                         "sample": "first %d electrons and their descendants, all 20000 steps (%d particle-steps, "
                                   "%.1f s)" % (w1.n, led1["particle_steps"], t3 - t2)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--electrons", type=int, default=1_000_000)
    ap.add_argument("--compact-every", type=int, default=100)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--ppt", type=int, default=4)
    ap.add_argument("--forms", default="fp64,fp32,batched,grid,uniform,feedback",
                    help="comma list of fp64, fp32, batched, grid, uniform; the first gives `value` and `roofline`")
    ap.add_argument("--no-full-run", dest="full_run", action="store_false",
                    help="skip the whole-schedule value of the collision forms")
    ap.add_argument("--cpu-families", type=int, default=1500)
    ap.add_argument("--cpu-families-1core", type=int, default=40,
                    help="families of the one-core oracle timing (a share of the --cpu-families sample)")
    ap.add_argument("--tune", choices=("auto", "replica", "none"), default="auto",
                    help="sweep launch shapes per form: auto = the tuned shapes cached in "
                         "paper_1311_5551_amd/tuned_launch.json for this device, form, workload and kernel sources, "
                         "else tune; replica = tune now; none = --block/--ppt")
    ap.add_argument("--tune-scale", type=float, default=1.0, help="electrons of the tuning run / --electrons")
    ap.add_argument("--tune-at", default="9000,9500,10000,10500,11000",
                    help="steps of the tuning run at which trials run (population-weighted sum)")
    ap.add_argument("--batched-scale", type=float, default=1.0, help="factor on every instance's electrons")
    ap.add_argument("--no-batched-retire", dest="batched_retire", action="store_false",
                    help="keep the photons whose pair window is over (they then need ~3x the memory)")
    ap.add_argument("--batched-window", type=int, default=4000)
    ap.add_argument("--batched-warmup", type=int, default=50)
    ap.add_argument("--grid-electrons", type=int, default=16_000_000)
    ap.add_argument("--grid-sort-every", type=int, default=10, help="grid form: steps between spatial sorts")
    ap.add_argument("--no-graphs", action="store_true",
                    help="time eager launches instead of graph replay")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run plain device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the QED step shards by particle family with no per-step "
              "communication, so only the single-GPU throughput is measured here (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = 1 << 27
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)                 # the runtime's copy kernel
        for _ in range(20):
            torch.mul(src, 1.0, out=dst)   # an elementwise kernel: 8 B read + 8 B written per element
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "launches": 20}))
        return
    from paper_1311_5551_amd.sim import Tables
    torch.cuda.set_device(0)
    log("building tables on the GPU")
    tables = Tables.build()
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    tuned = {}
    results = []
    for f in forms:
        key = "fp64" if f in ("fp64", "grid", "uniform", "feedback") else "fp32"
        if args.tune != "none" and key not in tuned and f in ("fp64", "fp32", "batched"):
            tuned[key] = tuned_launch(key, args, tables)
        results.append(run_form(f, args, tables, tuned.get(key) if f in ("fp64", "fp32", "batched") else None))
    main_r = results[0]
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    out = {
        "metric": METRIC,
        "value": main_r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": main_r["steps"],
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_r["form"] in ("fp64", "grid", "uniform", "feedback") else "f32+f64",
        "data": "synthetic",
        "config": {"workload": main_r["workload"], "form": main_r["form"], "instances": main_r["n_inst"],
                   "counted": "evaluated particle-steps: lepton steps + photon steps inside the photon's pair window",
                   # the shapes the run used: tuned (cache or replica) per sweep, else the command line
                   "launch": ({k: {"block": v["block"], "particles_per_thread": v["ppt"]}
                               for k, v in main_r["launch"].items() if v}
                              if any(main_r["launch"].values()) else
                              {"block": args.block, "particles_per_thread": args.ppt})},
        "roofline": main_r["roofline"],
        "cpu_baseline": cpu,
        "detail": {r["form"]: {k: v for k, v in r.items() if k not in ("workload",)} for r in results},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
