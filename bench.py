#!/usr/bin/env python3
"""Throughput of the QED Monte-Carlo step (push + emission + pairs) on one MI355X.

Workload (default): the head-on collision of 1e6 electrons (gamma ~ N(2000, 10%),
sigma = 2 um) with a linearly polarised a0 = 200, lambda = 1 um, 30 fs sin^2 pulse,
dt = lambda/(200 c), 20000 steps, photon emission and pair creation on, dead photons
compacted every 100 steps, FP64.  `warmup` untimed steps, then exactly `steps` timed
steps of the same run.  value = particle-steps (every electron, positron and photon
slot present at the start of a step) per second of the timed region.

Also printed on the same JSON line: the roofline of the dominant kernel (algorithmic
bytes per launch / its mean HIP-event duration over the timed region, against 8 TB/s),
and the FP64 oracle timed on the host cores over a bounded sample of the same workload.
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


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_bytes(form, kind, led0, led1, grid=False):
    """Algorithmic HBM bytes of one kernel class over the timed region.

    grid=True (the 2-D grid workload, FP64): lepton full step 48 B read (x, y, u, tau) + 48 B
    written; photon: 4 B per window and per group summary read + 44 B per photon inside its
    window (k, x and y at birth, birth step), the gather of the FP32 grid not counted (the
    201 MB grid is read from the cache hierarchy, its refresh is the set-up class).

    Lepton sweep, per particle-step in 3-D: with the full push 56 B read (x, u, tau) + 56 B
    written in FP64 (FP32-mixed: the same 112 B as hi/lo words of position and momentum plus
    the FP64 tau); outside the plane-wave pulse (field-free drift) x and u read, x written:
    72 B in FP64, 60 B in FP32-mixed (hi/lo position, high words of u); + 16 B per queued
    emission event.  The emission pass (separate class) reads the event's lepton and writes the
    photon.
    Photon sweep: 4 B per summary window of a group of 64 slots that was read, and 4 B per slot
    whose pair window was read (every slot, except in groups whose summary excludes the step);
    per photon inside its window, with
    a field that depends on x only (the plane-wave pulse), k (3 words), x at birth (1 word) and
    the birth step (4 B): 36 B in FP64, 20 B in FP32-mixed; + 16 B (tau read and written) for
    the photons that see a non-zero pair rate; + 8 B per queued pair event.  The pair pass
    (separate class) reads the event's photon and writes the two leptons."""
    d = lambda k, i=None: (led1[k][i] - led0[k][i]) if i is not None else (led1[k] - led0[k])
    if grid:
        if kind == "lepton":
            return (d("particle_steps", 0) + d("particle_steps", 1)) * 96 + (d("n_emit") + d("n_null")) * 16
        return ((d("photon_window_reads") + d("photon_group_reads")) * 4 + d("photon_steps_active") * 44
                + d("photon_steps_in_field") * 16 + d("n_pair") * 8)
    if kind == "lepton":
        steps = d("particle_steps", 0) + d("particle_steps", 1)
        full = d("lepton_steps_in_field")
        drift = 72 if form == "fp64" else 60
        return full * 112 + (steps - full) * drift + (d("n_emit") + d("n_null")) * 16
    full = 36 if form == "fp64" else 20
    return ((d("photon_window_reads") + d("photon_group_reads")) * 4 + d("photon_steps_active") * full
            + d("photon_steps_in_field") * 16 + d("n_pair") * 8)


def source_hash():
    h = hashlib.sha1()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1311_5551_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1311_5551_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(kernel, form):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, form))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def tune_launch(form, args, tables):
    """Autotuned sweep launch shapes for a form: the tuner runs on a separate run of the same
    collision (tune_scale times the electrons; the best shape depends on the population size, so
    full size by default), at points spread over the run (before, during and after the
    collision), and each kernel gets the shape with the smallest population-weighted sum of its
    per-particle times over the points, an estimate of its total time in the run."""
    from paper_1311_5551_amd import autotune, capi, workloads as W
    from paper_1311_5551_amd.sim import Run
    prec = capi.QED_FP64 if form == "fp64" else capi.QED_FP32_MIXED
    w = W.collision_config2(n=max(int(args.electrons * args.tune_scale), 1000), n_steps=20000)
    run = Run(w, tables, precision=prec)
    points = [int(x) for x in args.tune_at.split(",")]
    log("%s: autotuning launch shapes on a %d-electron replica at steps %s" % (form, w.n, points))
    results = []
    for p in points:
        while run.step_index < p:
            run.step(1)
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
    fresh tuning whose result is written to gpurun_out/tuned_launch.json (entries of that file
    are what the package's cache holds)."""
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


def size_batched(ws, tables, args, probe_n=64):
    """Buffer capacities of the batched instances from a probe run: the first `probe_n`
    electrons of every instance (the same families as in the full run) through the whole
    schedule; each species gets 1.3x its probe yield per initial electron plus a margin."""
    from paper_1311_5551_amd import capi, workloads as W
    from paper_1311_5551_amd.sim import Run
    probe = []
    for w in ws:
        p = W.subset(w, range(min(w.n, probe_n)))
        p.capacity = dict(electron=2000 * p.n + 4096, positron=2000 * p.n + 4096, photon=4000 * p.n + 8192)
        probe.append(p)
    run = Run(probe, tables, precision=capi.QED_FP32_MIXED)
    log("batched: sizing buffers from a %d-electron probe run" % sum(p.n for p in probe))
    for i in range(ws[0].n_steps):
        run.step(1)
        if (i + 1) % args.compact_every == 0:
            run.compact()
    led = run.ledger()
    run.close()
    if any(l["status"] != "QED_OK" for l in led):
        raise RuntimeError("batched probe run: %s" % sorted(set(l["status"] for l in led)))
    for w, p, l in zip(ws, probe, led):
        y_e = l["count"][0] / p.n
        y_p = l["count"][1] / p.n
        y_g = (l["n_emit"] + l["n_pair"]) / p.n  # photons emitted (an upper bound of the live ones)
        w.capacity = dict(electron=int(1.3 * y_e * w.n) + 4096, positron=int(1.3 * y_p * w.n) + 4096,
                          photon=int(1.3 * y_g * w.n) + 16384)


def run_form(form, args, tables, tuned):
    import torch
    from paper_1311_5551_amd import autotune, capi, workloads as W
    from paper_1311_5551_amd.sim import Run

    batched = form == "batched"
    if form == "grid":
        w = W.grid_config3(n=args.grid_electrons)
        steps = size_grid(w, tables, args)
        ws, warmup = [w], 0
        workload = ("grid_cp_standing_a500: %d electrons at rest, uniform over a periodic 4096x2048 FP32 Yee grid "
                    "(dx = lambda/128), standing wave of two CP lasers a0=500 refreshed analytically each step, "
                    "first-order gather, 2D3V, FP64 particles, dt=lambda/400c, steps 0..%d (until the population "
                    "reaches 4x), particles sorted by 8x8-cell tile every %d steps"
                    % (w.n, steps, args.grid_sort_every))
    elif not batched:
        total = args.warmup + args.steps
        w = W.collision_config2(n=args.electrons, n_steps=max(total, 20000))
        ws = [w]
        workload = ("collision_lp_a200: %d electrons gamma~N(2000,10%%) sigma 2um vs LP a0=200 lambda 1um "
                    "30fs sin^2, dt=lambda/200c, steps %d..%d of 20000, emission+pairs, compaction every %d"
                    % (w.n, args.warmup, total, args.compact_every))
        warmup, steps = args.warmup, args.steps
    else:
        # the C5 instance mix with every N_i scaled by batched_scale, on the collision schedule of
        # the FP64 line (dt = lambda/200c, the pulse meets each beam at the middle step); at full
        # size the collisions emit ~4.5e9 photons (~200 GB) and the run would take minutes
        total = args.batched_steps
        ws = W.batched_config5(n_steps=total, n_scale=args.batched_scale)
        size_batched(ws, tables, args)
        warmup, steps = args.batched_warmup, total - args.batched_warmup
        workload = ("batched_collisions: 256 instances, N_i=floor(%g*10^U(3,6)) (total %d electrons), a0~U(50,500), "
                    "gamma0 log-U[500,5000], FP32-mixed, dt=lambda/200c, steps %d..%d of %d (collisions at step "
                    "%d), hipGraph replay of %d-step graphs, compaction every %d"
                    % (args.batched_scale, sum(w.n for w in ws), warmup, total, total, total // 2,
                       args.compact_every, args.compact_every))
    prec = capi.QED_FP64 if form in ("fp64", "grid") else capi.QED_FP32_MIXED
    # the grid form reorders its particles between steps (qed_sort); --no-graphs runs every step
    # eagerly with the kernel timers on (for profilers that cannot follow graph replay)
    graphs = form != "grid" and not args.no_graphs

    def make_run():
        r = Run(ws, tables, precision=prec, block=args.block, ppt=args.ppt)
        if tuned is not None:
            autotune.apply(r, tuned)
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
                    if form == "grid" and (done + i) % args.grid_sort_every == 0:
                        run.sort()  # tile order for the grid gathers, inside the timed region
                    run.step(1)
            step += n
            done += n
            if step % args.compact_every == 0:
                run.compact()
            if done % 2000 < n and done < k:
                log("%s: step %d" % (form, step))
        return step

    log("%s: allocating and binding (%s)" % (form, workload[:60]))
    run = make_run()
    log("%s: %d warmup steps" % (form, warmup))
    step = advance(run, 0, warmup, graphs)
    led0 = run.ledger()
    if not graphs:
        run.profile(True)
    run.synchronize()
    log("%s: timing %d steps" % (form, steps))
    t0 = time.perf_counter()
    step = advance(run, step, steps, graphs)
    run.synchronize()
    t1 = time.perf_counter()
    led1 = run.ledger()
    # kernel times: HIP events around every kernel class on the run's stream, over the same
    # steps replayed eagerly from the same initial state (graph replay records no per-kernel
    # events, and the events would add launch gaps to the timed run)
    if graphs:
        run.close()
        del run
        torch.cuda.empty_cache()
        log("%s: kernel timing pass (eager, %d + %d steps)" % (form, warmup, steps))
        run = make_run()
        step = advance(run, 0, warmup, True)
        lk0 = run.ledger()
        run.profile(True)
        step = advance(run, step, steps, False)
        ms, launches = run.profile_read()
        run.profile(False)
        lk1 = run.ledger()
        lk0, lk1 = _aggregate(lk0), _aggregate(lk1)
    else:
        ms, launches = run.profile_read()
        run.profile(False)
    n_inst = len(ws)
    agg0 = _aggregate(led0)
    agg1 = _aggregate(led1)
    if not graphs:
        lk0, lk1 = agg0, agg1
    psteps = sum(agg1["particle_steps"]) - sum(agg0["particle_steps"])
    status = sorted(set(l["status"] for l in led1))
    res = dict(form=form, workload=workload, n_inst=n_inst, seconds=t1 - t0, particle_steps=int(psteps),
               value=psteps / (t1 - t0), ms_per_step=1e3 * (t1 - t0) / steps,
               kernel_ms=dict(setup=ms[0], lepton=ms[1], photon=ms[2], pair_events=ms[3], emit_events=ms[4]),
               launches=dict(setup=launches[0], lepton=launches[1], photon=launches[2], pair_events=launches[3],
                             emit_events=launches[4]),
               photons_end=int(agg1["count"][2]), pairs=int(agg1["n_pair"] - agg0["n_pair"]),
               emissions=int(agg1["n_emit"] - agg0["n_emit"]), drift_max=max(l["drift"] for l in led1),
               photon_steps_in_field=int(agg1["photon_steps_in_field"] - agg0["photon_steps_in_field"]),
               photon_steps_active=int(agg1["photon_steps_active"] - agg0["photon_steps_active"]),
               lepton_steps_in_field=int(agg1["lepton_steps_in_field"] - agg0["lepton_steps_in_field"]),
               photon_window_reads=int(agg1["photon_window_reads"] - agg0["photon_window_reads"]),
               photon_group_reads=int(agg1["photon_group_reads"] - agg0["photon_group_reads"]),
               dropped=int(sum(l["n_dropped"] for l in led1)), status=status,
               launch={k: (tuned.get(k) if tuned else None) for k in ("lepton", "photon")})
    if graphs:
        res["kernel_timing"] = ("HIP events per kernel class over the same steps replayed eagerly from the same "
                                "initial state (the timed run replays captured HIP graphs)")
    kind = "photon" if ms[2] >= ms[1] else "lepton"
    byts = kernel_bytes("fp64" if form in ("fp64", "grid") else "fp32", kind, lk0, lk1, grid=form == "grid")
    n_l = launches[2] if kind == "photon" else launches[1]
    avg_s = (ms[2] if kind == "photon" else ms[1]) / max(n_l, 1) * 1e-3
    achieved = byts / max(n_l, 1) / avg_s / 1e9
    traffic = measured_traffic(kind, form)
    res["roofline"] = {"kernel": "k_%s (%s)" % (kind, form), "bound": "hbm",
                       "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                       "traffic": traffic, "algorithmic_bytes_per_launch": byts / max(n_l, 1),
                       "mean_launch_us": avg_s * 1e6}
    run.close()
    del run
    torch.cuda.empty_cache()
    return res


def _aggregate(leds):
    out = {"particle_steps": [0, 0, 0], "count": [0, 0, 0]}
    for k in ("n_emit", "n_null", "n_pair", "photon_steps_in_field", "photon_steps_active", "lepton_steps_in_field",
              "photon_window_reads", "photon_group_reads"):
        out[k] = sum(l[k] for l in leds)
    for i in range(3):
        out["particle_steps"][i] = sum(l["particle_steps"][i] for l in leds)
        out["count"][i] = sum(l["count"][i] for l in leds)
    return out


def cpu_baseline(args):
    """The FP64 oracle on the host cores over the first `families` electrons of the same
    workload (their whole families, all 20000 steps)."""
    import oracle
    from paper_1311_5551_amd import workloads as W
    tables = oracle.build_tables()
    w = W.subset(W.collision_config2(n=args.electrons), range(args.cpu_families))
    cfg = oracle.RunConfig(field_kind=w.field_kind, field=w.field, dt=w.dt, n_steps=w.n_steps, flags=w.flags,
                           seed=w.seed, instance=w.instance)
    log("cpu baseline: oracle on %d families x %d steps, %d threads" % (w.n, w.n_steps, oracle.num_threads()))
    t0 = time.perf_counter()
    _, led = oracle.run(cfg, tables, electrons=w.electrons)
    t1 = time.perf_counter()
    return {"value": led["particle_steps"] / (t1 - t0), "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "first %d electrons of the 1e6-electron collision and all their descendants, all 20000 steps "
                      "(%d particle-steps, %.1f s); oracle tables built beforehand" % (w.n, led["particle_steps"],
                                                                                         t1 - t0)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=19800)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--electrons", type=int, default=1_000_000)
    ap.add_argument("--compact-every", type=int, default=100)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--ppt", type=int, default=4)
    ap.add_argument("--forms", default="fp64,fp32,batched,grid",
                    help="comma list of fp64, fp32, batched, grid; the first gives `value` and `roofline`")
    ap.add_argument("--cpu-families", type=int, default=1500)
    ap.add_argument("--tune", choices=("auto", "replica", "none"), default="auto",
                    help="sweep launch shapes per form: auto = the tuned shapes cached in "
                         "paper_1311_5551_amd/tuned_launch.json for this device, form, workload and kernel sources, "
                         "else tune; replica = tune now; none = --block/--ppt")
    ap.add_argument("--tune-scale", type=float, default=1.0, help="electrons of the tuning run / --electrons")
    ap.add_argument("--tune-at", default="5000,10000,11500,13000,14500,16000,17500,19000",
                    help="steps of the tuning run at which trials run (population-weighted sum)")
    ap.add_argument("--batched-scale", type=float, default=0.1)
    ap.add_argument("--grid-electrons", type=int, default=16_000_000)
    ap.add_argument("--grid-sort-every", type=int, default=10, help="grid form: steps between spatial sorts")
    ap.add_argument("--batched-warmup", type=int, default=200)
    ap.add_argument("--no-graphs", action="store_true",
                    help="time eager launches with per-kernel HIP events instead of graph replay")
    ap.add_argument("--batched-steps", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB, 20 times (reference for HBM byte counters)")
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
            dst.copy_(src)
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
        key = "fp64" if f in ("fp64", "grid") else "fp32"
        if args.tune != "none" and key not in tuned:
            tuned[key] = tuned_launch(key, args, tables)
        results.append(run_form(f, args, tables, tuned.get(key)))
    main_r = results[0]
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    out = {
        "metric": METRIC,
        "value": main_r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_r["form"] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": main_r["workload"], "form": main_r["form"], "instances": main_r["n_inst"],
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
