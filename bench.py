#!/usr/bin/env python3
"""Benchmark: trajectories/s and reaction-events/s on one MI355X.

A step advances the whole ensemble of the batched-particles workload to its
final time: 2^20 trajectories, particle p running network p mod 3 of
isomerisation (N_total 1000), birth-death and the bistable Schloegl network,
theta per particle from Gamma(2, 2/theta_nominal) priors, t_end = 50,
eps = 0.03, adaptive explicit/implicit/SSA.  Every step of the method runs
inside it, inputs resident in HBM, outputs preallocated.  The headline form is
the batched mixed-precision schedule (one launch, lx_simulate_set); the plain
fp64 form (one plain lx_simulate launch per network, one lane per trajectory
for life) is timed beside it.  Throughput counts the trajectories that end in
status OK; the others are reported by status.  ``--workload`` selects the
secondary single-network workloads and the particle filter.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one
GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "trajectories/s and reaction-events/s on 1 GPU, batched-mixed vs plain FP64"
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s
# (one fp64 or fp32 add/mul/fma, or one integer operation, per lane per cycle).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Device sources compiled into the simulation kernels at run time, and the host
# library that generates the network's tables and the kernel source around them.
KERNEL_SOURCES = ("lx_params.h", "lx_device.h", "lx_sim.h", "lx_api.cpp")
LARGE_SOURCES = ("lx_sim_large.h", "lx_sim_wave.h")  # networks beyond 16 x 32
METHOD_CONSTANTS = ("n_c", "delta", "n_stiff", "k_ssa", "k_crit", "n_ssa_ex", "n_ssa_im",
                    "lambda_thr", "newton_tol", "newton_maxit", "max_steps")
PROFILES = os.path.join(ROOT, "profiles")
# Workloads bench.py can time; the headline line is "mixed_set".
WORKLOADS = {
    "dimer": "dimer_workload",
    "birth_death": "birth_death_workload",
    "dimer_rathinam": "rathinam_workload",    # implicit leaps (Jacobian variants via --options)
    "random48x128": "random_network_workload",
    "stiff_padded45": "stiff_padded_workload",  # implicit leaps with 48 x 48 Newton systems
    "mixed_set": "mixed_set_workload",        # three networks in one launch (lx_simulate_set)
    "telegraph_pf": "telegraph_workload",     # the particle-filter interval loop (lx_pf_*)
}
FORMS = {
    "plain_fp64": {"precision": "fp64", "schedule": "plain"},
    "plain_mixed": {"precision": "mixed", "schedule": "plain"},
    "batched_fp64": {"precision": "fp64", "schedule": "batched"},
    "batched_mixed": {"precision": "mixed", "schedule": "batched"},
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="",
                    help="comma-separated forms (default: batched_mixed,plain_fp64,batched_fp64 "
                         "for the set, all four for single networks)")
    ap.add_argument("--headline", default="batched_mixed")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the oracle sample until this much time has passed")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--untuned", action="store_true", help="ignore autotuned batched knobs")
    ap.add_argument("--workload", default="mixed_set", choices=sorted(WORKLOADS),
                    help="mixed_set (the headline, default), a secondary single-network "
                         "workload, or the particle filter (telegraph_pf)")
    ap.add_argument("--t-end", type=float, default=0.0,
                    help="override the workload's t_end (secondary workloads only)")
    ap.add_argument("--options", default="",
                    help="JSON object of lx options applied to every form (knob exploration)")
    ap.add_argument("--times", type=int, default=0,
                    help="record the states at this many evenly spaced observation times "
                         "(lx_simulate_grid) instead of only at t_end")
    ap.add_argument("--segments", type=int, default=1,
                    help="run each step as this many consecutive launches over equal parts of "
                         "[0, t_end] (state, r and G carried on, random stream = part); for "
                         "horizons too long for one launch")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="trajectories the oracle baseline runs (default: 8192 per network for "
                         "the set, all for the dimer, 1024 otherwise)")
    ap.add_argument("--cycles", action="store_true",
                    help="after timing, run each form once more in the variant with cycle "
                         "timers and report the shares of the implicit solve spent on the "
                         "Jacobian and on the LU (single-network workloads)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes --steps times "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_calibration(args):
    import torch
    n = args.copy_bytes // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "copies": args.steps}), flush=True)


def kernel_id(opts, large=False):
    """Hash of the kernel sources, the host code that generates the kernel
    source, the launch options of one form and the library's method
    constants: HBM traffic measured with hardware counters is reported only
    for the kernel it was measured on.  `large`: the network takes the
    large-network kernels, whose sources are hashed too."""
    import hashlib
    from paper_1608_07058_amd import lx
    h = hashlib.sha1()
    for name in KERNEL_SOURCES + (LARGE_SOURCES if large else ()):
        with open(os.path.join(ROOT, "paper_1608_07058_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    h.update(json.dumps(opts, sort_keys=True).encode())
    # the library's defaults of the method constants compiled into the kernel
    d = lx.options()
    h.update(json.dumps({k: getattr(d, k) for k in METHOD_CONSTANTS}, sort_keys=True).encode())
    return h.hexdigest()[:16]


def kernel_name(net, form_result):
    """The kernel a single-network form launches."""
    large = net.N > 16 or net.M > 32
    if large:
        one_per_lane = (form_result["schedule"] == "plain"
                        or form_result.get("options", {}).get("lanes_per_traj") == 1)
        return "lx_sim_large" if one_per_lane else "lx_sim_wave"
    return "lx_sim_" + form_result["schedule"]


def recorded_traffic(kid):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) recorded
    in a profile summary for this kernel id, or None."""
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            for line in f:
                if line.startswith("<!-- traffic ") and line.rstrip().endswith("-->"):
                    rec = json.loads(line.strip()[len("<!-- traffic "):-len("-->")])
                    if rec.get("kernel_id") == kid:
                        return rec["fetch_bytes"] + rec["write_bytes"], name
    return None


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def time_form(args, lx, h, theta, x0, wl, form, out):
    import torch
    from paper_1608_07058_amd import autotune
    opts = dict(FORMS[form])
    if opts["schedule"] == "batched" and not args.untuned:
        # knobs found by paper_1608_07058_amd/autotune.py for this ensemble, if any
        net = wl.nets[0]
        opts.update(autotune.lookup(net.m, net.p, wl.P, opts["precision"], wl.mode,
                                    wl.theta[0], wl.x0[0]))
    if args.block_size:
        opts["block_size"] = args.block_size
    if args.options:
        opts.update(json.loads(args.options))
    stream = torch.cuda.current_stream()
    grid_times = observation_times(torch, args, wl)
    segs = max(1, args.segments)
    totals = {}
    if segs > 1:
        x_cur = torch.empty_like(x0)

    def launch():
        if segs > 1:
            # consecutive launches over equal parts of [0, t_end]; the per-part
            # statistics are read back after each part (a few MB) and summed
            x_cur.copy_(x0)
            out["r"].zero_()
            out["G"].zero_()
            totals.clear()
            for k in range(segs):
                lx.simulate(h, theta, x_cur, wl.t_end * (k + 1) / segs, wl.eps, wl.mode, out=out,
                            stream=stream, t_start=wl.t_end * k / segs, accumulate=1,
                            rng_stream=k, **opts)
                x_cur.copy_(out["x"])
                st = lx.stats_numpy(out["stats"])
                for f in ("attempts", "steps_ssa", "steps_explicit", "steps_implicit",
                          "rejections"):
                    totals[f] = totals.get(f, 0) + st[f].astype("int64")
                totals["bad"] = totals.get("bad", 0) + int((st["status"] != 0).sum())
                log(args, f"[bench] part {k + 1}/{segs} done")
        elif grid_times is None:
            lx.simulate(h, theta, x0, wl.t_end, wl.eps, wl.mode, out=out, stream=stream, **opts)
        else:
            lx.simulate_grid(h, theta, x0, grid_times, wl.eps, wl.mode, out=out, stream=stream,
                             **opts)

    if segs > 1:
        # compile the accumulating kernel outside the timed region (64 lanes, a
        # sliver of the first part)
        n = min(64, wl.P)
        lx.simulate(h, theta[:n].contiguous(), x0[:n].contiguous(), wl.t_end / segs / 1000.0,
                    wl.eps, wl.mode, stream=stream, accumulate=1, **opts)
    for _ in range(args.warmup):
        launch()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        launch()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms = sum(per) / len(per)
    r_total = int(out["r"].sum(dtype=torch.int64).item())
    stats = lx.stats_numpy(out["stats"])
    shares = None
    if args.cycles and segs == 1 and grid_times is None:
        # one more launch in the variant with cycle timers (not timed): clock
        # cycles per trajectory in the Jacobian assembly, the LU solves, the
        # implicit solves and the whole trajectory, summed over trajectories
        cyc = torch.zeros((wl.P, 4), dtype=torch.int64, device="cuda")
        lx.simulate(h, theta, x0, wl.t_end, wl.eps, wl.mode, out=out, stream=stream,
                    cycles=cyc.data_ptr(), **opts)
        torch.cuda.synchronize()
        c = cyc.sum(dim=0).tolist()
        shares = {"jacobian_of_implicit": c[0] / c[2] if c[2] else None,
                  "lu_of_implicit": c[1] / c[2] if c[2] else None,
                  "implicit_of_trajectory": c[2] / c[3] if c[3] else None,
                  "cycles": {"jacobian": c[0], "lu": c[1], "implicit": c[2], "trajectory": c[3]}}
    if segs > 1:
        import numpy as np
        stats = {f: totals[f] for f in ("attempts", "steps_ssa", "steps_explicit",
                                        "steps_implicit", "rejections")}
        stats["status"] = np.full(1, 0 if totals["bad"] == 0 else 1)
    return {
        "kernel_id": kernel_id(dict(opts, workload=args.workload, observation_times=args.times)
                               if args.times else
                               dict(opts, workload=args.workload, segments=segs) if segs > 1 else
                               dict(opts, workload=args.workload), large=h.large),
        "ms_per_step": ms,
        "wall_s": wall,
        "trajectories_per_s": wl.P / (ms / 1e3),
        "events_per_s": r_total / (ms / 1e3),
        "events_per_trajectory": r_total / wl.P,
        "attempts_per_trajectory": float(stats["attempts"].mean()),
        "steps_per_trajectory": {m: float(stats["steps_" + m].mean())
                                 for m in ("ssa", "explicit", "implicit")},
        "steps_per_s": {m: float(stats["steps_" + m].sum()) / (ms / 1e3)
                        for m in ("ssa", "explicit", "implicit")},
        "rejections_per_trajectory": float(stats["rejections"].mean()),
        "cycle_shares": shares,
        "lane_status_ok": bool((stats["status"] == 0).all()),
        "precision": opts["precision"],
        "schedule": opts["schedule"],
        "options": {k: v for k, v in opts.items() if k not in ("precision", "schedule")},
    }


def repeat_timed(run, min_seconds):
    """Run `run()` until at least `min_seconds` have passed (at least once);
    returns (first result, repetitions, seconds)."""
    t0 = time.perf_counter()
    first = run()
    reps = 1
    while time.perf_counter() - t0 < min_seconds:
        run()
        reps += 1
    return first, reps, time.perf_counter() - t0


def observation_times(torch, args, wl):
    """--times K: K evenly spaced times ending at t_end (device tensor), or None."""
    if not args.times:
        return None
    import numpy as np
    return torch.as_tensor(np.linspace(wl.t_end / args.times, wl.t_end, args.times),
                           device="cuda")


def timed(args, torch, launch, stream):
    """W untimed launches, then K launches bracketed by HIP events on `stream`;
    returns (mean ms per launch, wall seconds)."""
    for _ in range(args.warmup):
        launch()
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        launch()
        b.record(stream)
        b.synchronize()
        per.append(a.elapsed_time(b))
    return sum(per) / len(per), time.perf_counter() - t0


def line(args, metric_unit, value, ms, dtype, config, extra):
    out = {"metric": METRIC, "value": value, "unit": metric_unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def status_counts(lx, stats_list):
    """Trajectories per final status over a list of lx_stats tensors."""
    import numpy as np
    cnt = np.zeros(5, np.int64)
    for st in stats_list:
        cnt += np.bincount(lx.stats_numpy(st)["status"], minlength=5)[:5]
    return {lx.LANE_STATUS[k]: int(c) for k, c in enumerate(cnt) if c}


def set_roofline(hr, ops_per_launch, ops_note, P, kid):
    """Roofline of the set kernel: algorithmic lane-operations of one launch
    (oracle count per network x trajectories) over its mean duration."""
    achieved = ops_per_launch / (hr["ms_per_step"] / 1e3) / 1e12
    rec = recorded_traffic(kid)
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": rec[0] if rec else None,
            "traffic_unit": "bytes per launch", "traffic_source": rec[1] if rec else None,
            "ops_per_launch": ops_per_launch, "ops_source": ops_note,
            "kernel": "lx_sim_set", "kernel_id": kid}


def bench_set(args, torch, lx, W):
    """Three networks in one ensemble: 2^20 trajectories, particle p runs
    network p mod 3 (its RNG particle id).  The batched forms run the whole
    ensemble in one launch (lx_simulate_set); the plain forms run one plain
    lx_simulate launch per network (one lane per trajectory for life), all on
    the same stream, inside the same timed step."""
    import numpy as np
    wl = W.mixed_set_workload()
    hs = [lx.Network(n.m, n.p) for n in wl.nets]
    th = [torch.as_tensor(t, device="cuda") for t in wl.theta]
    xx = [torch.as_tensor(x, device="cuda") for x in wl.x0]
    K = len(hs)
    from paper_1608_07058_amd import autotune
    stream = torch.cuda.current_stream()
    results = {}
    for form in [f for f in args.forms.split(",") if f]:
        opts = dict(FORMS[form])
        sched = opts.pop("schedule")
        if sched == "batched" and not args.untuned:
            # knobs found by paper_1608_07058_amd/autotune.py for this set, if any
            opts.update(autotune.lookup_set([(n.m, n.p) for n in wl.nets], wl.P,
                                            opts["precision"], wl.mode))
        if args.options:
            opts.update(json.loads(args.options))
        outs = [{"x": torch.empty((t.shape[0], n.N), dtype=torch.int32, device="cuda"),
                 "r": torch.zeros((t.shape[0], n.M), dtype=torch.int32, device="cuda"),
                 "G": torch.zeros((t.shape[0], n.M), dtype=torch.float64, device="cuda"),
                 "stats": torch.empty((t.shape[0], lx.STATS_WORDS), dtype=torch.int64,
                                      device="cuda")}
                for t, n in zip(th, wl.nets)]

        if sched == "batched":
            def launch():
                items = [{"net": h, "theta": t, "x0": x, "pid_base": k, "pid_stride": K,
                          "out": outs[k]} for k, (h, t, x) in enumerate(zip(hs, th, xx))]
                lx.simulate_set(items, wl.t_end, wl.eps, wl.mode, stream=stream, **opts)
        else:
            def launch():
                for k in range(K):
                    lx.simulate(hs[k], th[k], xx[k], wl.t_end, wl.eps, wl.mode, out=outs[k],
                                stream=stream, schedule="plain", pid_base=k, pid_stride=K,
                                **opts)

        ms, wall = timed(args, torch, launch, stream)
        counts = status_counts(lx, [o["stats"] for o in outs])
        n_ok = counts.get("OK", 0)
        ev_ok = 0
        for o in outs:
            ok = (lx.stats_numpy(o["stats"])["status"] == 0)
            ev_ok += int(o["r"].sum(dim=1, dtype=torch.int64).cpu().numpy()[ok].sum())
        results[form] = {"ms_per_step": ms, "wall_s": wall,
                         "trajectories_per_s": n_ok / (ms / 1e3),
                         "events_per_s": ev_ok / (ms / 1e3),
                         "status_counts": counts,
                         "precision": opts["precision"], "schedule": sched,
                         "kernel_id": kernel_id(dict(opts, schedule=sched, workload="mixed_set")),
                         "options": {k: v for k, v in opts.items() if k != "precision"}}
        log(args, f"[bench] {form}: {results[form]}")
    head = args.headline if args.headline in results else sorted(results)[0]
    hr = results[head]
    cpu = None
    roof = None
    if not args.no_cpu_baseline:
        import oracle
        nth = args.cpu_threads or min(os.cpu_count() or 1, 16)
        n_cpu = args.cpu_sample or 8192
        subs = [min(n_cpu, t.shape[0]) for t in wl.theta]

        def run(precision="fp64"):
            return [oracle.simulate(net.m, net.p, wl.theta[k][:subs[k]], wl.x0[k][:subs[k]],
                                    wl.t_end, mode=wl.mode, nthreads=nth, pid_base=k,
                                    pid_stride=K, precision=precision)
                    for k, net in enumerate(wl.nets)]

        ref, reps, dt = repeat_timed(run, args.cpu_seconds)
        cpu = {"value": reps * sum(subs) / dt, "unit": "trajectories/s", "cores": nth,
               "kind": "oracle", "sample": f"the first {n_cpu} trajectories of each network "
                                           f"(fp64 oracle, {nth} threads, {reps} x in {dt:.1f} s)",
               "per_core": reps * sum(subs) / dt / nth}
        log(args, f"[bench] oracle: {cpu}")
        # algorithmic work of the headline launch: the oracle's operation count
        # of the same trajectories in the headline's precision, mean per
        # network over the sample, times the network's trajectories
        if hr["precision"] != "fp64":
            ref = run(hr["precision"])
        ops = 0.0
        se2 = 0.0
        for k, r in enumerate(ref):
            o = r["stats"]["ops"].astype(np.float64)
            Pk = wl.theta[k].shape[0]
            ops += o.mean() * Pk
            se2 += (o.std() / math.sqrt(len(o)) * Pk) ** 2
        roof = set_roofline(hr, ops, f"oracle operation count ({hr['precision']}) of the first "
                                     f"{n_cpu} trajectories of each network, scaled to the "
                                     f"ensemble; sampling SE {100 * math.sqrt(se2) / ops:.1f} %",
                            wl.P, hr["kernel_id"])
    plain = results.get("plain_fp64", {})
    line(args, "trajectories/s", hr["trajectories_per_s"], hr["ms_per_step"],
         "f32+f64" if hr["precision"] == "mixed" else "f64",
         {"workload": wl.name, "trajectories": wl.P, "t_end": wl.t_end, "eps": wl.eps,
          "mode": wl.mode, "form": head, "precision": hr["precision"],
          "schedule": hr["schedule"],
          "counted": "trajectories ending in status OK; the others are listed in "
                     "status_counts"},
         {"events_per_s": hr["events_per_s"], "status_counts": hr["status_counts"],
          "forms": results,
          "speedup_vs_plain_fp64": (hr["trajectories_per_s"] / plain["trajectories_per_s"]
                                    if "trajectories_per_s" in plain else None),
          "roofline": roof, "cpu_baseline": cpu})


def bench_pf(args, torch, lx, W):
    """The particle-filter interval loop: 2^18 particles of the telegraph model
    x 50 observation intervals of length 5, captured once into a HIP graph;
    a step is one replay of all 50 intervals.  Observations: a seeded random
    walk of the protein level (synthetic)."""
    import numpy as np
    wl = W.telegraph_workload()
    net = wl.nets[0]
    K, dt, obs, sd = 50, 5.0, 3, 10.0
    rng = np.random.default_rng(9)
    y = np.clip(100.0 + np.cumsum(rng.normal(0.0, 15.0, K)), 0.0, None)
    h = lx.Network(net.m, net.p)
    th0 = torch.as_tensor(wl.theta[0], device="cuda")
    x00 = torch.as_tensor(wl.x0[0], device="cuda")
    results = {}
    from paper_1608_07058_amd import autotune
    for form in [f for f in args.forms.split(",") if f]:
        opts = dict(FORMS[form])
        if opts["schedule"] == "batched" and not args.untuned:
            # knobs tuned on the first interval's ensemble, if any
            opts.update(autotune.lookup(net.m, net.p, wl.P, opts["precision"], wl.mode,
                                        wl.theta[0], wl.x0[0]))
        if args.options:
            opts.update(json.loads(args.options))
        th = th0.clone()
        xx = x00.clone()
        pf = lx.ParticleFilter(h, th, xx, torch.as_tensor(y, device="cuda"),
                               torch.full((net.M,), 2.0, dtype=torch.float64, device="cuda"),
                               torch.as_tensor(2.0 / net.theta, device="cuda"), dt, obs, sd,
                               **opts)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            pf.capture(s)

        def reset():
            pf.theta.copy_(th0)
            pf.x.copy_(x00)
            pf.r.zero_()
            pf.G.zero_()
            torch.cuda.synchronize()

        per = []
        for k in range(args.warmup + args.steps):
            reset()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(s)
            pf.replay(s)
            b.record(s)
            b.synchronize()
            if k >= args.warmup:
                per.append(a.elapsed_time(b))
        ms = sum(per) / len(per)
        ll = pf.loglik.cpu().numpy()
        results[form] = {"ms_per_step": ms, "particle_intervals_per_s": wl.P * K / (ms / 1e3),
                         "loglik_finite": bool(np.isfinite(ll).all()),
                         "precision": opts["precision"], "schedule": opts["schedule"],
                         "kernel_id": kernel_id(dict(opts, workload="telegraph_pf")),
                         "options": opts}
        pf.release()
        log(args, f"[bench] {form}: {results[form]}")
    head = args.headline if args.headline in results else sorted(results)[0]
    hr = results[head]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nth = args.cpu_threads or min(os.cpu_count() or 1, 16)
        n_cpu = args.cpu_sample or 65536
        _, reps, dtc = repeat_timed(
            lambda: oracle.pf_run(net.m, net.p, wl.theta[0][:n_cpu], wl.x0[0][:n_cpu], K, dt, obs,
                                  sd, y, np.full(net.M, 2.0), 2.0 / net.theta, nthreads=nth),
            args.cpu_seconds)
        cpu = {"value": reps * n_cpu * K / dtc, "unit": "particle-intervals/s", "cores": nth,
               "kind": "oracle", "sample": f"{n_cpu} particles x {K} intervals, fp64 oracle "
                                           f"filter, {nth} threads, {reps} x in {dtc:.1f} s",
               "per_core": reps * n_cpu * K / dtc / nth}
        # the simulations' algorithmic operations, in the headline's precision,
        # on the first particles, scaled to the filter (the weighting and
        # resampling kernels stream a few bytes per particle)
        n_ops = min(8192, wl.P)
        ref = oracle.pf_run(net.m, net.p, wl.theta[0][:n_ops], wl.x0[0][:n_ops], K, dt, obs, sd,
                            y, np.full(net.M, 2.0), 2.0 / net.theta, nthreads=nth,
                            precision=hr["precision"])
        ops_per_launch = ref["ops"] / n_ops * wl.P
        roof = set_roofline(hr, ops_per_launch,
                            f"oracle operation count ({hr['precision']}) of the simulations of "
                            f"a {n_ops}-particle filter over the {K} intervals, scaled to "
                            f"{wl.P} particles", wl.P, hr["kernel_id"])
        roof["kernel"] = "lx_sim_" + hr["schedule"] + " (in the filter's graph)"
    else:
        roof = None
    extra = {"forms": results, "roofline": roof, "cpu_baseline": cpu}
    if "plain_fp64" in results and head != "plain_fp64":
        extra["speedup_vs_plain_fp64"] = results["plain_fp64"]["ms_per_step"] / hr["ms_per_step"]
    line(args, "particle-intervals/s", hr["particle_intervals_per_s"], hr["ms_per_step"],
         "f32+f64" if hr["precision"] == "mixed" else "f64",
         {"workload": wl.name, "particles": wl.P, "intervals": K, "dt": dt, "form": head}, extra)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_bytes:
        copy_calibration(args)
        return
    import torch
    from paper_1608_07058_amd import lx, workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if (args.times or args.segments > 1) and args.workload in ("mixed_set", "telegraph_pf"):
        raise SystemExit("--times and --segments apply to single-network workloads")
    if args.times and args.segments > 1:
        raise SystemExit("--times and --segments are exclusive")
    if not args.forms:
        args.forms = ("batched_mixed,plain_fp64,batched_fp64"
                      if args.workload in ("mixed_set", "telegraph_pf")
                      else "batched_mixed,plain_fp64,plain_mixed,batched_fp64")
    if args.workload == "mixed_set":
        return bench_set(args, torch, lx, W)
    if args.workload == "telegraph_pf":
        return bench_pf(args, torch, lx, W)
    wl = getattr(W, WORKLOADS[args.workload])()
    if args.t_end > 0.0:
        if args.workload == "mixed_set":
            raise SystemExit("--t-end applies to secondary workloads only")
        wl.t_end = args.t_end
    net = wl.nets[0]
    theta = torch.as_tensor(wl.theta[0], device="cuda")
    x0 = torch.as_tensor(wl.x0[0], device="cuda")
    h = lx.Network(net.m, net.p)
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    for form in forms:
        out = {
            "x": torch.empty((wl.P, net.N), dtype=torch.int32, device="cuda"),
            "r": torch.empty((wl.P, net.M), dtype=torch.int32, device="cuda"),
            "G": torch.empty((wl.P, net.M), dtype=torch.float64, device="cuda"),
            "stats": torch.empty((wl.P, lx.STATS_WORDS), dtype=torch.int64, device="cuda"),
        }
        if args.times:
            out["x_grid"] = torch.empty((wl.P, args.times, net.N), dtype=torch.int32,
                                        device="cuda")
        try:
            results[form] = time_form(args, lx, h, theta, x0, wl, form, out)
        except lx.LxError as exc:
            results[form] = {"error": str(exc)}
        log(args, f"[bench] {form}: {results[form]}")
    head = args.headline if "error" not in results.get(args.headline, {"error": 1}) else None
    if head is None:
        ok = [f for f in forms if "error" not in results[f]]
        head = ok[0]
    hr = results[head]

    # Algorithmic work per trajectory, counted by the oracle on the same
    # workload (its trajectories are the kernels' trajectories).
    cpu = None
    ops_per_traj = None
    if not args.no_cpu_baseline:
        import oracle
        nth = args.cpu_threads or min(os.cpu_count() or 1, 16)
        n_cpu = args.cpu_sample or (wl.P if args.workload == "dimer" else min(wl.P, 1024))

        def run():
            if args.times:
                import numpy as np
                return oracle.simulate_grid(
                    net.m, net.p, wl.theta[0][:n_cpu], wl.x0[0][:n_cpu],
                    np.linspace(wl.t_end / args.times, wl.t_end, args.times), mode=wl.mode,
                    nthreads=nth)
            return oracle.simulate(net.m, net.p, wl.theta[0][:n_cpu], wl.x0[0][:n_cpu],
                                   wl.t_end, mode=wl.mode, nthreads=nth)

        ref, reps, dt = repeat_timed(run, args.cpu_seconds)
        ops_per_traj = float(ref["stats"]["ops"].mean())
        what = (f"all {wl.P} trajectories of the workload" if n_cpu == wl.P else
                f"the first {n_cpu} of the {wl.P} trajectories")
        cpu = {"value": reps * n_cpu / dt, "unit": "trajectories/s", "cores": nth,
               "kind": "oracle",
               "sample": f"{what}, fp64 oracle, {nth} threads, {reps} x in {dt:.1f} s",
               "per_core": reps * n_cpu / dt / nth}
        log(args, f"[bench] oracle: {cpu}")
    roof = None
    if ops_per_traj is not None:
        achieved = ops_per_traj * wl.P / (hr["ms_per_step"] / 1e3) / 1e12
        rec = recorded_traffic(hr["kernel_id"])
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": rec[0] if rec else None,
                "traffic_unit": "bytes per launch", "traffic_source": rec[1] if rec else None,
                "algorithmic_bytes": wl.P * (net.M * 8 + net.N * 4 + net.N * 4 + net.M * 4
                                             + net.M * 8 + lx.STATS_WORDS * 8),
                "ops_per_trajectory": ops_per_traj,
                "kernel": kernel_name(net, hr),
                "kernel_id": hr["kernel_id"]}
    dtype = "f32+f64" if hr["precision"] == "mixed" else "f64"
    line = {
        "metric": METRIC,
        "value": hr["trajectories_per_s"],
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "trajectories": wl.P, "t_end": wl.t_end, "eps": wl.eps,
                   "mode": wl.mode, "form": head, "precision": hr["precision"],
                   "schedule": hr["schedule"]},
        "events_per_s": hr["events_per_s"],
        "forms": results,
        "speedup_vs_plain_fp64": (hr["trajectories_per_s"] /
                                  results["plain_fp64"]["trajectories_per_s"]
                                  if "trajectories_per_s" in results.get("plain_fp64", {}) else None),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.times:
        line["config"]["observation_times"] = args.times
    if args.segments > 1:
        line["config"]["segments"] = args.segments
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
