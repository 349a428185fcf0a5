"""Autotuner for the batched schedule.

Sweeps the launch knobs of ``lx_simulate`` (active lanes per wave, SSA steps
per leap iteration, block size, resident blocks per CU, lanes per
trajectory) on a given ensemble, times each setting with HIP events on the
launch stream, and keeps the fastest; then refines it one knob at a time
with the register budget (waves per SIMD the kernel is compiled for) and the
lane groups that finish each block's last trajectories.  The knobs never change results (every trajectory's actions are
fixed by its particle id), so tuning is pure scheduling.  Results persist in a
JSON file keyed by network, ensemble size, precision, mode and architecture.

    python -m paper_1608_07058_amd.autotune --workload dimer
"""

from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_FILE = os.path.join(HERE, "tuned.json")

GRID = {
    "lanes_per_traj": (1, 2, 4, 8, 16),
    "lanes_per_wave": (16, 32, 64),
    "ssa_k": (4, 8, 16, 64),
    "block_size": (64, 256),
    "blocks_per_cu": (2, 4),
    "regroup": (0,),
}


# A smaller grid for ensembles too large to sweep the full one in minutes
# (--grid small).
SMALL_GRID = {
    "lanes_per_traj": (1, 2, 4),
    "lanes_per_wave": (64,),
    "ssa_k": (4, 8, 16),
    "block_size": (256,),
    "blocks_per_cu": (2, 4),
    "regroup": (0,),
}


# Networks beyond 16 species or 32 reactions (one trajectory per wave): the
# block size sets how many waves share one Newton area in LDS.
LARGE_GRID = {
    "block_size": (64, 128, 192, 256),  # blocks per CU: as many as their LDS fits
}


def valid(opts, P):
    if "lanes_per_wave" not in opts:  # LARGE_GRID
        return True
    tpl = opts.get("lanes_per_traj", 1)
    if tpl > 1 and opts.get("regroup", 0):
        return False
    if opts["lanes_per_wave"] < tpl:
        return False
    return (opts["lanes_per_wave"] // tpl) * (opts["block_size"] // 64) <= P


def key_of(net_m, net_p, P, precision, mode, theta, x0, arch="gfx950"):
    """Key of an ensemble: the network, its inputs (theta [P][M], x0 [P][N]:
    two ensembles of one network with other constants behave differently),
    P, precision and mode."""
    import numpy as np
    h = hashlib.sha1(np.ascontiguousarray(net_m, np.int32).tobytes() +
                     np.ascontiguousarray(net_p, np.int32).tobytes()).hexdigest()[:16]
    d = hashlib.sha1(np.ascontiguousarray(theta, np.float64).tobytes() +
                     np.ascontiguousarray(x0, np.int32).tobytes()).hexdigest()[:8]
    return f"{arch}/{h}-{d}/P{P}/{precision}/{mode}"


def load(path=DEFAULT_FILE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(net_m, net_p, P, precision, mode, theta, x0, path=DEFAULT_FILE):
    """Tuned options for this ensemble, or {} if it was never tuned."""
    key = key_of(net_m, net_p, P, precision, mode, theta, x0)
    return dict(load(path).get(key, {}).get("options", {}))


def tune(lx, h, theta, x0, t_end, eps, mode, precision, grid=None, reps=2, log=None):
    """Time every knob setting; return (best options, table of (options, ms))."""
    import torch
    grid = grid or GRID
    P = theta.shape[0]
    out = {
        "x": torch.empty((P, h.N), dtype=torch.int32, device="cuda"),
        "r": torch.empty((P, h.M), dtype=torch.int32, device="cuda"),
        "G": torch.empty((P, h.M), dtype=torch.float64, device="cuda"),
        "stats": torch.empty((P, lx.STATS_WORDS), dtype=torch.int64, device="cuda"),
    }
    stream = torch.cuda.current_stream()

    def timed(opts):
        kw = dict(schedule="batched", precision=precision, **opts)
        lx.simulate(h, theta, x0, t_end, eps, mode, out=out, stream=stream, **kw)  # warm-up
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lx.simulate(h, theta, x0, t_end, eps, mode, out=out, stream=stream, **kw)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        return min(times)

    names = list(grid)
    table = []
    for values in itertools.product(*(grid[n] for n in names)):
        opts = dict(zip(names, values))
        if not valid(opts, P):
            continue
        ms = timed(opts)
        table.append((opts, ms))
        if log:
            log(f"[tune] {opts} {ms:.3f} ms")
    best = min(table, key=lambda t: t[1])[0]
    best, rows = refine(best, timed, log, large=getattr(h, "large", False))
    table += rows
    return best, table


# Knobs swept for a network set (lx_simulate_set): one lane per trajectory,
# the set's blocks sized by the scheduler.
# second stage: each value on top of the best setting, one knob at a time
REFINE = {
    "waves_per_simd": (1, 2, 3, 4),
    "tail_lanes": (4, 8, 16),
}


def refine(best, timed, log=None, large=False):
    """Try every REFINE value on top of `best` (a dict of options), keeping a
    value when it is faster; `timed(opts)` returns milliseconds.  Returns the
    new best and the rows tried.  `large`: a network beyond 16 x 32, which
    has no tail lane groups."""
    rows = []
    best_ms = timed(best)
    rows.append((dict(best), best_ms))
    for name, values in REFINE.items():
        if large and name == "tail_lanes":
            continue
        for v in values:
            opts = dict(best, **{name: v})
            if name == "tail_lanes" and opts.get("lanes_per_traj", 1) > 1:
                continue
            if name == "tail_lanes" and opts.get("regroup", 0):
                continue
            ms = timed(opts)
            rows.append((opts, ms))
            if log:
                log(f"[refine] {opts} {ms:.3f} ms")
            if ms < best_ms:
                best, best_ms = opts, ms
    return best, rows


SET_GRID = {
    "lanes_per_wave": (64,),
    "ssa_k": (4, 8, 16),
    "block_size": (128, 256),
    "blocks_per_cu": (2, 4, 6, 8),
}


def key_of_set(nets, P, precision, mode, arch="gfx950"):
    import numpy as np
    h = hashlib.sha1()
    for m, p in nets:
        h.update(np.ascontiguousarray(m, np.int32).tobytes())
        h.update(np.ascontiguousarray(p, np.int32).tobytes())
    return f"{arch}/set-{h.hexdigest()[:16]}/P{P}/{precision}/{mode}"


def lookup_set(nets, P, precision, mode, path=DEFAULT_FILE):
    """Tuned options for a network set ([(m, p), ...], P trajectories in
    total), or {} if it was never tuned."""
    return dict(load(path).get(key_of_set(nets, P, precision, mode), {}).get("options", {}))


def tune_set(lx, items, t_end, eps, mode, precision, grid=None, reps=1, log=None, start=None):
    """tune() for lx_simulate_set: ``items`` as for lx.simulate_set.  With
    `start` (options), the grid is skipped and only the refine stage runs
    from there."""
    import torch
    grid = grid or SET_GRID
    stream = torch.cuda.current_stream()
    names = list(grid)
    table = []
    outs = [None] * len(items)

    def run(kw):
        res = lx.simulate_set([dict(it, out=outs[k]) for k, it in enumerate(items)], t_end, eps,
                              mode, stream=stream, **kw)
        for k in range(len(items)):
            outs[k] = res[k]

    def timed(opts):
        kw = dict(precision=precision, **opts)
        run(kw)  # warm-up
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run(kw)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        return min(times)

    if start is None:
        for values in itertools.product(*(grid[n] for n in names)):
            opts = dict(zip(names, values))
            ms = timed(opts)
            table.append((opts, ms))
            if log:
                log(f"[tune] {opts} {ms:.3f} ms")
        best = min(table, key=lambda t: t[1])[0]
    else:
        best = {k: v for k, v in start.items() if k not in REFINE}
    best, rows = refine(best, timed, log)
    table += rows
    return best, table


def save(key, options, ms, table, path=DEFAULT_FILE):
    """Record the chosen knobs of `key`; the sweep itself (`table`) is printed
    by the tuner, not stored with the package."""
    data = load(path)
    data[key] = {"options": options, "ms": ms}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="dimer",
                    choices=("dimer", "birth_death", "telegraph", "mixed_set", "dimer_rathinam",
                             "random48x128", "stiff_padded45"))
    ap.add_argument("--t-end", type=float, default=0.0,
                    help="tune on a shorter horizon than the workload's (single networks)")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--out", default=DEFAULT_FILE)
    ap.add_argument("--grid", choices=("full", "small"), default="full",
                    help="knob grid of single-network ensembles")
    ap.add_argument("--refine-only", action="store_true",
                    help="start from the stored knobs of the ensemble and run only the refine stage")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_1608_07058_amd import lx, workloads as W
    if args.workload == "mixed_set":
        return main_set(args, torch, lx, W)
    wl = {"dimer": W.dimer_workload, "birth_death": W.birth_death_workload,
          "telegraph": W.telegraph_workload, "dimer_rathinam": W.rathinam_workload,
          "random48x128": W.random_network_workload,
          "stiff_padded45": W.stiff_padded_workload}[args.workload]()
    if args.t_end > 0.0:
        wl.t_end = args.t_end
    net = wl.nets[0]
    h = lx.Network(net.m, net.p)
    theta = torch.as_tensor(wl.theta[0], device="cuda")
    x0 = torch.as_tensor(wl.x0[0], device="cuda")
    best, table = tune(lx, h, theta, x0, wl.t_end, wl.eps, wl.mode, args.precision,
                       grid=(LARGE_GRID if h.large else
                             SMALL_GRID if args.grid == "small" else None),
                       log=lambda s: print(s, flush=True))
    ms = min(t for o, t in table if o == best)
    key = key_of(net.m, net.p, wl.P, args.precision, wl.mode, wl.theta[0], wl.x0[0])
    save(key, best, ms, table, args.out)
    print(json.dumps({"key": key, "best": best, "ms": ms}), flush=True)


def main_set(args, torch, lx, W):
    """Tune the three-network set of the mixed-set workload (particle p runs
    network p mod 3)."""
    wl = W.mixed_set_workload()
    hs = [lx.Network(n.m, n.p) for n in wl.nets]
    items = [{"net": h, "theta": torch.as_tensor(t, device="cuda"),
              "x0": torch.as_tensor(x, device="cuda"), "pid_base": k, "pid_stride": len(hs)}
             for k, (h, t, x) in enumerate(zip(hs, wl.theta, wl.x0))]
    key = key_of_set([(n.m, n.p) for n in wl.nets], wl.P, args.precision, wl.mode)
    start = load(args.out).get(key, {}).get("options") if args.refine_only else None
    best, table = tune_set(lx, items, wl.t_end, wl.eps, wl.mode, args.precision,
                           reps=2 if start else 1, log=lambda s: print(s, flush=True),
                           start=start)
    ms = min(t for o, t in table if o == best)
    save(key, best, ms, table, args.out)
    print(json.dumps({"key": key, "best": best, "ms": ms}), flush=True)


if __name__ == "__main__":
    main()
