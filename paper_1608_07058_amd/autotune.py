"""Autotuner for the batched schedule.

Sweeps the launch knobs of ``lx_simulate`` (active lanes per wave, SSA steps
per leap iteration, block size, resident blocks per CU) on a given ensemble,
times each setting with HIP events on the launch stream, and keeps the
fastest.  The knobs never change results (every trajectory's actions are
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
    "ssa_k": (4, 8, 16),
    "block_size": (64, 256),
    "blocks_per_cu": (2, 4),
    "regroup": (0,),
}


def valid(opts, P):
    tpl = opts.get("lanes_per_traj", 1)
    if tpl > 1 and opts.get("regroup", 0):
        return False
    if opts["lanes_per_wave"] < tpl:
        return False
    return (opts["lanes_per_wave"] // tpl) * (opts["block_size"] // 64) <= P


def key_of(net_m, net_p, P, precision, mode, arch="gfx950"):
    import numpy as np
    h = hashlib.sha1(np.ascontiguousarray(net_m, np.int32).tobytes() +
                     np.ascontiguousarray(net_p, np.int32).tobytes()).hexdigest()[:16]
    return f"{arch}/{h}/P{P}/{precision}/{mode}"


def load(path=DEFAULT_FILE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(net_m, net_p, P, precision, mode, path=DEFAULT_FILE):
    """Tuned options for this ensemble, or {} if it was never tuned."""
    return dict(load(path).get(key_of(net_m, net_p, P, precision, mode), {}).get("options", {}))


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
    names = list(grid)
    table = []
    for values in itertools.product(*(grid[n] for n in names)):
        opts = dict(zip(names, values))
        if not valid(opts, P):
            continue
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
        ms = min(times)
        table.append((opts, ms))
        if log:
            log(f"[tune] {opts} {ms:.3f} ms")
    best = min(table, key=lambda t: t[1])
    return best[0], table


def save(key, options, ms, table, path=DEFAULT_FILE):
    data = load(path)
    data[key] = {"options": options, "ms": ms,
                 "sweep": [{"options": o, "ms": t} for o, t in table]}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="dimer", choices=("dimer", "birth_death", "telegraph"))
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--out", default=DEFAULT_FILE)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_1608_07058_amd import lx, workloads as W
    wl = {"dimer": W.dimer_workload, "birth_death": W.birth_death_workload,
          "telegraph": W.telegraph_workload}[args.workload]()
    net = wl.nets[0]
    h = lx.Network(net.m, net.p)
    theta = torch.as_tensor(wl.theta[0], device="cuda")
    x0 = torch.as_tensor(wl.x0[0], device="cuda")
    best, table = tune(lx, h, theta, x0, wl.t_end, wl.eps, wl.mode, args.precision,
                       log=lambda s: print(s, flush=True))
    ms = min(t for _, t in table)
    key = key_of(net.m, net.p, wl.P, args.precision, wl.mode)
    save(key, best, ms, table, args.out)
    print(json.dumps({"key": key, "best": best, "ms": ms}), flush=True)


if __name__ == "__main__":
    main()
