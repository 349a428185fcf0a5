"""Write tests/golden/moments_fp64.json: per-output moments (n, mean, variance,
fourth central moment) of the binary64 oracle over 10^5 trajectories of each
ensemble in tests/moment_configs.py.  Calls only the oracle.

    python tests/golden/make_moments.py [--threads 8]
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import moment_configs as MC  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--only", default="", help="substring of the configurations to redo")
    args = ap.parse_args()
    path = os.path.join(HERE, "moments_fp64.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for name in MC.CONFIGS:
        if args.only and args.only not in name:
            continue
        net, th, x0, t_end, mode, pid_base = MC.inputs(name, "oracle")
        t0 = time.time()
        res = oracle.simulate(net.m, net.p, th, x0, t_end, mode=mode, precision="fp64",
                              pid_base=pid_base, nthreads=args.threads)
        cols, n_ok, n_bad = MC.outputs(res)
        data[name] = {"trajectories": int(th.shape[0]), "excluded": n_bad,
                      "outputs": {k: MC.moments(v) for k, v in cols.items()}}
        print(f"{name}: {time.time() - t0:.1f} s, {n_bad} trajectories not OK", flush=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
