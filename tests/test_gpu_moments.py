"""Moment error of every output of the batched mixed-precision path against the
binary64 oracle, 10^5 trajectories per ensemble on each side, independent
draws (tests/moment_configs.py; the oracle's moments are stored in
tests/golden/moments_fp64.json by tests/golden/make_moments.py).

For every output (each species of X, each r_j and G_j) the relative error of
the mean and of the variance is stated with its standard error; each must lie
within 4.5 standard errors (about 70 outputs: a false alarm has probability
below 1e-3 per run), and a constant output must be equal.  With
LX_MOMENTS_OUT set, the table is written there as markdown.
"""

import json
import math
import os

import numpy as np
import pytest

import moment_configs as MC

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "moments_fp64.json")


@pytest.fixture(scope="module")
def lxm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_07058_amd import lx
    lx.lib()
    return lx


def _rel(g, o):
    """Relative errors of mean and variance, their standard errors."""
    scale_m = abs(o["mean"]) if o["mean"] != 0 else 1.0
    dm = (g["mean"] - o["mean"]) / scale_m
    se_m = math.sqrt(g["var"] / g["n"] + o["var"] / o["n"]) / scale_m
    if o["var"] > 0:
        dv = (g["var"] - o["var"]) / o["var"]
        se_v = math.sqrt(max(g["m4"] - g["var"] ** 2, 0.0) / g["n"]
                         + max(o["m4"] - o["var"] ** 2, 0.0) / o["n"]) / o["var"]
    else:
        dv, se_v = (0.0 if g["var"] == 0 else math.inf), 0.0
    return dm, se_m, dv, se_v


def test_moment_error_of_every_output(lxm):
    import torch
    ref = json.load(open(GOLDEN))
    rows, bad = [], []
    for name in MC.CONFIGS:
        net, th, x0, t_end, mode, pid_base = MC.inputs(name, "gpu")
        h = lxm.Network(net.m, net.p)
        res = lxm.simulate(h, torch.as_tensor(th, device="cuda"),
                           torch.as_tensor(x0, device="cuda"), t_end, 0.03, mode,
                           precision="mixed", schedule="batched", pid_base=pid_base)
        torch.cuda.synchronize()
        got = {"x": res["x"].cpu().numpy(), "r": res["r"].cpu().numpy(),
               "G": res["G"].cpu().numpy(), "stats": lxm.stats_numpy(res["stats"])}
        h.close()
        cols, n_ok, n_bad = MC.outputs(got)
        r = ref[name]
        for out, v in cols.items():
            g, o = MC.moments(v), r["outputs"][out]
            dm, se_m, dv, se_v = _rel(g, o)
            if o["var"] == 0 and g["var"] == 0:
                ok = abs(dm) <= 1e-12
            else:
                ok = abs(dm) <= 4.5 * se_m and abs(dv) <= 4.5 * se_v
            rows.append((name, out, g["n"], o["n"], o["mean"], dm, se_m, o["var"], dv, se_v, ok))
            if not ok:
                bad.append((name, out, dm, se_m, dv, se_v))
        rows.append((name, f"({n_bad} GPU / {r['excluded']} oracle trajectories not OK)",
                     None, None, None, None, None, None, None, None, True))
    path = os.environ.get("LX_MOMENTS_OUT")
    if path:
        with open(path, "w") as f:
            f.write("| ensemble | output | n GPU | n oracle | oracle mean | rel. err. of mean "
                    "(± SE) | oracle variance | rel. err. of variance (± SE) |\n"
                    "|---|---|---|---|---|---|---|---|\n")
            for (name, out, ng, no, om, dm, sm, ov, dv, sv, ok) in rows:
                if ng is None:
                    f.write(f"| {name} | {out} | | | | | | |\n")
                    continue
                f.write(f"| {name} | {out} | {ng} | {no} | {om:.6g} | {dm:+.2e} ± {sm:.1e} | "
                        f"{ov:.6g} | {dv:+.2e} ± {sv:.1e} |\n")
    assert not bad, bad
