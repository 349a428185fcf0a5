"""Ensembles of the moment-error table: the batched mixed-precision GPU path
against the binary64 oracle, every output (X, r, G) of every configuration.

Inputs only (networks, seeded parameters, initial states); no arithmetic of
the method.  The two sides use independent draws: different particle ids
(so different random streams) and, where parameters come from a prior,
different parameter samples.
"""

import numpy as np

from paper_1608_07058_amd import workloads as W

N_TRAJ = 100_000
ORACLE_PID_BASE = 1 << 30  # oracle particle ids start here, the GPU's at 0


def _tiled(net, P):
    return W.tile(net, P)


def _prior(net, P, seed):
    th = W.gamma_prior_theta(net, P, seed)
    x0 = np.ascontiguousarray(np.broadcast_to(net.x0, (P, net.N)), np.int32)
    return th, x0


# name -> (network factory, t_end, mode, inputs(P, side)); side is "gpu" or "oracle"
CONFIGS = {
    "birth-death (t 100, explicit)": (
        W.birth_death, 100.0, "explicit", lambda net, P, side: _tiled(net, P)),
    "decaying-dimerizing (t 30)": (
        W.dimer, 30.0, "adaptive", lambda net, P, side: _tiled(net, P)),
    "isomerisation, Gamma prior (t 50)": (
        W.isomerisation, 50.0, "adaptive",
        lambda net, P, side: _prior(net, P, 301 if side == "gpu" else 302)),
    "birth-death, Gamma prior (t 50)": (
        W.birth_death, 50.0, "adaptive",
        lambda net, P, side: _prior(net, P, 311 if side == "gpu" else 312)),
    "Schloegl, Gamma prior (t 50)": (
        W.schlogl, 50.0, "adaptive",
        lambda net, P, side: _prior(net, P, 321 if side == "gpu" else 322)),
    "random 48 x 128 network (t 1)": (
        W.random_network, 1.0, "adaptive", lambda net, P, side: _tiled(net, P)),
    "telegraph, Gamma prior, one interval (t 5)": (
        W.telegraph, 5.0, "adaptive",
        lambda net, P, side: _prior(net, P, 331 if side == "gpu" else 332)),
}


def inputs(name, side, P=N_TRAJ):
    make, t_end, mode, gen = CONFIGS[name]
    net = make()
    th, x0 = gen(net, P, side)
    pid_base = 0 if side == "gpu" else ORACLE_PID_BASE
    return net, th, x0, t_end, mode, pid_base


def outputs(res):
    """Columns of every output of status-OK trajectories: name -> values."""
    ok = res["stats"]["status"] == 0
    cols = {}
    for key in ("x", "r", "G"):
        a = res[key][ok]
        for c in range(a.shape[1]):
            cols[f"{key}[{c}]"] = a[:, c].astype(np.float64)
    return cols, int(ok.sum()), int((~ok).sum())


def moments(v):
    """n, mean, variance and fourth central moment of a sample."""
    m = float(v.mean())
    d = v - m
    return {"n": int(len(v)), "mean": m, "var": float((d * d).mean()),
            "m4": float((d ** 4).mean())}
