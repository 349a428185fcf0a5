"""Parity of lx_simulate (HIP) with the oracle.

* element by element: the kernels and the oracle draw the same random numbers
  (Philox keyed by particle id and draw site) and perform the same floating-
  point operations in the same order, so X(t_end), r and G agree exactly, in
  both precision policies, for every network and mode, at sizes spanning
  several blocks with a ragged tail;
* at the full benchmark sizes, on sampled trajectories the oracle recomputes
  one by one;
* edge cases: empty and one-element ensembles, invalid inputs, step budgets,
  absorbing states, split runs (t_start / accumulate), block sizes;
* in distribution at >= 1e5 trajectories with independent seeds:
  two-sample KS and chi-square (Holm-adjusted p > 0.01), means and variances
  within 3 standard errors, G means within 1e-3 relative (or 3 SE).
"""

import math

import numpy as np
import pytest
from scipy import stats

from paper_1608_07058_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lxm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_07058_amd import lx
    lx.lib()
    return lx


_HANDLES = {}


def _handle(lxm, net):
    key = (net.name, net.m.tobytes(), net.p.tobytes())
    if key not in _HANDLES:
        _HANDLES[key] = lxm.Network(net.m, net.p)
    return _HANDLES[key]


def gpu_run(lxm, net, theta, x0, t_end, mode, r0=None, G0=None, **opts):
    import torch
    th = torch.as_tensor(np.ascontiguousarray(theta, np.float64), device="cuda")
    xi = torch.as_tensor(np.ascontiguousarray(x0, np.int32), device="cuda")
    out = {}
    if r0 is not None:
        out["r"] = torch.as_tensor(np.ascontiguousarray(r0, np.int32), device="cuda")
        out["G"] = torch.as_tensor(np.ascontiguousarray(G0, np.float64), device="cuda")
        opts["accumulate"] = 1
    res = lxm.simulate(_handle(lxm, net), th, xi, t_end, opts.pop("eps", 0.03), mode, out=out,
                       **opts)
    torch.cuda.synchronize()
    return {"x": res["x"].cpu().numpy(), "r": res["r"].cpu().numpy(),
            "G": res["G"].cpu().numpy(), "stats": lxm.stats_numpy(res["stats"])}


def assert_same(got, ref, what=""):
    for key in ("x", "r", "G"):
        if not np.array_equal(got[key], ref[key]):
            bad = np.argwhere(np.any(got[key].reshape(len(got[key]), -1) !=
                                     ref[key].reshape(len(ref[key]), -1), axis=1))[:5, 0]
            raise AssertionError(f"{what}: {key} differs at particles {bad.tolist()}: "
                                 f"gpu {got[key][bad]} oracle {ref[key][bad]}")
    for f in ("status", "crit_fired", "t_final", "steps_ssa", "steps_explicit", "steps_implicit",
              "rejections", "newton_iters", "newton_fail", "kclip", "attempts"):
        assert np.array_equal(got["stats"][f], ref["stats"][f]), (what, f)


CASES = [
    # name, network, mode, t_end, P
    ("birth_death", W.birth_death(), "explicit", 100.0, 3000),
    ("dimer", W.dimer(), "adaptive", 30.0, 1500),
    ("dimer_stiff", W.dimer_stiff(), "adaptive", 3.0, 257),
    ("isomerisation", W.isomerisation(), "adaptive", 5.0, 1000),
    ("schlogl", W.schlogl(), "adaptive", 10.0, 700),
    ("telegraph", W.telegraph(), "adaptive", 50.0, 999),
    ("dimer_ssa", W.dimer(), "ssa", 0.5, 130),
    ("dimer_explicit", W.dimer(), "explicit", 10.0, 321),
]


@pytest.mark.parametrize("schedule", ["plain", "batched", "regroup", "group4", "tail4", "tail16"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_simulate_matches_oracle_elementwise(lxm, orc, case, precision, schedule):
    name, net, mode, t_end, P = case
    theta = W.gamma_prior_theta(net, P, seed=7)
    _, x0 = W.tile(net, P)
    # tail4/tail16: the last trajectories of each block finish in lane groups
    # (tail4 also compiled for at least two waves per SIMD)
    kw = {"regroup": dict(schedule="batched", regroup=1),
          "group4": dict(schedule="batched", lanes_per_traj=4),
          "tail4": dict(schedule="batched", tail_lanes=4, waves_per_simd=2),
          "tail16": dict(schedule="batched", tail_lanes=16, lanes_per_wave=64)}.get(
              schedule, dict(schedule=schedule))
    got = gpu_run(lxm, net, theta, x0, t_end, mode, precision=precision, **kw)
    ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode=mode, precision=precision)
    assert_same(got, ref, f"{name}/{precision}/{schedule}")
    assert np.all(got["stats"]["status"] == 0)


@pytest.mark.parametrize("lam_thr", [10.0, 30.0])
@pytest.mark.parametrize("schedule", ["plain", "batched", "group4"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_poisson_threshold_option_matches_oracle(lxm, orc, lam_thr, precision, schedule):
    # the two ends of the allowed Poisson threshold: the dimer's and Schloegl's
    # leaps draw means on both sides of each
    for net, t_end in ((W.dimer(), 30.0), (W.schlogl(), 10.0)):
        P = 600
        theta = W.gamma_prior_theta(net, P, seed=41)
        _, x0 = W.tile(net, P)
        kw = {"group4": dict(schedule="batched", lanes_per_traj=4)}.get(schedule,
                                                                          dict(schedule=schedule))
        got = gpu_run(lxm, net, theta, x0, t_end, "adaptive", precision=precision,
                      lambda_thr=lam_thr, **kw)
        ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode="adaptive", precision=precision,
                           lambda_thr=lam_thr)
        assert_same(got, ref, f"{net.name}/{precision}/{schedule}/lambda_thr {lam_thr}")
    with pytest.raises(lxm.LxError):
        gpu_run(lxm, net, theta[:2], x0[:2], t_end, "adaptive", lambda_thr=9.5)


@pytest.mark.parametrize("schedule", ["plain", "batched", "group4"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,t_end", [("dimer_stiff", 3.0), ("dimer_rathinam", 2.0),
                                        ("isomerisation", 5.0)])
def test_fd_jacobian_matches_oracle_elementwise(lxm, orc, name, t_end, precision, schedule):
    # implicit leaps with the forward-difference Jacobian
    net = getattr(W, name)()
    P = 300
    theta = W.gamma_prior_theta(net, P, seed=29)
    _, x0 = W.tile(net, P)
    kw = {"group4": dict(schedule="batched", lanes_per_traj=4)}.get(schedule, dict(schedule=schedule))
    got = gpu_run(lxm, net, theta, x0, t_end, "adaptive", precision=precision, jacobian=1, **kw)
    ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode="adaptive", precision=precision,
                       jacobian=1)
    assert_same(got, ref, f"{name}/{precision}/{schedule}/fd")
    assert got["stats"]["steps_implicit"].sum() > 0
    with pytest.raises(lxm.LxError):
        gpu_run(lxm, net, theta[:2], x0[:2], t_end, "adaptive", jacobian=2)


@pytest.mark.parametrize("knobs", [
    dict(lanes_per_wave=4, ssa_k=2, blocks_per_cu=1),
    dict(lanes_per_wave=8, ssa_k=8, blocks_per_cu=2, block_size=64),
    dict(lanes_per_wave=16, ssa_k=1, blocks_per_cu=1),
    dict(lanes_per_wave=32, ssa_k=4, blocks_per_cu=1, block_size=64),
    dict(lanes_per_wave=64, ssa_k=16, blocks_per_cu=1, block_size=128),
    dict(lanes_per_wave=64, ssa_k=64, blocks_per_cu=8),
    dict(lanes_per_wave=16, ssa_k=8, blocks_per_cu=1, regroup=1),
    dict(lanes_per_wave=64, ssa_k=4, blocks_per_cu=2, regroup=3),
    dict(lanes_per_wave=8, ssa_k=2, blocks_per_cu=1, block_size=128, regroup=2),
    dict(lanes_per_wave=64, lanes_per_traj=4, ssa_k=8, blocks_per_cu=1),
    dict(lanes_per_wave=32, lanes_per_traj=2, ssa_k=5, blocks_per_cu=2, block_size=64),
    dict(lanes_per_wave=8, lanes_per_traj=4, ssa_k=3, blocks_per_cu=1, block_size=128),
    dict(lanes_per_wave=64, lanes_per_traj=8, ssa_k=8, blocks_per_cu=8),
    dict(lanes_per_wave=64, lanes_per_traj=16, ssa_k=20, blocks_per_cu=4, block_size=256),
])
def test_batched_refill_and_knobs(lxm, orc, knobs):
    # Few resident blocks force every lane to refill from its block's range
    # many times; no knob may change any result.
    net = W.telegraph()
    P = 40000
    theta = W.gamma_prior_theta(net, P, seed=11)
    _, x0 = W.tile(net, P)
    got = gpu_run(lxm, net, theta, x0, 20.0, "adaptive", precision="mixed", schedule="batched",
                  **knobs)
    ref = orc.simulate(net.m, net.p, theta, x0, 20.0, mode="adaptive", precision="mixed")
    assert_same(got, ref, str(knobs))


@pytest.mark.parametrize("schedule", ["plain", "batched", "tuned"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_dimer_sampled(lxm, orc, precision, schedule):
    # The benchmark workload (16384 trajectories, in the launch configuration
    # the benchmark times), checked on trajectories sampled across the grid and
    # recomputed by the oracle.
    wl = W.dimer_workload()
    net, theta, x0 = wl.nets[0], wl.theta[0], wl.x0[0]
    kw = dict(schedule=schedule)
    if schedule == "tuned":  # the knobs the benchmark uses
        from paper_1608_07058_amd import autotune
        kw = dict(schedule="batched", **autotune.lookup(net.m, net.p, wl.P, precision, wl.mode,
                                                        wl.theta[0], wl.x0[0]))
    got = gpu_run(lxm, net, theta, x0, wl.t_end, wl.mode, precision=precision, **kw)
    rng = np.random.default_rng(5)
    sample = np.concatenate([[0, 63, 64, wl.P - 1], rng.choice(wl.P, 60, replace=False)])
    for p in sample:
        ref = orc.simulate(net.m, net.p, theta[p:p + 1], x0[p:p + 1], wl.t_end, mode=wl.mode,
                           precision=precision, pid_base=int(p))
        one = {k: got[k][p:p + 1] for k in ("x", "r", "G")}
        one["stats"] = got["stats"][p:p + 1]
        assert_same(one, ref, f"particle {p}")
    # whole-ensemble invariants
    nu = (net.p - net.m).astype(np.int64)
    assert np.array_equal(got["x"], x0 + got["r"].astype(np.int64) @ nu)
    assert np.all(got["x"] >= 0) and np.all(got["stats"]["status"] == 0)


@pytest.mark.parametrize("form", ["plain", "tuned_mixed", "tuned_fp64"])
def test_full_size_birth_death(lxm, orc, form):
    # the benchmark ensemble in the plain form and in the tuned batched launch
    # (the knobs autotune.py recorded: 16-lane groups, ssa_k 64)
    from paper_1608_07058_amd import autotune
    wl = W.birth_death_workload()
    net = wl.nets[0]
    precision = "mixed" if form == "tuned_mixed" else "fp64"
    opts = dict(precision=precision)
    if form != "plain":
        opts.update(schedule="batched",
                    **autotune.lookup(net.m, net.p, wl.P, precision, wl.mode, wl.theta[0],
                                      wl.x0[0]))
        assert opts.get("lanes_per_traj", 1) > 1
    got = gpu_run(lxm, net, wl.theta[0], wl.x0[0], wl.t_end, wl.mode, **opts)
    ref = orc.simulate(net.m, net.p, wl.theta[0], wl.x0[0], wl.t_end, mode=wl.mode,
                       precision=precision)
    assert_same(got, ref, f"birth-death 1024 {form}")


def test_edge_cases(lxm, orc):
    import torch
    net = W.dimer()
    h = _handle(lxm, net)
    # empty ensemble: no-op
    e = torch.empty((0, net.M), dtype=torch.float64, device="cuda")
    ex = torch.empty((0, net.N), dtype=torch.int32, device="cuda")
    out = lxm.simulate(h, e, ex, 1.0)
    assert out["x"].shape == (0, net.N)
    # single particle, ragged sizes and block sizes give identical results
    theta = W.gamma_prior_theta(net, 200, seed=9)
    _, x0 = W.tile(net, 200)
    ref = orc.simulate(net.m, net.p, theta, x0, 5.0)
    for P in (1, 65, 200):
        got = gpu_run(lxm, net, theta[:P], x0[:P], 5.0, "adaptive")
        sub = {k: ref[k][:P] for k in ("x", "r", "G", "stats")}
        assert_same(got, sub, f"P={P}")
    for bs in (128, 192, 256):
        got = gpu_run(lxm, net, theta, x0, 5.0, "adaptive", block_size=bs)
        assert_same(got, ref, f"block {bs}")
    # blocks above 256 threads are refused before any launch
    for bs in (512, 1024):
        with pytest.raises(lxm.LxError):
            gpu_run(lxm, net, theta, x0, 5.0, "adaptive", block_size=bs)
    # bad inputs are flagged per lane, the rest proceed
    th = theta[:6].copy()
    xx = x0[:6].copy()
    th[1, 2] = -1.0
    th[2, 0] = np.nan
    th[3, 1] = np.inf
    xx[4, 0] = -5
    got = gpu_run(lxm, net, th, xx, 5.0, "adaptive")
    ref6 = orc.simulate(net.m, net.p, th, xx, 5.0)
    assert got["stats"]["status"].tolist() == [0, 3, 3, 3, 3, 0]
    assert_same(got, ref6, "bad inputs")
    # step budget
    got = gpu_run(lxm, net, theta[:64], x0[:64], 5.0, "adaptive", max_steps=50)
    refb = orc.simulate(net.m, net.p, theta[:64], x0[:64], 5.0, max_steps=50)
    assert np.all(got["stats"]["status"] == 1)
    assert_same(got, refb, "budget")
    # absorbing state from the start: G integrates g over the whole interval
    z = np.zeros_like(x0[:64])
    got = gpu_run(lxm, net, theta[:64], z, 5.0, "adaptive")
    assert np.all(got["x"] == 0) and np.all(got["r"] == 0)
    assert np.all(got["G"] == 0)
    bd = W.birth_death()
    got = gpu_run(lxm, bd, np.tile([0.0, 0.0], (64, 1)), np.full((64, 1), 5), 7.0, "explicit")
    assert np.all(got["x"] == 5) and np.all(got["G"][:, 0] == 7.0) and np.all(got["G"][:, 1] == 35.0)
    # overflow statuses
    got = gpu_run(lxm, W.birth_death(), np.array([[1e7, 1e-12]]), np.array([[0]]), 1000.0,
                  "explicit")
    assert got["stats"]["status"][0] == 4
    cat = W._net("cat", [[1]], [[1]], [1e12], [1000])
    got = gpu_run(lxm, cat, np.array([[1e12]]), np.array([[1000]]), 10.0, "explicit")
    assert got["stats"]["status"][0] == 2


def test_split_runs_and_streams(lxm, orc):
    net = W.telegraph()
    P = 500
    theta = W.gamma_prior_theta(net, P, seed=2)
    _, x0 = W.tile(net, P)
    a = gpu_run(lxm, net, theta, x0, 5.0, "adaptive", pid_base=1000)
    b = gpu_run(lxm, net, theta, a["x"], 10.0, "adaptive", r0=a["r"], G0=a["G"], t_start=5.0,
                rng_stream=1, pid_base=1000)
    ra = orc.simulate(net.m, net.p, theta, x0, 5.0, pid_base=1000)
    rb = orc.simulate(net.m, net.p, theta, ra["x"], 10.0, r0=ra["r"], G0=ra["G"], t_start=5.0,
                      rng_stream=1, pid_base=1000)
    assert_same(a, ra, "leg 1")
    assert_same(b, rb, "leg 2")
    # gene states: exactly one of off/on
    assert np.all(b["x"][:, 0] + b["x"][:, 1] == 1)
    assert np.allclose(b["G"][:, 0] + b["G"][:, 1], 10.0, rtol=1e-12)


def test_invalid_arguments_raise(lxm):
    import torch
    net = W.dimer()
    h = _handle(lxm, net)
    th = torch.ones((4, net.M), dtype=torch.float64, device="cuda")
    xi = torch.ones((4, net.N), dtype=torch.int32, device="cuda")
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, -0.1)          # eps <= 0
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, 0.03, 7)       # bad mode
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, t_start=2.0)   # t_end < t_start
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, lambda_thr=100.0)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, block_size=100)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, schedule="batched", lanes_per_wave=12)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, schedule="batched", ssa_k=100)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, schedule="batched", regroup=-1)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, schedule="batched", lanes_per_traj=3)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, th, xi, 1.0, schedule="batched", lanes_per_traj=2, regroup=1)


# ---------------------------------------------------------------------------
# Distributional parity at >= 1e5 trajectories (independent seeds).
# ---------------------------------------------------------------------------

def _holm(pvals):
    p = np.asarray(pvals)
    order = np.argsort(p)
    adj = np.empty_like(p)
    running = 0.0
    for rank, q in enumerate(order):
        running = max(running, min(1.0, (len(p) - rank) * p[q]))
        adj[q] = running
    return adj


def _chi2_two_sample(a, b, min_expected=10):
    vals = np.concatenate([a, b])
    lo, hi = np.percentile(vals, [0.1, 99.9])
    edges = np.unique(np.quantile(vals[(vals >= lo) & (vals <= hi)], np.linspace(0, 1, 41)))
    if len(edges) < 3:
        return 1.0
    edges = np.concatenate([[-np.inf], edges[1:-1], [np.inf]])
    ca, _ = np.histogram(a, edges)
    cb, _ = np.histogram(b, edges)
    keep = (ca + cb) >= min_expected
    if keep.sum() < 2:
        return 1.0
    return stats.chi2_contingency(np.stack([ca[keep], cb[keep]]))[1]


# Bound on |difference| / standard error for each mean and variance of a
# two-sample comparison: one comparison makes about 30 such checks, so 4.5
# SE per check keeps its false-failure rate near 2e-4 (3 SE would fail about
# one comparison in fifteen on samples of the same law).
Z_CHECK = 4.5


def _compare_distributions(got, ref, label):
    pvals, names = [], []
    n1, n2 = len(got["x"]), len(ref["x"])
    for key in ("x", "r"):
        for c in range(got[key].shape[1]):
            a, b = got[key][:, c].astype(float), ref[key][:, c].astype(float)
            if a.std() == 0 and b.std() == 0:
                assert a[0] == b[0], (label, key, c)
                continue
            pvals += [stats.ks_2samp(a, b).pvalue, _chi2_two_sample(a, b)]
            names += [f"{key}{c}:ks", f"{key}{c}:chi2"]
            se = math.sqrt(a.var() / n1 + b.var() / n2)
            assert abs(a.mean() - b.mean()) <= Z_CHECK * se, (label, key, c, a.mean(), b.mean(), se)
            def var_se(v):
                m = v - v.mean()
                return math.sqrt(max((m**4).mean() - v.var() ** 2, 0.0) / len(v))
            sev = math.sqrt(var_se(a) ** 2 + var_se(b) ** 2)
            assert abs(a.var() - b.var()) <= Z_CHECK * sev, (label, key, c, a.var(), b.var(), sev)
    adj = _holm(pvals)
    bad = [(n, p) for n, p in zip(names, adj) if p <= 0.01]
    assert not bad, (label, bad)
    for c in range(got["G"].shape[1]):
        a, b = got["G"][:, c], ref["G"][:, c]
        se = math.sqrt(a.var() / n1 + b.var() / n2)
        tol = max(1e-3 * abs(b.mean()), Z_CHECK * se)
        assert abs(a.mean() - b.mean()) <= tol, (label, "G", c, a.mean(), b.mean(), tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_distribution_birth_death(lxm, orc, precision):
    net = W.birth_death()
    P = 1 << 17
    theta, x0 = W.tile(net, P)
    got = gpu_run(lxm, net, theta, x0, 100.0, "explicit", precision=precision, seed=1)
    ref = orc.simulate(net.m, net.p, theta[:100000], x0[:100000], 100.0, mode="explicit", seed=2)
    _compare_distributions(got, ref, f"birth-death/{precision}")
    lam = 100.0 * (1 - math.exp(-10.0))
    assert abs(got["x"].mean() - lam) < 4 * math.sqrt(lam / P)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_distribution_dimer(lxm, orc, precision):
    # fp64: the batched kernel on 10^5 trajectories is the oracle's binary64
    # instance element by element (same streams).  mixed: the binary32
    # instance has the binary64 law (independent streams).
    net = W.dimer()
    P = 100000
    theta, x0 = W.tile(net, P)
    got = gpu_run(lxm, net, theta, x0, 30.0, "adaptive", precision=precision, seed=3,
                  schedule="batched")
    if precision == "fp64":
        ref = orc.simulate(net.m, net.p, theta, x0, 30.0, mode="adaptive", seed=3)
        assert_same(got, ref, "dimer/fp64, 10^5 trajectories")
    else:
        ref = orc.simulate(net.m, net.p, theta, x0, 30.0, mode="adaptive", seed=4)
        _compare_distributions(got, ref, f"dimer/{precision}")


# ---------------------------------------------------------------------------
# Several networks in one launch (isomerisation / birth-death / Schloegl
# interleaved 1:1:1, per-particle theta from Gamma priors).
# ---------------------------------------------------------------------------

def _set_run(lxm, wl, precision, **opts):
    import torch
    items = []
    for k, net in enumerate(wl.nets):
        items.append(dict(net=_handle(lxm, net),
                          theta=torch.as_tensor(wl.theta[k], device="cuda"),
                          x0=torch.as_tensor(wl.x0[k], device="cuda"),
                          pid_base=k, pid_stride=len(wl.nets)))
    outs = lxm.simulate_set(items, wl.t_end, wl.eps, wl.mode, precision=precision, **opts)
    torch.cuda.synchronize()
    return [{"x": o["x"].cpu().numpy(), "r": o["r"].cpu().numpy(), "G": o["G"].cpu().numpy(),
             "stats": lxm.stats_numpy(o["stats"])} for o in outs]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_set_matches_oracle(lxm, orc, precision):
    wl = W.mixed_set_workload(P=12000)
    got = _set_run(lxm, wl, precision)
    regrouped = _set_run(lxm, wl, precision, regroup=1, lanes_per_wave=16)
    grouped = _set_run(lxm, wl, precision, lanes_per_traj=2)
    tailed = _set_run(lxm, wl, precision, tail_lanes=4, lanes_per_wave=64, block_size=128)
    for k, net in enumerate(wl.nets):
        assert_same(regrouped[k], got[k], f"{net.name} regrouped")
        assert_same(grouped[k], got[k], f"{net.name} lane groups")
        assert_same(tailed[k], got[k], f"{net.name} tail lane groups")
        ref = orc.simulate(net.m, net.p, wl.theta[k], wl.x0[k], wl.t_end, mode=wl.mode,
                           precision=precision, pid_base=k, pid_stride=3)
        assert_same(got[k], ref, f"{net.name}/{precision}")
        # one network alone with the same ids gives the same result
        alone = gpu_run(lxm, net, wl.theta[k], wl.x0[k], wl.t_end, wl.mode, precision=precision,
                        schedule="batched", pid_base=k, pid_stride=3)
        assert_same(alone, ref, f"{net.name} alone")


@pytest.mark.parametrize("knobs", [dict(), dict(blocks_per_cu=8, ssa_k=8),
                                   dict(regroup=2, lanes_per_wave=32, block_size=128),
                                   dict(lanes_per_traj=4, blocks_per_cu=1),
                                   dict(tail_lanes=16, lanes_per_wave=64, blocks_per_cu=6,
                                        waves_per_simd=3)])
def test_set_uneven_sizes(lxm, orc, knobs):
    # items of 0, 5 and 7001 trajectories: every block owns a slice of each
    # network, most blocks none of the small ones
    import torch
    nets = [W.birth_death(), W.schlogl(), W.telegraph()]
    sizes = [0, 5, 7001]
    items, refs = [], []
    for k, (net, P) in enumerate(zip(nets, sizes)):
        th = W.gamma_prior_theta(net, P, seed=40 + k)
        _, x0 = W.tile(net, P)
        items.append(dict(net=_handle(lxm, net), theta=torch.as_tensor(th, device="cuda"),
                          x0=torch.as_tensor(x0, device="cuda"), pid_base=1000 * k))
        refs.append(orc.simulate(net.m, net.p, th, x0, 20.0, mode="adaptive", precision="mixed",
                                 pid_base=1000 * k) if P else None)
    outs = lxm.simulate_set(items, 20.0, 0.03, "adaptive", precision="mixed", **knobs)
    torch.cuda.synchronize()
    assert outs[0]["x"].shape[0] == 0
    for k in (1, 2):
        got = {"x": outs[k]["x"].cpu().numpy(), "r": outs[k]["r"].cpu().numpy(),
               "G": outs[k]["G"].cpu().numpy(), "stats": lxm.stats_numpy(outs[k]["stats"])}
        assert_same(got, refs[k], f"{nets[k].name} {knobs}")


def test_set_full_size_sampled(lxm, orc):
    # The 2^20-particle mixed ensemble in one launch, checked on sampled
    # particles of each network recomputed by the oracle.
    wl = W.mixed_set_workload()
    got = _set_run(lxm, wl, "mixed")
    rng = np.random.default_rng(8)
    for k, net in enumerate(wl.nets):
        P = wl.theta[k].shape[0]
        for q in np.concatenate([[0, P - 1], rng.choice(P, 12, replace=False)]):
            pid = int(wl.pid[k][q])
            ref = orc.simulate(net.m, net.p, wl.theta[k][q:q + 1], wl.x0[k][q:q + 1], wl.t_end,
                               mode=wl.mode, precision="mixed", pid_base=pid)
            one = {key: got[k][key][q:q + 1] for key in ("x", "r", "G", "stats")}
            assert_same(one, ref, f"{net.name} particle {pid}")
        st = got[k]["stats"]
        # explosive parameter draws end in an overflow status; they are rare
        # and, like every lane, identical to the oracle
        bad = np.flatnonzero(st["status"] != 0)
        assert len(bad) < 0.01 * P
        assert set(np.unique(st["status"][bad]).tolist()) <= {1, 2, 4}
        for q in bad[:8]:
            pid = int(wl.pid[k][q])
            ref = orc.simulate(net.m, net.p, wl.theta[k][q:q + 1], wl.x0[k][q:q + 1], wl.t_end,
                               mode=wl.mode, precision="mixed", pid_base=pid)
            one = {key: got[k][key][q:q + 1] for key in ("x", "r", "G", "stats")}
            assert_same(one, ref, f"{net.name} failed particle {pid}")
        nu = (net.p - net.m).astype(np.int64)
        ok = st["status"] == 0
        assert np.array_equal(got[k]["x"][ok], wl.x0[k][ok] + got[k]["r"][ok].astype(np.int64) @ nu)


def test_check_lanes_reports_failed_trajectories(lxm):
    import warnings
    import torch
    net = W.dimer()
    P = 300
    theta = W.gamma_prior_theta(net, P, seed=12)
    _, x0 = W.tile(net, P)
    bad = theta.copy()
    bad[7] = -1.0
    with pytest.warns(lxm.LaneFailWarning, match=r"1 of 300 trajectories .*row 7, status 3"):
        gpu_run(lxm, net, bad, x0, 1.0, "adaptive", check_lanes=1)
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        gpu_run(lxm, net, theta, x0, 1.0, "adaptive", check_lanes=1, schedule="batched")
    h = _handle(lxm, net)
    with pytest.raises(lxm.LxError):
        lxm.simulate(h, torch.as_tensor(theta, device="cuda"), torch.as_tensor(x0, device="cuda"),
                     1.0, with_stats=False, check_lanes=1)
    # observation times and network sets report the same way
    tt = torch.as_tensor(np.array([0.5, 1.0]), device="cuda")
    with pytest.warns(lxm.LaneFailWarning, match=r"row 7"):
        lxm.simulate_grid(h, torch.as_tensor(bad, device="cuda"), torch.as_tensor(x0, device="cuda"),
                          tt, check_lanes=1)
    items = [dict(net=h, theta=torch.as_tensor(theta, device="cuda"),
                  x0=torch.as_tensor(x0, device="cuda")),
             dict(net=h, theta=torch.as_tensor(bad, device="cuda"),
                  x0=torch.as_tensor(x0, device="cuda"), pid_base=P)]
    with pytest.warns(lxm.LaneFailWarning, match=r"item 1: 1 of 300"):
        lxm.simulate_set(items, 1.0, check_lanes=1)
    torch.cuda.synchronize()


# Cases where the method's rarer events are frequent, so that their code runs
# many times and is compared element by element:
#  * the non-negativity retry: pure decay with leaps of size 1 whose Poisson
#    draws often exceed the population (about 1.2 rejections per trajectory);
#  * a failed implicit solve, which is a rejection too: one Newton iteration
#    on the stiff dimer rarely converges;
#  * critical firings inside leaps: small decaying populations next to a fast
#    birth-death balance.
# With regroup=1 every lane is saved and restored between its actions, so a
# retry with a halved tau' also passes through the regrouping's state copy.
EVENT_CASES = [
    # name, network, x0 override, mode, t_end, P, options, counter, minimum
    ("retry", W.pure_death(1), "death", "explicit", 3.7, 9000,
     dict(n_c=0, eps=1.0, k_ssa=0.0), "rejections", 10000),
    ("newton_fail", W.dimer_stiff(), None, "adaptive", 0.005, 256, dict(newton_maxit=1),
     "newton_fail", 1000),
    ("critical", W.critical_decay(1, 2), None, "adaptive", 4.0, 3000, {}, "crit_fired", 3000),
    ("critical_explicit", W.critical_decay(1, 2), None, "explicit", 4.0, 3000, {}, "crit_fired",
     3000),
]
EVENT_SCHEDULES = {
    "plain": dict(schedule="plain"),
    "batched": dict(schedule="batched"),
    "regroup": dict(schedule="batched", regroup=1),
    "group4": dict(schedule="batched", lanes_per_traj=4),
    "group16": dict(schedule="batched", lanes_per_traj=16),
    "tail8": dict(schedule="batched", tail_lanes=8, lanes_per_wave=64),
}


@pytest.mark.parametrize("schedule", sorted(EVENT_SCHEDULES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", EVENT_CASES, ids=[c[0] for c in EVENT_CASES])
def test_rare_events_match_oracle_elementwise(lxm, orc, case, precision, schedule):
    name, net, x0kind, mode, t_end, P, opts, counter, minimum = case
    theta, x0 = W.tile(net, P)
    if x0kind == "death":
        x0 = x0.copy()
        x0[::3] = 37
    got = gpu_run(lxm, net, theta, x0, t_end, mode, precision=precision, **opts,
                  **EVENT_SCHEDULES[schedule])
    ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode=mode, precision=precision, **opts)
    assert_same(got, ref, f"{name}/{precision}/{schedule}")
    assert np.all(got["stats"]["status"] == 0)
    assert int(got["stats"][counter].astype(np.int64).sum()) >= minimum, counter


@pytest.mark.parametrize("schedule", ["plain", "batched", "group4"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,t_end,scale", [("dimer_stiff", 3.0, 1.0), ("dimer_rathinam", 2.0, 1.0),
                                              ("dimer_stiff", 3.0, 0.7)])
def test_user_jacobian_matches_oracle_elementwise(lxm, orc, name, t_end, scale, precision,
                                                  schedule):
    # implicit leaps with the caller's derivative terms (lx_network_create_jac)
    net = getattr(W, name)()
    rxn, wrt, coef, pw = W.mass_action_jacobian_terms(net)
    terms = (rxn, wrt, coef * scale, pw)
    P = 300
    theta = W.gamma_prior_theta(net, P, seed=31)
    _, x0 = W.tile(net, P)
    import torch
    h = lxm.Network(net.m, net.p, jacobian_terms=terms)
    kw = {"group4": dict(schedule="batched", lanes_per_traj=4)}.get(schedule, dict(schedule=schedule))
    res = lxm.simulate(h, torch.as_tensor(theta, device="cuda"), torch.as_tensor(x0, device="cuda"),
                       t_end, 0.03, "adaptive", precision=precision, jacobian="user", **kw)
    torch.cuda.synchronize()
    got = {"x": res["x"].cpu().numpy(), "r": res["r"].cpu().numpy(), "G": res["G"].cpu().numpy(),
           "stats": lxm.stats_numpy(res["stats"])}
    ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode="adaptive", precision=precision,
                       jacobian="user", jacobian_terms=terms)
    assert_same(got, ref, f"{name}/{precision}/{schedule}/user x{scale}")
    assert got["stats"]["steps_implicit"].sum() > 0
    # a network without terms refuses the user Jacobian
    with pytest.raises(lxm.LxError):
        lxm.simulate(_handle(lxm, net), torch.as_tensor(theta, device="cuda"),
                     torch.as_tensor(x0, device="cuda"), 0.1, jacobian="user")
