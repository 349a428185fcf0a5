"""Pins for the oracle's observation-time output (simulate_grid).

* exact SSA states at the observation times follow the closed-form laws of
  linear networks: immigration-death from 0 is Poisson with mean
  (k1/k2)(1 - exp(-k2 t)); isomerisation A <-> B (rates 1, 1) from n copies
  of A leaves A ~ Binomial(n, (1 + exp(-2t))/2);
* the trajectory goes on through an observation time (it is not restarted):
  in immigration-death E[X(t2) | X(t1)] = X(t1) exp(-k2 (t2 - t1)) + const,
  so the regression slope of X(t2) on X(t1) is exp(-k2 (t2 - t1)) (0 for
  independent draws);
* structure: one time at t_end is simulate(); a time at t_start records x0;
  repeated times record equal rows; the last row is X(t_end); conservation
  holds on every row; invalid times and lanes give -1 rows and BAD_INPUT.
"""

import numpy as np
import pytest
from scipy import stats

from paper_1608_07058_amd import workloads as W


def _chi2_discrete(samples, dist):
    """p-value of a chi-square fit of integer samples to a scipy discrete law,
    with tail classes merged so that every class expects >= 20."""
    n = samples.size
    lo, hi = int(dist.ppf(1e-4)), int(dist.ppf(1 - 1e-4))
    ks = np.arange(lo, hi + 1)
    exp = n * dist.pmf(ks)
    exp[0] += n * dist.cdf(lo - 1)
    exp[-1] += n * dist.sf(hi)
    obs = np.bincount(np.clip(samples, lo, hi) - lo, minlength=ks.size).astype(float)
    # merge classes from both ends until every class expects >= 20
    o, e = list(obs), list(exp)
    while len(e) > 2 and e[0] < 20:
        ve, vo = e.pop(0), o.pop(0)
        e[0] += ve
        o[0] += vo
    while len(e) > 2 and e[-1] < 20:
        ve, vo = e.pop(), o.pop()
        e[-1] += ve
        o[-1] += vo
    o, e = np.array(o), np.array(e)
    return stats.chisquare(o, e * o.sum() / e.sum()).pvalue


def test_immigration_death_ssa_states_are_poisson(orc):
    net = W.birth_death()  # 0 -> X (10), X -> 0 (0.1), X(0) = 0
    P = 20000
    th, x0 = W.tile(net, P)
    times = np.array([0.0, 0.5, 2.0, 5.0, 10.0, 30.0, 100.0])
    g = orc.simulate_grid(net.m, net.p, th, x0, times, mode="ssa")
    assert np.all(g["stats"]["status"] == 0)
    assert np.all(g["x_grid"][:, 0, 0] == 0)
    pv = []
    for k, t in enumerate(times[1:], 1):
        lam = 100.0 * (1.0 - np.exp(-0.1 * t))
        pv.append(_chi2_discrete(g["x_grid"][:, k, 0], stats.poisson(lam)))
    assert min(pv) * len(pv) > 1e-3, pv


def test_isomerisation_ssa_states_are_binomial(orc):
    net = W.isomerisation(n_total=200)
    P = 20000
    th, x0 = W.tile(net, P)
    times = np.array([0.1, 0.3, 0.7, 1.5, 3.0])
    g = orc.simulate_grid(net.m, net.p, th, x0, times, mode="ssa")
    assert np.all(g["x_grid"].sum(axis=2) == 200)
    pv = [_chi2_discrete(g["x_grid"][:, k, 0], stats.binom(200, 0.5 * (1 + np.exp(-2 * t))))
          for k, t in enumerate(times)]
    assert min(pv) * len(pv) > 1e-3, pv


@pytest.mark.parametrize("mode", ["ssa", "explicit"])
def test_trajectory_continues_through_observation_times(orc, mode):
    net = W.birth_death()
    P = 20000
    th, x0 = W.tile(net, P)
    g = orc.simulate_grid(net.m, net.p, th, x0, [5.0, 10.0], mode=mode)
    x1 = g["x_grid"][:, 0, 0].astype(float)
    x2 = g["x_grid"][:, 1, 0].astype(float)
    slope = np.cov(x1, x2)[0, 1] / np.var(x1, ddof=1)
    resid = x2 - x2.mean() - slope * (x1 - x1.mean())
    se = np.sqrt(resid.var() / (P * np.var(x1)))
    assert abs(slope - np.exp(-0.5)) < 4 * se + 0.01, (slope, se)


def test_explicit_leap_means_follow_the_ode(orc):
    # for a linear network the leap's mean follows the rate equation up to the
    # leap's O(tau) bias, small at eps = 0.03
    net = W.birth_death()
    P = 20000
    th, x0 = W.tile(net, P)
    times = np.linspace(10.0, 100.0, 10)
    g = orc.simulate_grid(net.m, net.p, th, x0, times, mode="explicit")
    exact = 100.0 * (1.0 - np.exp(-0.1 * times))
    m = g["x_grid"][:, :, 0].mean(axis=0)
    se = g["x_grid"][:, :, 0].std(axis=0) / np.sqrt(P)
    assert np.all(np.abs(m - exact) < 4 * se + 0.01 * exact), (m, exact)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_time_is_simulate(orc, precision):
    net = W.dimer()
    P = 200
    th = W.gamma_prior_theta(net, P, seed=2)
    _, x0 = W.tile(net, P)
    g = orc.simulate_grid(net.m, net.p, th, x0, [30.0], precision=precision)
    s = orc.simulate(net.m, net.p, th, x0, 30.0, precision=precision)
    for k in ("x", "r", "G", "stats"):
        assert np.array_equal(g[k], s[k]), k
    assert np.array_equal(g["x_grid"][:, 0], s["x"])


def test_structure_and_invalid_times(orc):
    net = W.isomerisation()
    P = 100
    th = W.gamma_prior_theta(net, P, seed=4)
    _, x0 = W.tile(net, P)
    th[3] = -1.0
    g = orc.simulate_grid(net.m, net.p, th, x0, [0.0, 0.0, 1.0, 1.0, 2.5], mode="adaptive")
    ok = np.arange(P) != 3
    assert np.all(g["stats"]["status"][ok] == 0) and g["stats"]["status"][3] == 3
    assert np.all(g["x_grid"][3] == -1)
    xg = g["x_grid"][ok]
    assert np.array_equal(xg[:, 0], x0[ok]) and np.array_equal(xg[:, 1], x0[ok])
    assert np.array_equal(xg[:, 2], xg[:, 3])
    assert np.array_equal(xg[:, 4], g["x"][ok])
    assert np.all(xg.sum(axis=2) == 1000)
    for times, first_bad in (([1.0, 0.5, 2.0], 1), ([1.0, np.inf], 1), ([np.nan, 1.0], 0),
                             ([-0.5, 1.0], 0)):
        g = orc.simulate_grid(net.m, net.p, th, x0, times)
        assert np.all(g["stats"]["status"] == 3)
        assert np.all(g["x_grid"][:, first_bad:] == -1)
        assert np.all(g["x_grid"][ok, :first_bad] >= 0)
    with pytest.raises(ValueError):
        orc.simulate_grid(net.m, net.p, th, x0, [])


def test_observation_times_keep_the_law_of_the_final_state(orc):
    # Requesting observation times ends SSA bursts in progress there, so the
    # step sequence (not the method's target law) depends on the times: the
    # state at t_end with 20 observation times and without any must agree in
    # distribution (independent streams).
    net = W.dimer()
    P = 12000
    th, x0 = W.tile(net, P)
    plain = orc.simulate(net.m, net.p, th, x0, 30.0, mode="adaptive", pid_base=0)
    times = np.linspace(1.5, 30.0, 20)
    g = orc.simulate_grid(net.m, net.p, th, x0, times, mode="adaptive", pid_base=1 << 20)
    assert np.all(g["stats"]["status"] == 0) and np.all(plain["stats"]["status"] == 0)
    assert g["stats"]["steps_ssa"].sum() > 0
    for i in range(net.N):
        a = plain["x"][:, i].astype(float)
        b = g["x"][:, i].astype(float)
        assert stats.ks_2samp(a, b).pvalue > 1e-3, i
        se = np.sqrt(a.var() / P + b.var() / P)
        assert abs(a.mean() - b.mean()) < 4.5 * se, (i, a.mean(), b.mean(), se)
