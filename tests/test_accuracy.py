"""Pins for the KL-divergence accuracy measure (paper_1608_07058_amd.accuracy).

The estimator is checked against exact divergences between known laws
(Poisson pairs in closed form, binomial pairs summed exactly over their
support), against its own definition on hand-built histograms, and for the
properties a divergence has (zero for equal samples, positive otherwise,
invariant under a common shift of integer samples)."""

import numpy as np
import pytest
from scipy import stats

from paper_1608_07058_amd import accuracy as A


def test_equal_samples_give_zero():
    x = np.random.default_rng(0).poisson(30, 5000)
    assert A.kl_divergence(x, x) == 0.0
    assert A.kl_divergence(np.full(10, 7), np.full(20, 7)) == 0.0


def test_poisson_pair_matches_closed_form():
    # KL(Poisson(a) || Poisson(b)) = a log(a/b) + b - a
    rng = np.random.default_rng(1)
    a, b = 12.0, 13.5
    n = 2_000_000
    est = A.kl_divergence(rng.poisson(a, n), rng.poisson(b, n))
    exact = a * np.log(a / b) + b - a
    assert abs(est - exact) < 0.05 * exact, (est, exact)


def test_binomial_pair_matches_exact_sum():
    rng = np.random.default_rng(2)
    n = 2_000_000
    d1, d2 = stats.binom(25, 0.4), stats.binom(25, 0.46)
    k = np.arange(26)
    exact = float(np.sum(d1.pmf(k) * np.log(d1.pmf(k) / d2.pmf(k))))
    est = A.kl_divergence(d1.rvs(n, random_state=rng), d2.rvs(n, random_state=rng))
    assert abs(est - exact) < 0.05 * exact, (est, exact)


def test_definition_on_small_histograms():
    # samples {0,0,1} and {1,2}: pooled range 0..2, one bin per value, half a
    # count added per bin
    est = A.kl_divergence([0, 0, 1], [1, 2])
    p = (np.array([2, 1, 0]) + 0.5) / (3 + 1.5)
    q = (np.array([0, 1, 1]) + 0.5) / (2 + 1.5)
    assert est == pytest.approx(float(np.sum(p * np.log(p / q))), rel=1e-15)


def test_wide_ranges_use_at_most_max_bins():
    # values 0..99 in bins of width 4 (25 bins): samples differing only inside
    # a bin have divergence 0
    a = np.arange(0, 100, 4)
    b = a + 3
    assert A.kl_divergence(a, b) == 0.0
    assert A.kl_divergence(a, b + 1) > 0.0


def test_shift_invariance_and_positivity():
    rng = np.random.default_rng(3)
    a, b = rng.poisson(40, 4000), rng.poisson(45, 4000)
    k = A.kl_divergence(a, b)
    assert k > 0.0
    assert A.kl_divergence(a + 1000, b + 1000) == pytest.approx(k, rel=1e-12)


def test_variance_ratio():
    rng = np.random.default_rng(5)
    a = rng.poisson(20, (20000, 3, 1))
    b = 2 * rng.poisson(20, (20000, 3, 1))   # Var(2X) = 4 Var(X)
    assert abs(A.variance_ratio(a, b)[0] - 4.0) < 0.2
    assert A.variance_ratio(a, a)[0] == 1.0


def test_mean_kl_averages_times_and_species():
    rng = np.random.default_rng(4)
    ref = rng.poisson(20, (3000, 4, 2)).astype(np.int32)
    test = rng.poisson(22, (3000, 4, 2)).astype(np.int32)
    want = np.mean([A.kl_divergence(ref[:, k, i], test[:, k, i]) for k in range(4)
                    for i in range(2)])
    assert A.mean_kl(ref, test) == pytest.approx(want, rel=1e-14)
    with pytest.raises(ValueError):
        A.mean_kl(ref, test[:, :3])
    bad = test.copy()
    bad[0, 1, 0] = -1
    with pytest.raises(ValueError):
        A.mean_kl(ref, bad)


def test_oracle_ssa_floor_is_small_and_leaping_is_close(orc):
    # the measure on the oracle: two independent exact-SSA ensembles of
    # immigration-death differ by sampling noise only; explicit leaping at
    # eps = 0.03 stays within a few times that floor
    from paper_1608_07058_amd import workloads as W
    net = W.birth_death()
    P = 10000
    th, x0 = W.tile(net, P)
    times = np.linspace(5.0, 100.0, 20)
    ref = orc.simulate_grid(net.m, net.p, th, x0, times, mode="ssa", seed=1)["x_grid"]
    ssa2 = orc.simulate_grid(net.m, net.p, th, x0, times, mode="ssa", seed=2)["x_grid"]
    leap = orc.simulate_grid(net.m, net.p, th, x0, times, mode="explicit", seed=3)["x_grid"]
    floor = A.mean_kl(ref, ssa2)
    assert floor < 0.006
    assert A.mean_kl(ref, leap) < 3 * floor + 0.002
