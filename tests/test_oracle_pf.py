"""Pins for the oracle's particle-filter pieces: the Gamma sampler against
the Gamma law, multinomial resampling against its integer definition and the
multinomial law, and the filter against data generated from the model."""

import math

import numpy as np
import pytest
from scipy import stats

from paper_1608_07058_amd import workloads as W

SEED = 160807058


@pytest.mark.parametrize("shape", [0.05, 0.3, 0.7, 0.999, 1.0, 1.5, 2.5, 20.0, 500.0, 1e5])
def test_gamma_law(orc, shape):
    n = 100000
    g = orc.gamma(np.full(n, shape), np.arange(n), 3, 2)
    assert stats.kstest(g, stats.gamma(shape).cdf).pvalue > 1e-3
    assert abs(g.mean() - shape) < 5 * math.sqrt(shape / n)


def test_gamma_invalid_shape_is_nan(orc):
    g = orc.gamma(np.array([0.0, -1.0, np.inf, np.nan]), np.arange(4), 3, 2)
    assert np.all(np.isnan(g))


def test_gamma_sites_differ(orc):
    a = orc.gamma(np.full(1000, 3.0), np.arange(1000), 1, 0)
    b = orc.gamma(np.full(1000, 3.0), np.arange(1000), 1, 1)
    c = orc.gamma(np.full(1000, 3.0), np.arange(1000), 2, 0)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.1 and abs(np.corrcoef(a, c)[0, 1]) < 0.1


def test_resampling_is_the_integer_quantile(orc):
    rng = np.random.default_rng(3)
    P = 5000
    codes = rng.integers(0, 2**40, size=P, dtype=np.uint64)
    codes[::7] = 0
    k = 4
    anc = orc.resample(codes, k)
    S = np.cumsum(codes.astype(object))
    total = int(S[-1])
    ctr = np.stack([np.arange(P), np.full(P, k), np.full(P, orc.SITE_RESAMPLE), np.zeros(P)],
                   1).astype(np.uint32)
    key = np.tile(np.array([SEED & 0xFFFFFFFF, SEED >> 32], np.uint32), (P, 1))
    w = orc.philox(ctr, key)
    for q in range(P):
        r64 = (int(w[q, 0]) << 32) | int(w[q, 1])
        U = (r64 * total) >> 64
        a = int(anc[q])
        assert (a == 0 or int(S[a - 1]) <= U) and U < int(S[a])
        assert codes[a] > 0


def test_resampling_law(orc):
    rng = np.random.default_rng(4)
    m = 50
    codes_small = rng.integers(1, 1000, size=m).astype(np.uint64) * (2**30)
    P = 200000
    codes = np.zeros(P, np.uint64)
    codes[:m] = codes_small
    anc = orc.resample(codes, 1)
    cnt = np.bincount(anc, minlength=P)[:m]
    assert cnt.sum() == P
    p = codes_small.astype(float) / codes_small.astype(float).sum()
    assert stats.chisquare(cnt, p * P).pvalue > 1e-3


def _telegraph_data(orc, K=20, seed=77):
    net = W.telegraph()
    x = net.x0[None].copy()
    r = np.zeros((1, net.M), np.int32)
    G = np.zeros((1, net.M))
    ys = []
    for k in range(1, K + 1):
        o = orc.simulate(net.m, net.p, net.theta[None], x, 5.0 * k, t_start=5.0 * (k - 1),
                         rng_stream=k, seed=seed, r0=r, G0=G)
        x, r, G = o["x"], o["r"], o["G"]
        ys.append(x[0, 3])
    return np.array(ys, float) + np.random.default_rng(seed).normal(0.0, 10.0, K)


def test_filter_recovers_parameters_and_prefers_the_truth(orc):
    net = W.telegraph()
    y = _telegraph_data(orc)
    P = 3000
    _, x0 = W.tile(net, P)
    alpha = np.full(net.M, 2.0)
    good = orc.pf_run(net.m, net.p, W.gamma_prior_theta(net, P, seed=5), x0, len(y), 5.0, 3,
                      10.0, y, alpha, alpha / net.theta)
    # the protein channels are identified by the observations
    post = good["theta"].mean(0)
    assert 0.5 * net.theta[4] < post[4] < 2.0 * net.theta[4]
    assert 0.5 * net.theta[5] < post[5] < 2.0 * net.theta[5]
    assert np.all(np.isfinite(good["loglik"]))
    wrong_nom = net.theta * np.array([1, 1, 1, 1, 5.0, 0.2])
    wrong = W.Network("w", net.m, net.p, wrong_nom, net.x0)
    bad = orc.pf_run(net.m, net.p, W.gamma_prior_theta(wrong, P, seed=5), x0, len(y), 5.0, 3,
                     10.0, y, np.full(net.M, 200.0), 200.0 / wrong_nom)
    assert good["loglik"].sum() > bad["loglik"].sum() + 10.0
    # statistics stay consistent with the gathered states
    nu = (net.p - net.m).astype(np.int64)
    assert np.array_equal(good["x"], x0 + good["r"].astype(np.int64) @ nu)
    assert np.allclose(good["G"][:, 0] + good["G"][:, 1], 5.0 * len(y), rtol=1e-12)


def test_filter_weights_are_relative_and_failed_lanes_weigh_zero(orc):
    net = W.telegraph()
    P = 500
    th = W.gamma_prior_theta(net, P, seed=2)
    _, x0 = W.tile(net, P)
    alpha = np.full(net.M, 2.0)
    # far-off observations: weights are relative to the best particle
    res = orc.pf_run(net.m, net.p, th, x0, 2, 5.0, 3, 1e-3, np.array([1e9, 1e9]), alpha,
                     alpha / net.theta)
    assert np.all(np.isfinite(res["loglik"])) and np.all(res["loglik"] < -1e20)
    # every lane invalid in the first interval (negative theta): uniform
    # resampling, log-likelihood -inf; the refreshed theta is valid afterwards
    res = orc.pf_run(net.m, net.p, -th, x0, 2, 5.0, 3, 10.0, np.array([10.0, 10.0]), alpha,
                     alpha / net.theta)
    assert res["loglik"][0] == -np.inf and np.isfinite(res["loglik"][1])
    assert np.all(res["theta"] > 0)
