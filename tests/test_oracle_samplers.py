"""Pins for the oracle's random-number layer: Philox, uniform maps, exp/log,
log-factorial and the Poisson / exponential samplers.

Each pin checks the oracle against something other than itself: the
mathematical definition of a constant, a multiple-precision or libm value,
an exact probability law (scipy.stats), or an exact quantile function.
"""

import math

import numpy as np
import pytest
from scipy import stats

SEED = 160807058


def ulp_diff64(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ia = a.view(np.int64).astype(np.int64)
    ib = b.view(np.int64).astype(np.int64)
    ia = np.where(ia < 0, np.int64(-(2**63)) - ia, ia)
    ib = np.where(ib < 0, np.int64(-(2**63)) - ib, ib)
    return np.abs(ia - ib)


def ulp_diff32(a, b):
    ia = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(2**31) - ia, ia)
    ib = np.where(ib < 0, -(2**31) - ib, ib)
    return np.abs(ia - ib)


# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al. 2011)
# ---------------------------------------------------------------------------

def _philox_py(ctr, key):
    """Philox4x32-10 written from the SC'11 description (second implementation)."""
    M0, M1 = 0xD2511F53, 0xCD9E8D57
    W0 = int((math.sqrt(5.0) - 1.0) / 2.0 * 2**32)      # golden ratio fraction
    W1 = int((math.sqrt(3.0) - 1.0) * 2**32)            # sqrt(3) - 1
    c = [int(v) for v in ctr]
    k = [int(v) for v in key]
    mask = 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k = [(k[0] + W0) & mask, (k[1] + W1) & mask]
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k[0]) & mask, p1 & mask, ((p0 >> 32) ^ c[3] ^ k[1]) & mask,
             p0 & mask]
    return c


def test_philox_weyl_constants_are_the_published_irrationals():
    # The key schedule adds floor(2^32 (phi - 1)) and floor(2^32 (sqrt 3 - 1)).
    from mpmath import mp, mpf, sqrt, floor
    mp.prec = 100
    assert int(floor((sqrt(5) - 1) / 2 * mpf(2) ** 32)) == 0x9E3779B9
    assert int(floor((sqrt(3) - 1) * mpf(2) ** 32)) == 0xBB67AE85


def test_philox_matches_independent_implementation(orc):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(500, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(500, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    out = orc.philox(ctr, key)
    for q in range(len(ctr)):
        assert list(out[q]) == _philox_py(ctr[q], key[q])


def test_philox_output_is_uniform_and_avalanches(orc):
    n = 1 << 16
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)  # sequential counters, the hardest case
    key = np.tile(np.array([SEED & 0xFFFFFFFF, SEED >> 32], np.uint32), (n, 1))
    out = orc.philox(ctr, key).reshape(-1)
    # byte histogram chi-square
    b = out.view(np.uint8)
    cnt = np.bincount(b, minlength=256)
    assert stats.chisquare(cnt).pvalue > 1e-4
    # each output bit is set half the time
    bits = np.unpackbits(out.view(np.uint8)).reshape(-1, 32)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / math.sqrt(bits.shape[0]))
    # flipping one counter bit flips about half the 128 output bits
    ctr2 = ctr.copy()
    ctr2[:, 1] ^= 1
    d = orc.philox(ctr2, key) ^ orc.philox(ctr, key)
    flips = np.unpackbits(d.view(np.uint8)).reshape(n, -1).sum(axis=1)
    assert abs(flips.mean() - 64.0) < 0.2
    assert stats.binomtest(int(flips.sum()), n * 128, 0.5).pvalue > 1e-4


# ---------------------------------------------------------------------------
# Uniform maps: exact closed forms at the extremes, open interval (0, 1)
# ---------------------------------------------------------------------------

def test_uniform_maps_exact_extremes(orc):
    u = orc.uniform_f64([[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0x80000000, 0]])
    assert u[0] == 2.0**-53
    assert u[1] == 1.0 - 2.0**-53
    assert u[2] == 0.5 + 2.0**-53
    f = orc.uniform_f32(np.array([0, 0xFFFFFFFF, 0x80000000], np.uint32))
    assert f[0] == np.float32(2.0**-24)
    assert f[1] == np.float32(1.0 - 2.0**-24)
    assert f[2] == np.float32(0.5 + 2.0**-24)


def test_uniform_maps_match_integer_definition(orc):
    rng = np.random.default_rng(2)
    w = rng.integers(0, 2**32, size=(10000, 2), dtype=np.uint64)
    u = orc.uniform_f64(w.astype(np.uint32))
    exact = ((w[:, 0] >> 6) * 2**26 + (w[:, 1] >> 6)).astype(np.float64)
    assert np.array_equal(u, (exact + 0.5) / 2.0**52)
    f = orc.uniform_f32(w[:, 0].astype(np.uint32))
    assert np.array_equal(f.astype(np.float64), ((w[:, 0] >> 9).astype(np.float64) + 0.5) / 2**23)


# ---------------------------------------------------------------------------
# exp / log / log-factorial against multiple precision and libm
# ---------------------------------------------------------------------------

def _mp_ref(fn, xs, prec=120):
    from mpmath import mp, mpf
    mp.prec = prec
    return np.array([float(fn(mpf(float(v)))) for v in xs])


def test_exp_f64_within_one_ulp(orc):
    from mpmath import exp
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-40, 0, 3000), rng.uniform(-700, 700, 1000),
                         [0.0, -0.0, 1e-300, -1e-300, 0.5, -0.34657359, 0.34657359, -10.0]])
    got = orc.exp_f64(xs)
    ref = _mp_ref(exp, xs)
    assert ulp_diff64(got, ref).max() <= 1
    assert orc.exp_f64([-800.0, 800.0]).tolist() == [0.0, math.inf]


def test_log_f64_within_one_ulp(orc):
    from mpmath import log
    rng = np.random.default_rng(4)
    xs = np.concatenate([rng.uniform(0, 1, 3000), 10.0 ** rng.uniform(-300, 300, 1000),
                         rng.uniform(0.7, 1.42, 1000), [2.0**-53, 1 - 2.0**-53, 0.5, 1.0, 2.0]])
    got = orc.log_f64(xs)
    ref = _mp_ref(log, xs)
    assert ulp_diff64(got, ref).max() <= 1
    assert orc.log_f64([1.0])[0] == 0.0


def test_exp_log_f32_within_one_ulp(orc):
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.uniform(-30, 0, 20000), rng.uniform(-87, 88, 5000)]).astype(np.float32)
    got = orc.exp_f32(xs)
    ref = np.exp(xs.astype(np.float64)).astype(np.float32)
    assert ulp_diff32(got, ref).max() <= 1
    ys = np.concatenate([rng.uniform(0, 1, 20000), 10.0 ** rng.uniform(-30, 30, 5000)]).astype(np.float32)
    got = orc.log_f32(ys)
    ref = np.log(ys.astype(np.float64)).astype(np.float32)
    assert ulp_diff32(got, ref).max() <= 1


def test_lfact_matches_lgamma(orc):
    k = np.concatenate([np.arange(0, 200), np.unique(np.round(10 ** np.linspace(2, 9, 500)))])
    got = orc.lfact(k.astype(np.float64))
    ref = np.array([math.lgamma(v + 1.0) for v in k])
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() < 4e-15
    assert got[0] == 0.0 and got[1] == 0.0


# ---------------------------------------------------------------------------
# Samplers
# ---------------------------------------------------------------------------

def _site_uniform(orc, pid, e, site, trial=0, seed=SEED, stream=0, precision="fp64"):
    # the first uniform of the draw site: words 0-1 (binary64) or word 0 (binary32)
    n = len(pid)
    ctr = np.stack([pid, np.full(n, e), np.full(n, site), np.full(n, trial)], 1).astype(np.uint32)
    key = np.tile(np.array([seed & 0xFFFFFFFF, ((seed >> 32) + stream) & 0xFFFFFFFF], np.uint32),
                  (n, 1))
    w = orc.philox(ctr, key)
    if precision == "mixed":
        return orc.uniform_f32(w[:, 0]).astype(np.float64)
    return orc.uniform_f64(w[:, :2])


@pytest.mark.parametrize("precision,margin", [("fp64", 1e-12), ("mixed", 2e-5)])
@pytest.mark.parametrize("lam", [1e-6, 0.05, 0.5, 1.0, 3.0, 7.5, 9.99, 12.0, 20.0, 29.9])
def test_poisson_inversion_is_the_exact_quantile(orc, lam, precision, margin):
    # Below the threshold (here its largest allowed value, 30) the sampler
    # must return the smallest k with u <= F(k) for the site's first uniform:
    # scipy's exact Poisson
    # quantile function, except where u lies within the rounding of the
    # summed CDF (a few units of the policy's precision times the number of
    # terms) of one of its steps.
    n = 20000
    pid = np.arange(n, dtype=np.uint32)
    u = _site_uniform(orc, pid, 7, 3, precision=precision)
    k = orc.poisson(np.full(n, lam), pid, 7, 3, precision=precision, lambda_thr=30.0)
    ref = stats.poisson.ppf(u, lam)
    cdf_k = stats.poisson.cdf(ref, lam)
    cdf_km1 = stats.poisson.cdf(ref - 1, lam)
    clear = (np.abs(u - cdf_k) > margin) & (np.abs(u - cdf_km1) > margin)
    assert clear.mean() > 0.99
    assert np.array_equal(k[clear], ref[clear].astype(np.int64))


def test_poisson_inversion_tail_stops_at_the_cdf_resolution(orc):
    # In binary32 the summed CDF ends just below 1; a uniform above that
    # ceiling must not run the search to the cap (20 + 4*30 = 140) but stop
    # where the terms stop adding to the sum, deep in the tail.  The particle
    # ids with the largest first uniforms among 2^24 are exactly such inputs.
    n = 1 << 24
    pid = np.arange(n, dtype=np.uint32)
    u = _site_uniform(orc, pid, 7, 3, precision="mixed")
    top = pid[np.argsort(u)[-64:]]
    assert u.max() > 1.0 - 2.0 ** -22
    for lam in (1.0, 3.0, 9.9, 20.0, 29.9):
        k = orc.poisson(np.full(top.size, lam), top, 7, 3, precision="mixed", lambda_thr=30.0)
        assert k.max() < 140, lam
        assert k.max() <= stats.poisson.ppf(1.0 - 1e-10, lam) + 10, (lam, k.max())


def _chi2_poisson(samples, lam):
    lo = int(max(0, stats.poisson.ppf(1e-7, lam)))
    hi = int(stats.poisson.ppf(1 - 1e-7, lam))
    edges = [lo]
    # bins with expected count >= 20
    n = len(samples)
    k = lo
    while k <= hi:
        acc = 0.0
        start = k
        while k <= hi and acc * n < 20:
            acc += stats.poisson.pmf(k, lam)
            k += 1
        edges.append(k)
        del start
    edges = np.array(edges)
    obs = np.histogram(samples, bins=np.concatenate([[-np.inf], edges[1:-1] - 0.5, [np.inf]]))[0]
    cdf = stats.poisson.cdf(edges[1:-1] - 1, lam)
    probs = np.diff(np.concatenate([[0.0], cdf, [1.0]]))
    return stats.chisquare(obs, probs * n).pvalue


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("lam_thr", [10.0, 15.0, 30.0])
@pytest.mark.parametrize("lam", [0.3, 4.0, 9.99, 10.0, 10.5, 14.99, 15.0, 17.3, 29.9, 30.0, 250.0, 1e4,
                                 1e6])
def test_poisson_law(orc, lam, precision, lam_thr):
    # both samplers over the range where the threshold lets either draw:
    # inversion up to 30, PTRS from 10 (its published range)
    if lam_thr != 15.0 and not 9.0 < lam < 31.0:
        pytest.skip("same sampler as the default threshold")
    n = 200000
    pid = np.arange(n, dtype=np.uint32)
    k = orc.poisson(np.full(n, lam), pid, 11, 5, precision=precision, lambda_thr=lam_thr)
    assert k.min() >= 0
    assert _chi2_poisson(k, lam) > 1e-4
    z_mean = (k.mean() - lam) / math.sqrt(lam / n)
    assert abs(z_mean) < 4.5


def _logpmf_mp(k, lam):
    import mpmath
    with mpmath.workdps(40):
        return float(k * mpmath.log(lam) - lam - mpmath.loggamma(k + 1))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("mixed", 2e-6)])
def test_ptrs_log_density_is_the_poisson_log_pmf(orc, precision, tol):
    # The acceptance test's right side minus the log of its left factor is
    # log p(k; lam) (Hoermann 1993's final test), checked against 40-digit
    # arithmetic: the exact-product branch (k <= 17), the Stirling branch with
    # its series for log(1 + d) - d (|d| <= 1/4) and with the log beyond, at
    # the means the sampler sees (10 to 2^22).  The bound is a few units in the
    # last place of the policy's precision, relative to 1 + |log p|.
    ks, lams = [], []
    for lam in (10.0, 10.5, 17.3, 30.0, 250.0, 1e4, 1e6, 4e6):
        r = math.sqrt(lam)
        kk = np.concatenate([np.arange(0, 60), np.round(lam + r * np.linspace(-8, 8, 41)),
                             np.round(lam * np.array([0.5, 0.79, 0.81, 1.2, 1.26, 2.0]))])
        kk = np.unique(kk[kk >= 0])
        ks.append(kk)
        lams.append(np.full(kk.shape, lam))
    k, lam = np.concatenate(ks), np.concatenate(lams)
    if precision == "mixed":
        lam = lam.astype(np.float32).astype(np.float64)
    fac, rhs = orc.ptrs_log_density(k, lam, precision=precision)
    got = rhs - np.log(fac)
    ref = np.array([_logpmf_mp(int(a), float(b)) for a, b in zip(k, lam)])
    err = np.abs(got - ref) / (1.0 + np.abs(ref))
    assert err.max() < tol, (k[err.argmax()], lam[err.argmax()], err.max())


def test_poisson_large_lambda_fp64(orc):
    lam = 1e8
    n = 50000
    k = orc.poisson(np.full(n, lam), np.arange(n, dtype=np.uint32), 2, 0)
    assert abs((k.mean() - lam) / math.sqrt(lam / n)) < 4.5
    assert abs(k.var() / lam - 1.0) < 0.03
    # beyond the 2^30 range both policies report overflow (-1)
    assert orc.poisson([2e9], [0], 0, 0)[0] == -1
    assert orc.poisson([2e9], [0], 0, 0, precision="mixed")[0] == -1


def test_poisson_large_lambda_mixed(orc):
    # From 2^22 the binary32 policy hands the mean to the binary64 sampler at
    # the same draw site: identical counts there, the Poisson law (mean and
    # variance within sampling error) up to the 2^30 range, and binary32 PTRS
    # just below the seam.
    n = 50000
    pid = np.arange(n, dtype=np.uint32)
    for lam in (2.0**22, 1e7, 1e9):
        km = orc.poisson(np.full(n, lam), pid, 2, 0, precision="mixed")
        kd = orc.poisson(np.full(n, lam), pid, 2, 0, precision="fp64")
        assert np.array_equal(km, kd)
        assert abs((km.mean() - lam) / math.sqrt(lam / n)) < 4.5
        assert abs(km.var() / lam - 1.0) < 0.03
    below = np.float32(2.0**22 - 0.5)
    km = orc.poisson(np.full(n, below, np.float64), pid, 2, 0, precision="mixed")
    kd = orc.poisson(np.full(n, below, np.float64), pid, 2, 0, precision="fp64")
    assert not np.array_equal(km, kd)
    assert abs((km.mean() - below) / math.sqrt(below / n)) < 4.5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exponential_law(orc, precision):
    n = 200000
    pid = np.arange(n, dtype=np.uint32)
    e = orc.exponential(pid, 3, precision=precision)
    assert stats.kstest(e, "expon").pvalue > 1e-3
    # it is -log of the site's first uniform
    if precision == "fp64":
        u = _site_uniform(orc, pid[:1000], 3, orc.SITE_SSA)
        assert np.all(ulp_diff64(e[:1000], -np.log(u)) <= 2)


def test_sites_are_independent_streams(orc):
    # the same (pid, e) at two sites, or two attempts, must not be correlated
    n = 100000
    pid = np.arange(n, dtype=np.uint32)
    u1 = _site_uniform(orc, pid, 0, 0)
    u2 = _site_uniform(orc, pid, 0, 1)
    u3 = _site_uniform(orc, pid, 1, 0)
    assert abs(np.corrcoef(u1, u2)[0, 1]) < 0.02
    assert abs(np.corrcoef(u1, u3)[0, 1]) < 0.02
    u4 = _site_uniform(orc, pid, 0, 0, stream=1)
    assert abs(np.corrcoef(u1, u4)[0, 1]) < 0.02
