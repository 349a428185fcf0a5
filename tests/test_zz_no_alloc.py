"""lx_pf_run_static (the filter entry point that allocates nothing) against
lx_pf_run with a caller workspace: identical theta, states, cumulative r and
G and log-likelihood increments, on two calls in a row, the second with a
smaller ensemble; filters beyond the static scratch and kernels not yet
loaded are refused."""

import numpy as np
import pytest

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


def _observations(K, seed=3):
    rng = np.random.default_rng(seed)
    return np.clip(100.0 + np.cumsum(rng.normal(0.0, 15.0, K)), 0.0, None)


def _pf(lxm, h, net, theta, x0, y, workspace, **opts):
    import torch
    alpha = torch.full((net.M,), 2.0, dtype=torch.float64, device="cuda")
    beta = torch.as_tensor(2.0 / net.theta, device="cuda")
    return lxm.ParticleFilter(h, torch.as_tensor(theta.copy(), device="cuda"),
                              torch.as_tensor(x0.copy(), device="cuda"),
                              torch.as_tensor(y, device="cuda"), alpha, beta, 5.0, 3, 10.0,
                              workspace=workspace, **opts)


def _get(pf):
    import torch
    torch.cuda.synchronize()
    return {k: getattr(pf, k).cpu().numpy() for k in ("theta", "x", "r", "G", "loglik")}


def test_static_scratch_filter_matches_workspace_filter(lxm):
    net = W.telegraph()
    h = lxm.Network(net.m, net.p)
    opts = dict(schedule="batched", precision="mixed")
    y = _observations(8)
    for P, seed in ((6000 + 37, 5), (1500 + 3, 6)):   # the second call is smaller
        theta = W.gamma_prior_theta(net, P, seed=seed)
        _, x0 = W.tile(net, P)
        ref_pf = _pf(lxm, h, net, theta, x0, y, True, **opts)
        ref_pf.run()                      # loads the kernel (allocating path)
        ref = _get(ref_pf)
        got_pf = _pf(lxm, h, net, theta, x0, y, False, **opts)
        got_pf.run_static()
        got = _get(got_pf)
        for k in ("theta", "x", "r", "G", "loglik"):
            assert np.array_equal(got[k], ref[k]), (P, k)
        assert np.all(np.isfinite(got["loglik"]))


def test_static_scratch_limits(lxm):
    net = W.telegraph()
    y = _observations(2)
    # a kernel variant never loaded through the allocating path is refused
    h = lxm.Network(net.m, net.p)
    theta = W.gamma_prior_theta(net, 300, seed=7)
    _, x0 = W.tile(net, 300)
    pf = _pf(lxm, h, net, theta, x0, y, False, schedule="batched", precision="fp64", ssa_k=5)
    with pytest.raises(lxm.LxError, match="not loaded"):
        pf.run_static()
    # beyond 64 MiB of scratch (checked before any launch)
    P = 1 << 20
    big = _pf(lxm, h, net, np.ones((P, net.M)), np.zeros((P, net.N), np.int32), y, False,
              schedule="batched", precision="mixed")
    with pytest.raises(lxm.LxError, match="static maximum"):
        big.run_static()
