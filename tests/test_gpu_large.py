"""Networks beyond the register-resident kernels: the random 48 x 128
mass-action network and a 48-species stiff network whose implicit leaps solve
a 48 x 48 Newton system.  Schedules: "plain" (lx_sim_large, one trajectory
per lane), "batched" (lx_sim_wave, one trajectory per wave, 4-wave blocks
sharing the Newton area), "wave64" (one wave per block) and "lane"
(lx_sim_large refilling lanes from the block's range).

The large-network kernels perform the operations of the oracle in the same
order, so results are compared exactly, as for the small networks: whole
simulations element by element (X, r, G and every lane statistic), the step
decision (propensities, critical and equilibrium sets over four mask words,
tau) and the implicit solve on fixed states; at the full size of the random
network's workload (65536 trajectories) on sampled trajectories.
"""

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


_H = {}


def _handle(lxm, net):
    if net.name not in _H:
        _H[net.name] = lxm.Network(net.m, net.p)
    return _H[net.name]


def _gpu(lxm, net, theta, x0, t_end, mode, **opts):
    import torch
    th = torch.as_tensor(np.ascontiguousarray(theta, np.float64), device="cuda")
    xi = torch.as_tensor(np.ascontiguousarray(x0, np.int32), device="cuda")
    res = lxm.simulate(_handle(lxm, net), th, xi, t_end, opts.pop("eps", 0.03), mode, **opts)
    torch.cuda.synchronize()
    return {"x": res["x"].cpu().numpy(), "r": res["r"].cpu().numpy(),
            "G": res["G"].cpu().numpy(), "stats": lxm.stats_numpy(res["stats"])}


def _same(got, ref, what):
    for k in ("x", "r", "G"):
        assert np.array_equal(got[k], ref[k]), (what, k)
    for k in ref["stats"].dtype.names:
        if k == "ops":
            continue
        assert np.array_equal(got["stats"][k], ref["stats"][k]), (what, k)


RANDOM = W.random_network()
STIFF = W.stiff_padded()


# the largest size: 64 species, 256 reactions (four reaction slots per lane
# in the one-trajectory-per-wave kernel)
BIGGEST = W.random_network(seed=9, N=64, M=256, n_pairs=48, n_fast=6)


def _random_inputs(P):
    wl = W.random_network_workload(P=P)
    return wl.theta[0], wl.x0[0]


_REF = {}

SCHED = {"plain": dict(schedule="plain"), "batched": dict(schedule="batched"),
         "wave64": dict(schedule="batched", block_size=64),
         "lane": dict(schedule="batched", lanes_per_traj=1)}


@pytest.mark.parametrize("schedule", ["plain", "batched", "wave64", "lane"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_random_network_elementwise(lxm, orc, precision, schedule):
    # 300 trajectories: several waves and a ragged tail; to t_end 0.2 a
    # trajectory takes ~4000 leaps, then SSA bursts (~20000 steps).
    net = RANDOM
    theta, x0 = _random_inputs(300)
    got = _gpu(lxm, net, theta, x0, 0.2, "adaptive", precision=precision, **SCHED[schedule])
    if precision not in _REF:
        _REF[precision] = orc.simulate(net.m, net.p, theta, x0, 0.2, mode="adaptive",
                                       precision=precision)
    _same(got, _REF[precision], f"random/{precision}/{schedule}")
    assert got["stats"]["steps_explicit"].sum() > 0 and got["stats"]["steps_ssa"].sum() > 0


@pytest.mark.parametrize("schedule", ["plain", "batched", "lane"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_largest_network_elementwise(lxm, orc, precision, schedule):
    # 64 x 256: the block of the one-trajectory-per-wave kernel is the largest
    # whose LDS the device allows
    net = BIGGEST
    theta, x0 = W.tile(net, 96)
    got = _gpu(lxm, net, theta, x0, 0.05, "adaptive", precision=precision, **SCHED[schedule])
    ref = orc.simulate(net.m, net.p, theta, x0, 0.05, mode="adaptive", precision=precision)
    _same(got, ref, f"64x256/{precision}/{schedule}")
    assert np.all(got["stats"]["status"] == 0)
    assert got["stats"]["steps_explicit"].sum() + got["stats"]["steps_ssa"].sum() > 0


@pytest.mark.parametrize("mode", ["adaptive", "explicit", "ssa", "adaptive-fd"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stiff_padded_elementwise(lxm, orc, precision, mode):
    jac = {"jacobian": 1} if mode == "adaptive-fd" else {}
    mode = mode.replace("-fd", "")
    net = STIFF
    P = 200
    theta, x0 = W.tile(net, P)
    theta = theta * np.random.default_rng(7).gamma(4.0, 0.25, size=theta.shape)
    t_end = 0.05 if mode == "ssa" else 0.5
    got = _gpu(lxm, net, theta, x0, t_end, mode, precision=precision, schedule="batched",
               lanes_per_wave=32, ssa_k=3, **jac)
    ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode=mode, precision=precision, **jac)
    _same(got, ref, f"stiff/{precision}/{mode}")
    if mode == "adaptive":
        assert got["stats"]["steps_implicit"].sum() > 0
        assert got["stats"]["newton_iters"].sum() > 0


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_random_network_full_ensemble_sampled(lxm, orc, precision):
    # The random network's full ensemble (65536 trajectories) in the launch
    # configuration bench.py times for it (batched, default knobs), to
    # t_end 0.1 (~2100 leaps per trajectory); 48 sampled trajectories, spread
    # over the grid, are recomputed by the oracle and must agree exactly.
    wl = W.random_network_workload()
    net = wl.nets[0]
    theta, x0 = wl.theta[0], wl.x0[0]
    got = _gpu(lxm, net, theta, x0, 0.1, "adaptive", precision=precision, schedule="batched")
    assert np.all(got["stats"]["status"] == 0)
    idx = np.unique(np.concatenate([np.arange(0, wl.P, wl.P // 40), [1, 255, 256, wl.P - 1]]))
    for p in idx:
        ref = orc.simulate(net.m, net.p, theta[p:p + 1], x0[p:p + 1], 0.1, mode="adaptive",
                           precision=precision, pid_base=int(p), nthreads=1)
        sub = {"x": got["x"][p:p + 1], "r": got["r"][p:p + 1], "G": got["G"][p:p + 1],
               "stats": got["stats"][p:p + 1]}
        _same(sub, ref, f"random full/{precision}/p={p}")


def test_random_network_full_horizon_sampled(lxm, orc):
    # The whole random-network workload as bench.py times it: 65536
    # trajectories to t_end 10 in one launch (batched mixed), implicit leaps
    # with the cooperative 48 x 48 Newton solve included; 32 trajectories
    # spread over the grid recomputed by the oracle must agree exactly, and
    # every trajectory satisfies X = x0 + nu r.
    wl = W.random_network_workload()
    net = wl.nets[0]
    theta, x0 = wl.theta[0], wl.x0[0]
    got = _gpu(lxm, net, theta, x0, wl.t_end, "adaptive", precision="mixed", schedule="batched")
    st = got["stats"]
    assert np.all(st["status"] == 0)
    assert st["steps_implicit"].sum() > 50 * wl.P
    nu = (net.p - net.m).astype(np.int64)
    assert np.array_equal(got["x"], x0 + got["r"].astype(np.int64) @ nu)
    idx = np.unique(np.concatenate([np.arange(0, wl.P, wl.P // 30), [1, wl.P - 1]]))
    for p in idx:
        ref = orc.simulate(net.m, net.p, theta[p:p + 1], x0[p:p + 1], wl.t_end, mode="adaptive",
                           precision="mixed", pid_base=int(p), nthreads=1)
        sub = {"x": got["x"][p:p + 1], "r": got["r"][p:p + 1], "G": got["G"][p:p + 1],
               "stats": got["stats"][p:p + 1]}
        _same(sub, ref, f"random t_end 10/p={p}")


def _states(net, Q, rng):
    scale = np.maximum(net.x0, 50)
    x = rng.integers(0, 3 * scale + 1, size=(Q, net.N))
    x[: Q // 4] = rng.integers(0, 12, size=(Q // 4, net.N))
    th = net.theta * rng.gamma(2.0, 0.5, size=(Q, net.M))
    return x.astype(np.int32), th


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["random", "stiff"])
def test_step_decision_bit_exact(lxm, orc, name, precision):
    net = RANDOM if name == "random" else STIFF
    rng = np.random.default_rng(5)
    x, th = _states(net, 1000, rng)
    if name == "stiff":  # reversible pair near balance: equilibrium sets
        x[::2, 1] = np.maximum(1, (th[::2, 1] * x[::2, 0] * (x[::2, 0] - 1) / 2 / th[::2, 2]).astype(np.int64)).clip(max=2**30)
    got = lxm.test_tau_select(_handle(lxm, net), th, x, 0.03, "adaptive", precision=precision)
    ref = orc.tau_select(net.m, net.p, th, x, mode="adaptive", precision=precision)
    for k in ("a", "crit", "eq", "tau_ex", "tau_im", "action"):
        assert np.array_equal(got[k], ref[k]), k
    if name == "stiff":
        assert ref["eq"].any()


@pytest.mark.parametrize("jacobian", [0, 1, 2])
def test_implicit_solve_48_bit_exact(lxm, orc, jacobian):
    net = STIFF
    assert net.N == 48
    rng = np.random.default_rng(9)
    Q = 500
    x, th = _states(net, Q, rng)
    x = np.maximum(x, 1)
    tau = rng.uniform(1e-4, 0.5, Q)
    res = orc.tau_select(net.m, net.p, th, x)
    Pj = rng.poisson(np.minimum(res["a"] * tau[:, None], 1e6))
    jc = np.where(rng.uniform(size=Q) < 0.3, rng.integers(0, net.M, Q), -1).astype(np.int32)
    if jacobian == 2:   # the caller's terms (the mass-action derivative)
        terms = W.mass_action_jacobian_terms(net)
        h = lxm.Network(net.m, net.p, jacobian_terms=terms)
        got = lxm.test_implicit(h, th, x, tau, Pj, jc, jacobian=2)
        ref = orc.implicit(net.m, net.p, th, x, tau, Pj, jc, jacobian=2, jacobian_terms=terms)
    else:
        got = lxm.test_implicit(_handle(lxm, net), th, x, tau, Pj, jc, jacobian=jacobian)
        ref = orc.implicit(net.m, net.p, th, x, tau, Pj, jc, jacobian=jacobian)
    assert np.array_equal(got["ok"], ref["ok"])
    assert np.array_equal(got["iters"], ref["iters"])
    assert np.array_equal(got["k"], ref["k"])
    assert got["ok"].mean() > 0.5


def test_large_network_limits(lxm):
    m = np.zeros((257, 2), np.int32)
    with pytest.raises(lxm.LxError):
        lxm.Network(m, m)
    m = np.zeros((4, 65), np.int32)
    with pytest.raises(lxm.LxError):
        lxm.Network(m, m)
    import torch
    theta, x0 = _random_inputs(64)
    th = torch.as_tensor(theta, device="cuda")
    xi = torch.as_tensor(x0, device="cuda")
    for bad in (dict(lanes_per_traj=4), dict(regroup=2), dict(tail_lanes=4),
                dict(lanes_per_traj=1, block_size=128)):
        with pytest.raises(lxm.LxError):
            lxm.simulate(_handle(lxm, RANDOM), th, xi, 0.01, schedule="batched", **bad)


@pytest.mark.parametrize("schedule", ["plain", "batched", "lane"])
def test_observation_times_elementwise(lxm, orc, schedule):
    # lx_simulate_grid on both large networks: states at every observation
    # time, X, r, G and statistics identical to the oracle's
    import torch
    cases = ((RANDOM, *_random_inputs(150), np.array([0.02, 0.05, 0.05, 0.1]), "adaptive"),
             (STIFF, *W.tile(STIFF, 100), np.array([0.0, 0.2, 0.4, 0.5]), "adaptive"))
    for net, theta, x0, times, mode in cases:
        print(f"large grid {net.name} {schedule}", flush=True)
        res = lxm.simulate_grid(_handle(lxm, net), torch.as_tensor(theta, device="cuda"),
                                torch.as_tensor(np.ascontiguousarray(x0, np.int32), device="cuda"),
                                torch.as_tensor(times, device="cuda"), 0.03, mode,
                                precision="mixed", **SCHED[schedule])
        torch.cuda.synchronize()
        got = {"x_grid": res["x_grid"].cpu().numpy(), "x": res["x"].cpu().numpy(),
               "r": res["r"].cpu().numpy(), "G": res["G"].cpu().numpy(),
               "stats": lxm.stats_numpy(res["stats"])}
        ref = orc.simulate_grid(net.m, net.p, theta, x0, times, mode=mode, precision="mixed")
        assert np.array_equal(got["x_grid"], ref["x_grid"]), net.name
        _same(got, ref, f"{net.name} grid {schedule}")
        assert np.all(got["stats"]["status"] == 0)


# The rarer method events in the large-network kernels (see the matching
# small-network cases): leap retries after a negative population, failed
# 48 x 48 implicit solves (one Newton iteration), critical firings inside
# leaps over 24 small decaying species.
LARGE_EVENTS = [
    ("retry48", W.pure_death(48), "explicit", 3.7, 300, dict(n_c=0, eps=1.0, k_ssa=0.0),
     "rejections", 5000),
    ("newton_fail48", STIFF, "adaptive", 0.0005, 100, dict(newton_maxit=1), "newton_fail", 100),
    ("critical48", W.critical_decay(24, 24), "adaptive", 4.0, 300, {}, "crit_fired", 10000),
]


@pytest.mark.parametrize("schedule", ["plain", "batched", "lane"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", LARGE_EVENTS, ids=[c[0] for c in LARGE_EVENTS])
def test_large_rare_events_elementwise(lxm, orc, case, precision, schedule):
    name, net, mode, t_end, P, opts, counter, minimum = case
    theta, x0 = W.tile(net, P)
    got = _gpu(lxm, net, theta, x0, t_end, mode, precision=precision, **SCHED[schedule], **opts)
    ref = orc.simulate(net.m, net.p, theta, x0, t_end, mode=mode, precision=precision, **opts)
    _same(got, ref, f"{name}/{precision}/{schedule}")
    assert np.all(got["stats"]["status"] == 0)
    assert int(got["stats"][counter].astype(np.int64).sum()) >= minimum, counter
