"""Observation-time output (lx_simulate_grid) on the GPU against the oracle.

Element by element: the states at every observation time (x_grid), X, r, G
and every lane statistic are identical to the oracle's for the same seeded
inputs, for every small network and mode, both precision policies and every
schedule (plain, batched, regrouped, lane groups), at sizes spanning several
blocks with a ragged tail; edge cases (a time at t_start, repeated times, a
time going backwards, a non-finite time, invalid lanes, empty ensembles,
argument errors); one observation time at t_end reproduces lx_simulate.
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


_HANDLES = {}


def _handle(lxm, net):
    key = (net.name, net.m.tobytes(), net.p.tobytes())
    if key not in _HANDLES:
        _HANDLES[key] = lxm.Network(net.m, net.p)
    return _HANDLES[key]


def gpu_grid(lxm, net, theta, x0, times, mode, **opts):
    import torch
    th = torch.as_tensor(np.ascontiguousarray(theta, np.float64), device="cuda")
    xi = torch.as_tensor(np.ascontiguousarray(x0, np.int32), device="cuda")
    tt = torch.as_tensor(np.ascontiguousarray(times, np.float64), device="cuda")
    res = lxm.simulate_grid(_handle(lxm, net), th, xi, tt, opts.pop("eps", 0.03), mode, **opts)
    torch.cuda.synchronize()
    return {"x_grid": res["x_grid"].cpu().numpy(), "x": res["x"].cpu().numpy(),
            "r": res["r"].cpu().numpy(), "G": res["G"].cpu().numpy(),
            "stats": lxm.stats_numpy(res["stats"])}


def assert_same(got, ref, what=""):
    for key in ("x_grid", "x", "r", "G"):
        if not np.array_equal(got[key], ref[key]):
            bad = np.argwhere(np.any(got[key].reshape(len(got[key]), -1) !=
                                     ref[key].reshape(len(ref[key]), -1), axis=1))[:5, 0]
            raise AssertionError(f"{what}: {key} differs at particles {bad.tolist()}")
    for f in ("status", "crit_fired", "t_final", "steps_ssa", "steps_explicit", "steps_implicit", "rejections",
              "newton_iters", "newton_fail", "kclip", "attempts"):
        assert np.array_equal(got["stats"][f], ref["stats"][f]), (what, f)


CASES = [
    # name, network, mode, times, P
    ("birth_death", W.birth_death(), "explicit", np.linspace(0.0, 100.0, 21), 3000),
    ("dimer", W.dimer(), "adaptive", np.linspace(1.5, 30.0, 20), 1500),
    ("dimer_stiff", W.dimer_stiff(), "adaptive", np.array([0.1, 0.5, 0.5, 1.0, 2.0, 3.0]), 257),
    ("isomerisation", W.isomerisation(), "adaptive", np.linspace(0.25, 5.0, 20), 1000),
    ("schlogl", W.schlogl(), "adaptive", np.linspace(0.5, 10.0, 20), 700),
    ("telegraph", W.telegraph(), "adaptive", np.linspace(0.0, 50.0, 11), 999),
    ("dimer_ssa", W.dimer(), "ssa", np.linspace(0.05, 0.5, 10), 130),
    ("dimer_explicit", W.dimer(), "explicit", np.linspace(1.0, 10.0, 10), 321),
]

SCHEDULES = {"plain": dict(schedule="plain"), "batched": dict(schedule="batched"),
             "regroup": dict(schedule="batched", regroup=1),
             "tail8": dict(schedule="batched", tail_lanes=8, lanes_per_wave=64),
             "group4": dict(schedule="batched", lanes_per_traj=4)}


@pytest.mark.parametrize("schedule", list(SCHEDULES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_grid_matches_oracle_elementwise(lxm, orc, case, precision, schedule):
    name, net, mode, times, P = case
    theta = W.gamma_prior_theta(net, P, seed=17)
    _, x0 = W.tile(net, P)
    print(f"grid {name} {precision} {schedule} P={P} K={len(times)}", flush=True)
    got = gpu_grid(lxm, net, theta, x0, times, mode, precision=precision, **SCHEDULES[schedule])
    ref = orc.simulate_grid(net.m, net.p, theta, x0, times, mode=mode, precision=precision)
    assert_same(got, ref, f"{name}/{precision}/{schedule}")
    assert np.all(got["stats"]["status"] == 0)
    assert np.array_equal(got["x_grid"][:, -1], got["x"])


@pytest.mark.parametrize("knobs", [
    dict(lanes_per_wave=4, ssa_k=2, blocks_per_cu=1),
    dict(lanes_per_wave=16, ssa_k=8, blocks_per_cu=1, regroup=2),
    dict(lanes_per_wave=64, lanes_per_traj=4, ssa_k=8, blocks_per_cu=1),
    dict(lanes_per_wave=16, lanes_per_traj=8, ssa_k=8, blocks_per_cu=2),
    dict(lanes_per_wave=64, lanes_per_traj=16, ssa_k=20, blocks_per_cu=4),
])
def test_grid_refill_and_knobs(lxm, orc, knobs):
    # few resident blocks: lanes refill many times, each trajectory crossing
    # every observation time
    net = W.telegraph()
    P = 20000
    theta = W.gamma_prior_theta(net, P, seed=19)
    _, x0 = W.tile(net, P)
    times = np.linspace(1.0, 20.0, 12)
    print(f"grid knobs {knobs}", flush=True)
    got = gpu_grid(lxm, net, theta, x0, times, "adaptive", precision="mixed", schedule="batched",
                   **knobs)
    ref = orc.simulate_grid(net.m, net.p, theta, x0, times, mode="adaptive", precision="mixed")
    assert_same(got, ref, str(knobs))


def test_one_time_is_simulate(lxm):
    import torch
    net = W.dimer()
    P = 2048 + 5
    theta = W.gamma_prior_theta(net, P, seed=3)
    _, x0 = W.tile(net, P)
    for opts in (dict(schedule="plain", precision="fp64"),
                 dict(schedule="batched", precision="mixed", lanes_per_traj=4)):
        got = gpu_grid(lxm, net, theta, x0, [30.0], "adaptive", **opts)
        h = _handle(lxm, net)
        ref = lxm.simulate(h, torch.as_tensor(theta, device="cuda"),
                           torch.as_tensor(x0, device="cuda"), 30.0, 0.03, "adaptive", **opts)
        torch.cuda.synchronize()
        assert np.array_equal(got["x_grid"][:, 0], ref["x"].cpu().numpy())
        assert np.array_equal(got["x"], ref["x"].cpu().numpy())
        assert np.array_equal(got["r"], ref["r"].cpu().numpy())
        assert np.array_equal(got["G"], ref["G"].cpu().numpy())
        assert np.array_equal(got["stats"], lxm.stats_numpy(ref["stats"]))


def test_grid_edge_cases(lxm, orc):
    net = W.dimer()
    P = 300
    theta = W.gamma_prior_theta(net, P, seed=23)
    _, x0 = W.tile(net, P)
    theta[5] = -1.0         # invalid lane: every row -1
    theta[6, 2] = np.inf
    x0[7, 0] = -3
    for times, what in (
        (np.array([0.0, 0.0, 2.0, 2.0, 5.0]), "times at t_start and repeated"),
        (np.array([1.0, 3.0, 2.0, 4.0]), "a time going backwards"),
        (np.array([1.0, np.inf]), "an infinite time"),
        (np.array([1.0, np.nan, 2.0]), "a NaN time"),
        (np.array([-1.0, 2.0]), "a first time before t_start"),
        (np.array([0.0]), "only t_start"),
    ):
        for sched in (dict(schedule="plain"), dict(schedule="batched", lanes_per_traj=4),
                      dict(schedule="batched", regroup=1)):
            got = gpu_grid(lxm, net, theta, x0, times, "adaptive", precision="mixed", **sched)
            ref = orc.simulate_grid(net.m, net.p, theta, x0, times, mode="adaptive",
                                    precision="mixed")
            assert_same(got, ref, f"{what} {sched}")
        assert np.all(got["x_grid"][5:8] == -1)
        st = got["stats"]["status"]
        assert np.all(st[5:8] == 3)
        ok = np.ones(P, bool)
        ok[5:8] = False
        if what == "times at t_start and repeated":
            assert np.all(st[ok] == 0)
            assert np.array_equal(got["x_grid"][ok, 0], x0[ok])
            assert np.array_equal(got["x_grid"][:, 0], got["x_grid"][:, 1])
            assert np.array_equal(got["x_grid"][:, 2], got["x_grid"][:, 3])
        elif what == "a time going backwards":
            assert np.all(st[ok] == 3)
            assert np.all(got["x_grid"][ok, 2:] == -1) and np.all(got["x_grid"][ok, :2] >= 0)
            assert np.all(got["stats"]["t_final"][ok] == 3.0)
        elif what == "a first time before t_start":
            assert np.all(got["x_grid"] == -1) and np.all(st == 3)


def test_grid_empty_and_errors(lxm):
    import torch
    net = W.birth_death()
    h = _handle(lxm, net)
    z = lxm.simulate_grid(h, torch.zeros((0, net.M), dtype=torch.float64, device="cuda"),
                          torch.zeros((0, net.N), dtype=torch.int32, device="cuda"),
                          torch.ones(3, dtype=torch.float64, device="cuda"))
    assert z["x_grid"].shape == (0, 3, net.N)
    th = torch.ones((4, net.M), dtype=torch.float64, device="cuda")
    xi = torch.zeros((4, net.N), dtype=torch.int32, device="cuda")
    with pytest.raises(lxm.LxError):
        lxm.simulate_grid(h, th, xi, torch.zeros(0, dtype=torch.float64, device="cuda"))
    with pytest.raises(lxm.LxError):
        lxm.simulate_grid(h, th, xi, torch.ones(2, dtype=torch.float64, device="cuda"), eps=-1.0)
    with pytest.raises(ValueError):
        lxm.simulate_grid(h, th, xi, torch.ones((2, 2), dtype=torch.float64, device="cuda"))


def test_grid_full_size_dimer_sampled(lxm, orc):
    # the benchmark ensemble (16384 trajectories, t_end 30) with 31 observation
    # times in the tuned headline launch; sampled trajectories recomputed by
    # the oracle one by one
    wl = W.dimer_workload()
    net = wl.nets[0]
    times = np.linspace(0.0, wl.t_end, 31)
    got = gpu_grid(lxm, net, wl.theta[0], wl.x0[0], times, wl.mode, precision="mixed",
                   schedule="batched", lanes_per_traj=4, lanes_per_wave=64, ssa_k=8,
                   block_size=256, blocks_per_cu=2)
    assert np.all(got["stats"]["status"] == 0)
    idx = np.random.default_rng(5).choice(wl.P, 48, replace=False)
    idx[0], idx[1] = 0, wl.P - 1
    for p in idx:  # particle id = ensemble index
        one = orc.simulate_grid(net.m, net.p, wl.theta[0][p:p + 1], wl.x0[0][p:p + 1], times,
                                mode=wl.mode, precision="mixed", pid_base=int(p), nthreads=1)
        for k in ("x_grid", "x", "r", "G"):
            assert np.array_equal(got[k][p], one[k][0]), (int(p), k)
        assert got["stats"]["attempts"][p] == one["stats"]["attempts"][0]


def test_grid_split_run_with_accumulation(lxm, orc):
    # the second half of a run: t_start 10, r and G carried in (accumulate),
    # observation times from t_start on; another random stream
    import torch
    net = W.telegraph()
    P = 1500
    theta = W.gamma_prior_theta(net, P, seed=31)
    _, x0 = W.tile(net, P)
    first = orc.simulate(net.m, net.p, theta, x0, 10.0, mode="adaptive", precision="mixed")
    times = np.array([10.0, 12.5, 15.0, 20.0])
    ref = orc.simulate_grid(net.m, net.p, theta, first["x"], times, mode="adaptive",
                            precision="mixed", t_start=10.0, rng_stream=1, r0=first["r"],
                            G0=first["G"])
    for sched in (dict(schedule="plain"), dict(schedule="batched", lanes_per_traj=4)):
        out = {"r": torch.as_tensor(first["r"], device="cuda"),
               "G": torch.as_tensor(first["G"], device="cuda")}
        res = lxm.simulate_grid(_handle(lxm, net), torch.as_tensor(theta, device="cuda"),
                                torch.as_tensor(first["x"], device="cuda"),
                                torch.as_tensor(times, device="cuda"), out=out, precision="mixed",
                                t_start=10.0, rng_stream=1, accumulate=1, **sched)
        torch.cuda.synchronize()
        got = {"x_grid": res["x_grid"].cpu().numpy(), "x": res["x"].cpu().numpy(),
               "r": res["r"].cpu().numpy(), "G": res["G"].cpu().numpy(),
               "stats": lxm.stats_numpy(res["stats"])}
        assert_same(got, ref, f"split {sched}")
        assert np.array_equal(got["x_grid"][:, 0], first["x"])
