"""The accuracy measure end to end on the GPU (paper_1608_07058_amd.accuracy):
SSA reference, independent SSA floor and leaping methods on a small
immigration-death ensemble."""

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


def test_accuracy_run_network(lxm, orc):
    from paper_1608_07058_amd import accuracy as A
    net = W.birth_death()
    rows = A.run_network(lxm, net, 50.0, P=4000, replicates=2, n_times=5)
    assert set(rows) == {"SSA (independent)", *A.METHODS}
    for label, r in rows.items():
        assert np.isfinite(r["kl_mean"]) and r["kl_mean"] >= 0.0, label
        assert len(r["kl_per_species"]) == net.N and r["s_per_trajectory"] > 0.0
    # two exact-SSA ensembles differ by sampling noise only (~31 bins / 4000)
    assert rows["SSA (independent)"]["kl_mean"] < 0.03
    assert abs(rows["SSA (independent)"]["variance_ratio_per_species"][0] - 1.0) < 0.1
    # explicit leaping on a linear network stays near that floor
    assert rows["explicit, mixed"]["kl_mean"] < 3 * rows["SSA (independent)"]["kl_mean"] + 0.01
    # the reference is the library's SSA mode, trajectory by trajectory the oracle's
    import torch
    h = lxm.Network(net.m, net.p)
    theta, x0 = W.tile(net, 300)
    times = np.linspace(10.0, 50.0, 5)
    got = lxm.simulate_grid(h, torch.as_tensor(theta, device="cuda"),
                            torch.as_tensor(x0, device="cuda"), torch.as_tensor(times, device="cuda"),
                            0.03, "ssa", precision="fp64", schedule="batched", seed=A.SEED_REF)
    torch.cuda.synchronize()
    ref = orc.simulate_grid(net.m, net.p, theta, x0, times, mode="ssa", seed=A.SEED_REF)
    assert np.array_equal(got["x_grid"].cpu().numpy(), ref["x_grid"])
