"""The C ABI without a GPU: the library loads, exports every function that
include/lx.h declares, validates networks and arguments, compiles kernels
with hipRTC, and is independent of the oracle."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1608_07058_amd import lx, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lx_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 16
    L = lx.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(lx.EXPORTS) == set(names)


def test_library_does_not_use_the_oracle():
    so = lx.LIB_PATH
    syms = subprocess.run(["nm", "-D", so], capture_output=True, text=True).stdout
    assert "orc_" not in syms
    deps = subprocess.run(["ldd", so], capture_output=True, text=True).stdout
    assert "oracle" not in deps


def test_struct_layouts_and_defaults():
    assert C.sizeof(lx.Options) == 160
    assert lx.STATS_DTYPE.itemsize == 80
    o = lx.options()
    assert (o.precision, o.schedule, o.n_c, o.n_ssa_ex, o.n_ssa_im, o.newton_maxit) == (0, 0, 10, 100, 10, 20)
    assert (o.delta, o.n_stiff, o.k_ssa, o.k_crit, o.lambda_thr, o.newton_tol) == (0.05, 100.0, 10.0, 10.0, 15.0, 1e-10)
    assert o.seed == 160807058 and o.max_steps == 10_000_000


def _create(m, p):
    m = np.ascontiguousarray(m, np.int32)
    p = np.ascontiguousarray(p, np.int32)
    h = C.c_void_p()
    rc = lx.lib().lx_network_create(m.shape[1], m.shape[0], m.ctypes.data, p.ctypes.data, C.byref(h))
    return rc, h


def test_network_validation():
    L = lx.lib()
    assert _create([[4]], [[0]])[0] == -1            # order above 3
    assert b"order" in L.lx_last_error()
    assert _create([[2, 2]], [[0, 0]])[0] == -1      # order 4 across species
    assert _create([[-1]], [[0]])[0] == -1           # negative entry
    assert _create([[1]], [[-2]])[0] == -1
    assert _create(np.zeros((257, 1)), np.ones((257, 1)))[0] == -1   # M above 256
    assert _create(np.zeros((1, 65)), np.ones((1, 65)))[0] == -1     # N above 64
    for shape in ((33, 1), (4, 17), (128, 48)):  # large-network kernels
        rc, h = _create(np.zeros(shape), np.ones(shape))
        assert rc == 0
        assert L.lx_network_destroy(h) == 0
    rc, h = _create(W.dimer().m, W.dimer().p)
    assert rc == 0
    n, m, q = C.c_int32(), C.c_int32(), C.c_int32()
    assert L.lx_network_info(h, C.byref(n), C.byref(m), C.byref(q)) == 0
    assert (n.value, m.value, q.value) == (3, 4, 1)
    assert L.lx_network_destroy(h) == 0
    assert L.lx_network_destroy(None) == 0
    h = C.c_void_p()
    assert L.lx_network_create(0, 1, None, None, C.byref(h)) == -1


def test_pairs_found():
    assert lx.Network(W.isomerisation().m, W.isomerisation().p).info()["n_pairs"] == 1
    assert lx.Network(W.birth_death().m, W.birth_death().p).info()["n_pairs"] == 1
    assert lx.Network(W.schlogl().m, W.schlogl().p).info()["n_pairs"] == 2
    # pairs are reactions with exactly opposite net changes: switching, and
    # synthesis/decay of mRNA and of protein
    assert lx.Network(W.telegraph().m, W.telegraph().p).info()["n_pairs"] == 3


def test_prepare_compiles_without_a_gpu(tmp_path, monkeypatch):
    net = lx.Network(W.schlogl().m, W.schlogl().p)
    net.prepare("mixed", "batched")
    with pytest.raises(lx.LxError):
        net.prepare("fp64", "plain", block_size=512)


def test_argument_validation_before_any_device_call():
    L = lx.lib()
    net = lx.Network(W.dimer().m, W.dimer().p)
    o = lx.options()
    # P = 0 is a no-op; null buffers with P > 0 are rejected
    assert L.lx_simulate(net.handle, 0, None, None, 1.0, 0.03, 0, C.byref(o), None, None, None,
                         None, None) == 0
    assert L.lx_simulate(net.handle, 5, None, None, 1.0, 0.03, 0, C.byref(o), None, None, None,
                         None, None) == -1
    for bad in (dict(eps=-1.0), dict(mode=3), dict(t_end=-1.0)):
        kw = dict(eps=0.03, mode=0, t_end=1.0)
        kw.update(bad)
        assert L.lx_simulate(net.handle, 0, None, None, kw["t_end"], kw["eps"], kw["mode"],
                             C.byref(o), None, None, None, None, None) == -1
    for field, value in (("lambda_thr", 50.0), ("lambda_thr", 9.5), ("n_ssa_ex", 0), ("lanes_per_wave", 12),
                         ("ssa_k", 65), ("blocks_per_cu", 9), ("max_steps", 1 << 33),
                         ("block_size", 96), ("precision", 2), ("regroup", 65), ("lanes_per_traj", 3), ("lanes_per_traj", 32)):
        ob = lx.options(**{field: value})
        assert L.lx_simulate(net.handle, 0, None, None, 1.0, 0.03, 0, C.byref(ob), None, None,
                             None, None, None) == -1, field
    # particle ids beyond 2^32
    ob = lx.options(pid_base=2**32 - 10, pid_stride=4)
    assert L.lx_simulate(net.handle, 5, None, None, 1.0, 0.03, 0, C.byref(ob), None, None, None,
                         None, None) == -1
    # set: K out of range, null items
    assert L.lx_simulate_set(0, None, 1.0, 0.03, 0, None, None) == -1
    assert L.lx_simulate_set(9, None, 1.0, 0.03, 0, None, None) == -1
    # hooks: n = 0 is a no-op, bad arguments rejected
    assert L.lx_test_philox(0, None, None, None, None) == 0
    assert L.lx_test_math(7, 1, None, None, None) == -1
    assert L.lx_test_poisson(1, None, None, None, None, 0, 0, 10.0, 0, None, None) == -1
