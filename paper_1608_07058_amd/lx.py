"""Python binding of liblx (include/lx.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; this module
converts numpy/torch inputs into the C ABI's pointers and sizes.  torch
provides device memory and the stream.  If ``liblx.so`` is missing the import
fails loudly: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblx.so")

MODES = {"adaptive": 0, "explicit": 1, "ssa": 2}
JACOBIANS = {"analytic": 0, "fd": 1, "user": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
SCHEDULES = {"plain": 0, "batched": 1}
LANE_STATUS = {0: "OK", 1: "STEP_BUDGET", 2: "LAMBDA_OVERFLOW", 3: "BAD_INPUT",
               4: "COUNT_OVERFLOW"}

EXPORTS = (
    "lx_options_default", "lx_last_error", "lx_network_create", "lx_network_prepare",
    "lx_network_destroy", "lx_network_info", "lx_simulate", "lx_test_philox",
    "lx_test_uniform_f64", "lx_test_uniform_f32", "lx_test_math", "lx_test_poisson",
    "lx_test_exponential", "lx_test_tau_select", "lx_test_implicit", "lx_simulate_set",
    "lx_pf_workspace_size", "lx_pf_run", "lx_pf_graph_create", "lx_pf_graph_launch",
    "lx_pf_graph_destroy", "lx_test_gamma", "lx_simulate_grid", "lx_pf_run_static",
    "lx_network_create_jac",
)


class LxError(RuntimeError):
    pass


class PfProblem(C.Structure):
    _fields_ = [
        ("net", C.c_void_p), ("P", C.c_int64), ("K", C.c_int32), ("obs_species", C.c_int32),
        ("dt", C.c_double), ("obs_sd", C.c_double), ("y", C.c_void_p), ("alpha", C.c_void_p),
        ("beta", C.c_void_p), ("theta", C.c_void_p), ("x", C.c_void_p), ("r", C.c_void_p),
        ("G", C.c_void_p), ("loglik", C.c_void_p), ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
    ]


class SetItem(C.Structure):
    _fields_ = [
        ("net", C.c_void_p), ("P", C.c_int64), ("theta", C.c_void_p), ("x0", C.c_void_p),
        ("x_out", C.c_void_p), ("r_out", C.c_void_p), ("G_out", C.c_void_p),
        ("stats", C.c_void_p), ("pid_base", C.c_uint32), ("pid_stride", C.c_uint32),
    ]


class Options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("schedule", C.c_int32), ("seed", C.c_uint64),
        ("rng_stream", C.c_uint32), ("pid_base", C.c_uint32), ("t_start", C.c_double),
        ("accumulate", C.c_int32), ("n_c", C.c_int32), ("delta", C.c_double),
        ("n_stiff", C.c_double), ("k_ssa", C.c_double), ("k_crit", C.c_double),
        ("n_ssa_ex", C.c_int32), ("n_ssa_im", C.c_int32), ("lambda_thr", C.c_double),
        ("newton_tol", C.c_double), ("newton_maxit", C.c_int32), ("block_size", C.c_int32),
        ("max_steps", C.c_int64), ("lanes_per_wave", C.c_int32), ("ssa_k", C.c_int32),
        ("blocks_per_cu", C.c_int32), ("pid_stride", C.c_uint32), ("regroup", C.c_int32), ("lanes_per_traj", C.c_int32), ("jacobian", C.c_int32),
        ("check_lanes", C.c_int32), ("cycles", C.c_uint64),
        ("tail_lanes", C.c_int32), ("waves_per_simd", C.c_int32),
    ]


STATS_DTYPE = np.dtype([
    ("status", np.int32), ("crit_fired", np.uint32), ("t_final", np.float64),
    ("steps_ssa", np.int64), ("steps_explicit", np.int64), ("steps_implicit", np.int64),
    ("rejections", np.int64), ("newton_iters", np.int64), ("newton_fail", np.int64),
    ("kclip", np.int64), ("attempts", np.int64),
])
STATS_WORDS = STATS_DTYPE.itemsize // 8  # stats are carried in an int64 tensor

_lib = None


def lib():
    """Load liblx.so (raises if it has not been built).

    torch is imported first: its HIP runtime is then the one liblx binds to,
    so that device memory and streams of torch tensors and the library's
    kernels belong to one runtime (loading liblx first would bring in a
    second copy of the runtime next to torch's)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LxError(f"{LIB_PATH} is missing: build it with paper_1608_07058_amd/build.py")
        import torch  # noqa: F401  (see above)
        L = C.CDLL(LIB_PATH)
        P, I32, I64, U32, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.lx_options_default.argtypes = [C.POINTER(Options)]
        L.lx_options_default.restype = None
        L.lx_last_error.restype = C.c_char_p
        L.lx_network_create.argtypes = [I32, I32, P, P, C.POINTER(C.c_void_p)]
        L.lx_network_create_jac.argtypes = [I32, I32, P, P, I32, P, P, P, P,
                                            C.POINTER(C.c_void_p)]
        L.lx_network_prepare.argtypes = [P, I32, I32, I32]
        L.lx_network_destroy.argtypes = [P]
        L.lx_network_info.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]
        L.lx_simulate.argtypes = [P, I64, P, P, D, D, I32, C.POINTER(Options), P, P, P, P, P]
        L.lx_simulate_grid.argtypes = [P, I64, P, P, I32, P, D, I32, C.POINTER(Options), P, P, P,
                                       P, P, P]
        L.lx_simulate_set.argtypes = [I32, C.POINTER(SetItem), D, D, I32, C.POINTER(Options), P]
        L.lx_pf_workspace_size.argtypes = [I64, I32, I32, C.POINTER(C.c_size_t)]
        L.lx_pf_run.argtypes = [C.POINTER(PfProblem), D, I32, C.POINTER(Options), P]
        L.lx_pf_run_static.argtypes = [C.POINTER(PfProblem), D, I32, C.POINTER(Options), P]
        L.lx_pf_graph_create.argtypes = [C.POINTER(PfProblem), D, I32, C.POINTER(Options), P,
                                         C.POINTER(C.c_void_p)]
        L.lx_pf_graph_launch.argtypes = [P, P]
        L.lx_pf_graph_destroy.argtypes = [P]
        L.lx_test_gamma.argtypes = [I64, P, P, P, P, U64, U32, P, P]
        L.lx_test_philox.argtypes = [I64, P, P, P, P]
        L.lx_test_uniform_f64.argtypes = [I64, P, P, P]
        L.lx_test_uniform_f32.argtypes = [I64, P, P, P]
        L.lx_test_math.argtypes = [I32, I64, P, P, P]
        L.lx_test_poisson.argtypes = [I64, P, P, P, P, U64, U32, D, I32, P, P]
        L.lx_test_exponential.argtypes = [I64, P, P, U64, U32, I32, P, P]
        L.lx_test_tau_select.argtypes = [P, I64, P, P, D, I32, C.POINTER(Options), P, P, P, P, P, P]
        L.lx_test_implicit.argtypes = [P, I64, P, P, P, P, P, C.POINTER(Options), P, P, P, P]
        for name in EXPORTS:
            fn = getattr(L, name)
            if name not in ("lx_options_default", "lx_last_error"):
                fn.restype = C.c_int32
        if C.sizeof(Options) != 160:
            raise LxError("lx_options layout mismatch")
        _lib = L
    return _lib


class LaneFailWarning(UserWarning):
    """Some trajectories ended with a status other than OK (check_lanes=1)."""


LX_W_LANE_FAIL = 1


def _check(rc: int, what: str):
    if rc == LX_W_LANE_FAIL:
        import warnings
        msg = lib().lx_last_error().decode(errors="replace")
        warnings.warn(f"{what}: {msg}", LaneFailWarning, stacklevel=3)
    elif rc != 0:
        msg = lib().lx_last_error().decode(errors="replace")
        raise LxError(f"{what} failed ({rc}): {msg}")


def options(**kw) -> Options:
    o = Options()
    lib().lx_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "schedule" and isinstance(v, str):
            v = SCHEDULES[v]
        if k == "jacobian" and isinstance(v, str):
            v = JACOBIANS[v]
        if k not in dict(Options._fields_):
            raise KeyError(f"unknown option {k!r}")
        setattr(o, k, v)
    return o


class Network:
    """A compiled reaction network (lx_network_create)."""

    def __init__(self, reactant_order, product_coeff, jacobian_terms=None):
        """``jacobian_terms=(rxn, wrt, coef, powers)``: derivative terms for
        jacobian="user" (lx_network_create_jac)."""
        m = np.ascontiguousarray(reactant_order, dtype=np.int32)
        p = np.ascontiguousarray(product_coeff, dtype=np.int32)
        if m.ndim != 2 or m.shape != p.shape:
            raise ValueError("reactant/product tables must both be [M][N]")
        self.M, self.N = m.shape
        h = C.c_void_p()
        if jacobian_terms is None:
            _check(lib().lx_network_create(self.N, self.M, m.ctypes.data, p.ctypes.data,
                                           C.byref(h)), "lx_network_create")
        else:
            rxn, wrt, coef, pw = jacobian_terms
            rxn = np.ascontiguousarray(rxn, np.int32)
            wrt = np.ascontiguousarray(wrt, np.int32)
            coef = np.ascontiguousarray(coef, np.float64)
            pw = np.ascontiguousarray(pw, np.int32).reshape(len(rxn), self.N)
            _check(lib().lx_network_create_jac(self.N, self.M, m.ctypes.data, p.ctypes.data,
                                               len(rxn), rxn.ctypes.data, wrt.ctypes.data,
                                               coef.ctypes.data, pw.ctypes.data, C.byref(h)),
                   "lx_network_create_jac")
        self._h = h

    @property
    def large(self):
        """Beyond 16 species or 32 reactions: the large-network kernels."""
        return self.N > 16 or self.M > 32

    @property
    def handle(self):
        return self._h

    def info(self):
        n, m, q = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lx_network_info(self._h, C.byref(n), C.byref(m), C.byref(q)), "lx_network_info")
        return {"N": n.value, "M": m.value, "n_pairs": q.value}

    def prepare(self, precision="fp64", schedule="plain", block_size=0):
        _check(lib().lx_network_prepare(self._h, PRECISIONS.get(precision, precision),
                                        SCHEDULES.get(schedule, schedule), block_size),
               "lx_network_prepare")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lx_network_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous {dtype} of shape {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def simulate(net: Network, theta, x0, t_end: float, eps: float = 0.03, mode="adaptive", *,
             out=None, with_stats=True, stream=None, **opts):
    """lx_simulate on device tensors.

    theta: float64 [P][M], x0: int32 [P][N] (CUDA tensors).  ``out`` may hold
    preallocated ``x``, ``r``, ``G`` (and ``stats``) tensors; with
    ``accumulate=1`` r and G are read as starting values.  Returns a dict of
    tensors; ``stats`` is an int64 [P][10] view of lx_stats records.
    """
    import torch
    P = theta.shape[0]
    dev = theta.device
    th = _dev(theta, torch.float64, (P, net.M), "theta")
    xi = _dev(x0, torch.int32, (P, net.N), "x0")
    out = dict(out or {})
    if "x" not in out:
        out["x"] = torch.empty((P, net.N), dtype=torch.int32, device=dev)
    if "r" not in out:
        out["r"] = torch.zeros((P, net.M), dtype=torch.int32, device=dev)
    if "G" not in out:
        out["G"] = torch.zeros((P, net.M), dtype=torch.float64, device=dev)
    if with_stats and "stats" not in out:
        out["stats"] = torch.empty((P, STATS_WORDS), dtype=torch.int64, device=dev)
    xo = _dev(out["x"], torch.int32, (P, net.N), "x_out")
    ro = _dev(out["r"], torch.int32, (P, net.M), "r_out")
    go = _dev(out["G"], torch.float64, (P, net.M), "G_out")
    so = _dev(out["stats"], torch.int64, (P, STATS_WORDS), "stats") if with_stats else None
    o = options(**opts)
    _check(lib().lx_simulate(net.handle, P, th, xi, float(t_end), float(eps),
                             MODES.get(mode, mode), C.byref(o), xo, ro, go, so,
                             _stream_ptr(stream)), "lx_simulate")
    return out


def simulate_grid(net: Network, theta, x0, times, eps: float = 0.03, mode="adaptive", *,
                  out=None, with_stats=True, stream=None, **opts):
    """lx_simulate_grid on device tensors: ``simulate`` that also records the
    state at each observation time.  ``times`` is a float64 [K] CUDA tensor
    (non-decreasing, from t_start; the last one ends the simulation).  Returns
    the dict of ``simulate`` plus ``x_grid`` int32 [P][K][N] (-1 in rows whose
    time a trajectory did not reach with status OK).
    """
    import torch
    P = theta.shape[0]
    dev = theta.device
    K = int(times.shape[0]) if times.dim() == 1 else -1
    tt = _dev(times, torch.float64, (max(K, 0),), "times")
    th = _dev(theta, torch.float64, (P, net.M), "theta")
    xi = _dev(x0, torch.int32, (P, net.N), "x0")
    out = dict(out or {})
    if "x_grid" not in out:
        out["x_grid"] = torch.empty((P, max(K, 0), net.N), dtype=torch.int32, device=dev)
    if "x" not in out:
        out["x"] = torch.empty((P, net.N), dtype=torch.int32, device=dev)
    if "r" not in out:
        out["r"] = torch.zeros((P, net.M), dtype=torch.int32, device=dev)
    if "G" not in out:
        out["G"] = torch.zeros((P, net.M), dtype=torch.float64, device=dev)
    if with_stats and "stats" not in out:
        out["stats"] = torch.empty((P, STATS_WORDS), dtype=torch.int64, device=dev)
    xg = _dev(out["x_grid"], torch.int32, (P, max(K, 0), net.N), "x_grid")
    xo = _dev(out["x"], torch.int32, (P, net.N), "x_out")
    ro = _dev(out["r"], torch.int32, (P, net.M), "r_out")
    go = _dev(out["G"], torch.float64, (P, net.M), "G_out")
    so = _dev(out["stats"], torch.int64, (P, STATS_WORDS), "stats") if with_stats else None
    o = options(**opts)
    _check(lib().lx_simulate_grid(net.handle, P, th, xi, K, tt, float(eps), MODES.get(mode, mode),
                                  C.byref(o), xg, xo, ro, go, so, _stream_ptr(stream)),
           "lx_simulate_grid")
    return out


def simulate_set(items, t_end: float, eps: float = 0.03, mode="adaptive", *, with_stats=True,
                 stream=None, **opts):
    """lx_simulate_set: ``items`` is a list of dicts with keys net, theta, x0
    and optionally pid_base, pid_stride and out (preallocated x/r/G/stats).
    Returns one output dict per item."""
    import torch
    arr = (SetItem * len(items))()
    outs = []
    for k, it in enumerate(items):
        net, theta, x0 = it["net"], it["theta"], it["x0"]
        P = theta.shape[0]
        dev = theta.device
        out = dict(it.get("out") or {})
        out.setdefault("x", torch.empty((P, net.N), dtype=torch.int32, device=dev))
        out.setdefault("r", torch.zeros((P, net.M), dtype=torch.int32, device=dev))
        out.setdefault("G", torch.zeros((P, net.M), dtype=torch.float64, device=dev))
        if with_stats:
            out.setdefault("stats", torch.empty((P, STATS_WORDS), dtype=torch.int64, device=dev))
        d = arr[k]
        d.net = net.handle.value
        d.P = P
        d.theta = _dev(theta, torch.float64, (P, net.M), "theta").value
        d.x0 = _dev(x0, torch.int32, (P, net.N), "x0").value
        d.x_out = _dev(out["x"], torch.int32, (P, net.N), "x_out").value
        d.r_out = _dev(out["r"], torch.int32, (P, net.M), "r_out").value
        d.G_out = _dev(out["G"], torch.float64, (P, net.M), "G_out").value
        d.stats = (_dev(out["stats"], torch.int64, (P, STATS_WORDS), "stats").value
                   if with_stats else None)
        d.pid_base = int(it.get("pid_base", 0))
        d.pid_stride = int(it.get("pid_stride", 0))
        outs.append(out)
    o = options(**opts)
    _check(lib().lx_simulate_set(len(items), arr, float(t_end), float(eps), MODES.get(mode, mode),
                                 C.byref(o), _stream_ptr(stream)), "lx_simulate_set")
    return outs


class ParticleFilter:
    """lx_pf_*: particle filter over K observation intervals on device tensors.

    theta [P][M] f64, x [P][N] i32 (updated in place), y [K], alpha/beta [M].
    Allocates r, G, loglik and (unless ``workspace=False``) the workspace with
    torch.  ``run()`` enqueues direct launches; ``capture(stream)`` records a
    HIP graph once and ``replay(stream)`` launches it; ``run_static()`` is
    lx_pf_run_static, which uses the library's own scratch instead of the
    workspace.
    """

    def __init__(self, net, theta, x, y, alpha, beta, dt, obs_species, obs_sd, eps=0.03,
                 mode="adaptive", workspace=True, **opts):
        import torch
        self.net = net
        P, K = theta.shape[0], y.shape[0]
        dev = theta.device
        self.theta, self.x = theta, x
        self.y = y.to(torch.float64).contiguous()
        self.alpha = alpha.to(torch.float64).contiguous()
        self.beta = beta.to(torch.float64).contiguous()
        self.r = torch.zeros((P, net.M), dtype=torch.int32, device=dev)
        self.G = torch.zeros((P, net.M), dtype=torch.float64, device=dev)
        self.loglik = torch.empty(K, dtype=torch.float64, device=dev)
        nb = C.c_size_t()
        _check(lib().lx_pf_workspace_size(P, net.N, net.M, C.byref(nb)), "lx_pf_workspace_size")
        if workspace:
            self.work = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
            base = self.work.data_ptr()
            aligned = (base + 255) // 256 * 256
        else:
            self.work, aligned, nb = None, None, C.c_size_t(0)
        pb = PfProblem()
        pb.net = net.handle.value
        pb.P, pb.K, pb.obs_species = P, K, obs_species
        pb.dt, pb.obs_sd = float(dt), float(obs_sd)
        pb.y = _dev(self.y, torch.float64, (K,), "y").value
        pb.alpha = _dev(self.alpha, torch.float64, (net.M,), "alpha").value
        pb.beta = _dev(self.beta, torch.float64, (net.M,), "beta").value
        pb.theta = _dev(theta, torch.float64, (P, net.M), "theta").value
        pb.x = _dev(x, torch.int32, (P, net.N), "x").value
        pb.r = self.r.data_ptr()
        pb.G = self.G.data_ptr()
        pb.loglik = self.loglik.data_ptr()
        pb.workspace = aligned
        pb.workspace_bytes = nb.value
        self.pb = pb
        self.eps, self.mode = float(eps), MODES.get(mode, mode)
        self.opts = options(**opts)
        self.graph = C.c_void_p()

    def run(self, stream=None):
        _check(lib().lx_pf_run(C.byref(self.pb), self.eps, self.mode, C.byref(self.opts),
                               _stream_ptr(stream)), "lx_pf_run")

    def run_static(self, stream=None):
        _check(lib().lx_pf_run_static(C.byref(self.pb), self.eps, self.mode, C.byref(self.opts),
                                      _stream_ptr(stream)), "lx_pf_run_static")

    def capture(self, stream):
        self.release()
        _check(lib().lx_pf_graph_create(C.byref(self.pb), self.eps, self.mode, C.byref(self.opts),
                                        _stream_ptr(stream), C.byref(self.graph)),
               "lx_pf_graph_create")

    def replay(self, stream=None):
        _check(lib().lx_pf_graph_launch(self.graph, _stream_ptr(stream)), "lx_pf_graph_launch")

    def release(self):
        if self.graph.value:
            lib().lx_pf_graph_destroy(self.graph)
            self.graph = C.c_void_p()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def test_gamma(shape, pid, e, j, *, seed=160807058, stream_id=0, device="cuda"):
    import torch
    shape = np.asarray(shape, np.float64).reshape(-1)
    n = shape.shape[0]
    u = lambda v: _t(np.broadcast_to(np.asarray(v, np.uint32), n).view(np.int32), torch.int32, device)
    st = _t(shape, torch.float64, device)
    pt, et, jt = u(pid), u(e), u(j)
    out = torch.empty(n, dtype=torch.float64, device=device)
    _check(lib().lx_test_gamma(n, _ptr(st), _ptr(pt), _ptr(et), _ptr(jt), seed, stream_id,
                               _ptr(out), _stream_ptr(None)), "lx_test_gamma")
    return out.cpu().numpy()


def stats_numpy(stats_tensor) -> np.ndarray:
    """Structured numpy view of an lx_stats tensor."""
    a = stats_tensor.detach().cpu().numpy()
    return a.view(STATS_DTYPE).reshape(-1)


# ---- test hooks -----------------------------------------------------------

def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev).to(dtype).contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def test_philox(ctr, key, device="cuda"):
    import torch
    c = _t(np.asarray(ctr, np.uint32).view(np.int32).reshape(-1, 4), torch.int32, device)
    k = _t(np.asarray(key, np.uint32).view(np.int32).reshape(-1, 2), torch.int32, device)
    out = torch.empty_like(c)
    _check(lib().lx_test_philox(c.shape[0], _ptr(c), _ptr(k), _ptr(out), _stream_ptr(None)),
           "lx_test_philox")
    return out.cpu().numpy().view(np.uint32)


def test_uniform_f64(w, device="cuda"):
    import torch
    ww = _t(np.asarray(w, np.uint32).view(np.int32).reshape(-1, 2), torch.int32, device)
    out = torch.empty(ww.shape[0], dtype=torch.float64, device=device)
    _check(lib().lx_test_uniform_f64(ww.shape[0], _ptr(ww), _ptr(out), _stream_ptr(None)),
           "lx_test_uniform_f64")
    return out.cpu().numpy()


def test_uniform_f32(w, device="cuda"):
    import torch
    ww = _t(np.asarray(w, np.uint32).view(np.int32).reshape(-1), torch.int32, device)
    out = torch.empty(ww.shape[0], dtype=torch.float32, device=device)
    _check(lib().lx_test_uniform_f32(ww.shape[0], _ptr(ww), _ptr(out), _stream_ptr(None)),
           "lx_test_uniform_f32")
    return out.cpu().numpy()


MATH_FN = {"exp_f64": 0, "log_f64": 1, "lfact": 2, "sqrt_f64": 3, "exp_f32": 10, "log_f32": 11,
           "sqrt_f32": 12}


def test_math(fn, x, device="cuda"):
    import torch
    code = MATH_FN[fn]
    dt = torch.float64 if code < 10 else torch.float32
    xs = _t(np.asarray(x).reshape(-1), dt, device)
    out = torch.empty_like(xs)
    _check(lib().lx_test_math(code, xs.shape[0], _ptr(xs), _ptr(out), _stream_ptr(None)),
           "lx_test_math")
    return out.cpu().numpy()


def test_poisson(lam, pid, e, site, *, seed=160807058, stream_id=0, lambda_thr=15.0,
                 precision="fp64", device="cuda"):
    import torch
    lam = np.asarray(lam, np.float64).reshape(-1)
    n = lam.shape[0]
    u = lambda v: _t(np.broadcast_to(np.asarray(v, np.uint32), n).view(np.int32), torch.int32, device)
    lt = _t(lam, torch.float64, device)
    pt, et, st = u(pid), u(e), u(site)
    out = torch.empty(n, dtype=torch.int64, device=device)
    _check(lib().lx_test_poisson(n, _ptr(lt), _ptr(pt), _ptr(et), _ptr(st), seed, stream_id,
                                 float(lambda_thr), PRECISIONS.get(precision, precision),
                                 _ptr(out), _stream_ptr(None)), "lx_test_poisson")
    return out.cpu().numpy()


def test_exponential(pid, e, *, seed=160807058, stream_id=0, precision="fp64", device="cuda"):
    import torch
    pid = np.asarray(pid, np.uint32).reshape(-1)
    n = pid.shape[0]
    pt = _t(pid.view(np.int32), torch.int32, device)
    et = _t(np.broadcast_to(np.asarray(e, np.uint32), n).view(np.int32), torch.int32, device)
    out = torch.empty(n, dtype=torch.float64, device=device)
    _check(lib().lx_test_exponential(n, _ptr(pt), _ptr(et), seed, stream_id,
                                     PRECISIONS.get(precision, precision), _ptr(out),
                                     _stream_ptr(None)), "lx_test_exponential")
    return out.cpu().numpy()


def test_tau_select(net: Network, theta, x, eps=0.03, mode="adaptive", device="cuda", **opts):
    import torch
    x = np.asarray(x, np.int32).reshape(-1, net.N)
    Q = x.shape[0]
    th = np.broadcast_to(np.asarray(theta, np.float64).reshape(-1, net.M), (Q, net.M))
    tt, xt = _t(th, torch.float64, device), _t(x, torch.int32, device)
    a = torch.empty((Q, net.M), dtype=torch.float64, device=device)
    W = (net.M + 31) // 32  # mask words per case
    crit = torch.empty((Q, W), dtype=torch.int32, device=device)
    eq = torch.empty((Q, W), dtype=torch.int32, device=device)
    tau = torch.empty((Q, 2), dtype=torch.float64, device=device)
    act = torch.empty(Q, dtype=torch.int32, device=device)
    o = options(**opts)
    _check(lib().lx_test_tau_select(net.handle, Q, _ptr(tt), _ptr(xt), float(eps),
                                    MODES.get(mode, mode), C.byref(o), _ptr(a), _ptr(crit),
                                    _ptr(eq), _ptr(tau), _ptr(act), _stream_ptr(None)),
           "lx_test_tau_select")
    bits = lambda m: ((m.cpu().numpy().view(np.uint32)[:, :, None] >> np.arange(32, dtype=np.uint32))
                      & 1).reshape(Q, W * 32)[:, :net.M].astype(np.int32)
    return {"a": a.cpu().numpy(), "crit": bits(crit), "eq": bits(eq),
            "tau_ex": tau[:, 0].cpu().numpy(), "tau_im": tau[:, 1].cpu().numpy(),
            "action": act.cpu().numpy()}


def test_implicit(net: Network, theta, x, tau, Pj, jc, device="cuda", **opts):
    import torch
    x = np.asarray(x, np.int32).reshape(-1, net.N)
    Q = x.shape[0]
    th = np.broadcast_to(np.asarray(theta, np.float64).reshape(-1, net.M), (Q, net.M))
    tt, xt = _t(th, torch.float64, device), _t(x, torch.int32, device)
    taut = _t(np.broadcast_to(np.asarray(tau, np.float64), Q), torch.float64, device)
    pt = _t(np.asarray(Pj, np.int64).reshape(Q, net.M), torch.int64, device)
    jt = _t(np.broadcast_to(np.asarray(jc, np.int32), Q), torch.int32, device)
    k = torch.empty((Q, net.M), dtype=torch.int64, device=device)
    ok = torch.empty(Q, dtype=torch.int32, device=device)
    it = torch.empty(Q, dtype=torch.int32, device=device)
    o = options(**opts)
    _check(lib().lx_test_implicit(net.handle, Q, _ptr(tt), _ptr(xt), _ptr(taut), _ptr(pt),
                                  _ptr(jt), C.byref(o), _ptr(k), _ptr(ok), _ptr(it),
                                  _stream_ptr(None)), "lx_test_implicit")
    return {"k": k.cpu().numpy(), "ok": ok.cpu().numpy().astype(bool), "iters": it.cpu().numpy()}
