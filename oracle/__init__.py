"""CPU oracle for ensemble adaptive explicit/implicit tau-leaping (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links, calls
or falls back to it.  It wraps ``liblx_oracle.so`` (built from
``lx_oracle.cpp`` with g++, ``build()`` below) through ctypes and numpy.

The method follows matLeap (arXiv 1608.07058): propensities a_j = theta_j g_j(X)
and the summary statistics r_j, G_j (Background section); the adaptive
explicit/implicit tau-leap with critical reactions and the SSA switch
(Implementation section).  The per-step readings are documented in
``lx_oracle.cpp``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lx_oracle.cpp")
_LIB = os.path.join(_HERE, "liblx_oracle.so")

MODES = {"adaptive": 0, "explicit": 1, "ssa": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
STATUS = {0: "OK", 1: "STEP_BUDGET", 2: "LAMBDA_OVERFLOW", 3: "BAD_INPUT", 4: "COUNT_OVERFLOW"}
SITE_CRIT = 0x40000000
SITE_SSA = 0x40000001


class Options(C.Structure):
    _fields_ = [
        ("eps", C.c_double), ("delta", C.c_double), ("n_stiff", C.c_double),
        ("k_ssa", C.c_double), ("k_crit", C.c_double), ("lambda_thr", C.c_double),
        ("newton_tol", C.c_double), ("t_start", C.c_double),
        ("max_steps", C.c_int64), ("seed", C.c_uint64),
        ("n_c", C.c_int32), ("n_ssa_ex", C.c_int32), ("n_ssa_im", C.c_int32),
        ("newton_maxit", C.c_int32), ("rng_stream", C.c_uint32), ("pid_base", C.c_uint32),
        ("accumulate", C.c_int32), ("mode", C.c_int32), ("precision", C.c_int32),
        ("nthreads", C.c_int32), ("pid_stride", C.c_uint32), ("jacobian", C.c_int32),
        ("n_jt", C.c_int32), ("jt_rxn", C.c_void_p), ("jt_wrt", C.c_void_p),
        ("jt_coef", C.c_void_p), ("jt_pow", C.c_void_p),
    ]


STATS_DTYPE = np.dtype([
    ("status", np.int32), ("crit_fired", np.uint32), ("t_final", np.float64),
    ("steps_ssa", np.int64), ("steps_explicit", np.int64), ("steps_implicit", np.int64),
    ("rejections", np.int64), ("newton_iters", np.int64), ("newton_fail", np.int64),
    ("kclip", np.int64), ("attempts", np.int64), ("ops", np.int64),
])


def build(force: bool = True) -> str:
    """Compile ``liblx_oracle.so`` with g++ (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-Wall", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_default_options.argtypes = [C.POINTER(Options)]
        L.orc_options_size.restype = C.c_int
        L.orc_stats_size.restype = C.c_int
        L.orc_simulate.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int64, P, P, C.c_double,
                                   C.POINTER(Options), P, P, P, P]
        L.orc_simulate.restype = C.c_int
        L.orc_simulate_grid.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int64, P, P, C.c_int32,
                                        P, C.POINTER(Options), P, P, P, P, P]
        L.orc_simulate_grid.restype = C.c_int
        L.orc_philox.argtypes = [C.c_int64, P, P, P]
        L.orc_uniform_f64.argtypes = [C.c_int64, P, P]
        L.orc_uniform_f32.argtypes = [C.c_int64, P, P]
        for nm in ("orc_exp_f64", "orc_log_f64", "orc_exp_f32", "orc_log_f32", "orc_lfact"):
            getattr(L, nm).argtypes = [C.c_int64, P, P]
        L.orc_poisson.argtypes = [C.c_int64, P, P, P, P, C.c_uint64, C.c_uint32, C.c_double,
                                  C.c_int32, P]
        L.orc_exponential.argtypes = [C.c_int64, P, P, C.c_uint64, C.c_uint32, C.c_int32, P]
        L.orc_ptrs_log_density.argtypes = [C.c_int64, P, P, C.c_int32, P, P]
        L.orc_tau_select.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int64, P, P,
                                     C.POINTER(Options), P, P, P, P, P]
        L.orc_tau_select.restype = C.c_int
        L.orc_implicit.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int64, P, P, P, P, P,
                                   C.POINTER(Options), P, P, P, P]
        L.orc_implicit.restype = C.c_int
        L.orc_gamma.argtypes = [C.c_int64, P, P, P, P, C.c_uint64, C.c_uint32, P]
        L.orc_resample.argtypes = [C.c_int64, P, C.c_uint64, C.c_uint32, C.c_uint32, P]
        L.orc_pf_run.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int64, C.c_int32, C.c_double,
                                 C.c_int32, C.c_double, P, P, P, P, P, P, P, P,
                                 C.POINTER(Options)]
        L.orc_pf_run.restype = C.c_int
        L.orc_pf_last_ops.argtypes = []
        L.orc_pf_last_ops.restype = C.c_double
        assert L.orc_options_size() == C.sizeof(Options)
        assert L.orc_stats_size() == STATS_DTYPE.itemsize
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


JACOBIANS = {"analytic": 0, "fd": 1, "user": 2}


def options(**kw) -> Options:
    """Oracle options; ``jacobian_terms=(rxn, wrt, coef, powers)`` supplies
    derivative terms (with ``jacobian="user"``), kept alive by the returned
    object."""
    o = Options()
    lib().orc_default_options(C.byref(o))
    terms = kw.pop("jacobian_terms", None)
    if terms is not None:
        rxn, wrt, coef, pw = terms
        arrs = (np.ascontiguousarray(rxn, np.int32), np.ascontiguousarray(wrt, np.int32),
                np.ascontiguousarray(coef, np.float64), np.ascontiguousarray(pw, np.int32))
        o._keep = arrs
        o.n_jt = len(arrs[0])
        o.jt_rxn, o.jt_wrt, o.jt_coef, o.jt_pow = (a.ctypes.data for a in arrs)
    for k, v in kw.items():
        if k == "jacobian" and isinstance(v, str):
            v = JACOBIANS[v]
        if k == "mode" and isinstance(v, str):
            v = MODES[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(o, k):
            raise KeyError(f"unknown oracle option {k!r}")
        setattr(o, k, v)
    return o


def _net_arrays(m, p):
    m = np.ascontiguousarray(m, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.int32)
    if m.ndim != 2 or m.shape != p.shape:
        raise ValueError("reactant/product tables must both be [M][N]")
    return m, p


def simulate(m, p, theta, x0, t_end, *, r0=None, G0=None, **kw):
    """Run the oracle on P trajectories.

    m, p: [M][N] reactant orders and product coefficients; theta [P][M];
    x0 [P][N].  Keyword options as in ``Options`` (mode/precision may be
    strings).  Returns dict with x [P][N] int32, r [P][M] int32, G [P][M]
    float64 and stats (structured array).
    """
    m, p = _net_arrays(m, p)
    M, N = m.shape
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    P = theta.shape[0]
    if theta.shape != (P, M) or x0.shape != (P, N):
        raise ValueError("theta must be [P][M] and x0 [P][N]")
    kw.setdefault("nthreads", min(16, os.cpu_count() or 1))
    o = options(**kw)
    x = np.empty((P, N), np.int32)
    r = np.zeros((P, M), np.int32) if r0 is None else np.array(r0, dtype=np.int32, copy=True)
    G = np.zeros((P, M), np.float64) if G0 is None else np.array(G0, dtype=np.float64, copy=True)
    if r0 is not None or G0 is not None:
        o.accumulate = 1
    st = np.zeros(P, STATS_DTYPE)
    rc = lib().orc_simulate(N, M, _ptr(m), _ptr(p), P, _ptr(theta), _ptr(x0), float(t_end),
                            C.byref(o), _ptr(x), _ptr(r), _ptr(G), _ptr(st))
    if rc != 0:
        raise ValueError(f"oracle rejected the network or options (code {rc})")
    return {"x": x, "r": r, "G": G, "stats": st}


def simulate_grid(m, p, theta, x0, times, *, r0=None, G0=None, **kw):
    """``simulate`` with observation times: the state at each of ``times``
    (non-decreasing, from t_start; the last one ends the simulation) as
    x_grid [P][K][N] int32, -1 where a trajectory did not reach a time in
    status OK.  Returns the dict of ``simulate`` plus ``x_grid``."""
    m, p = _net_arrays(m, p)
    M, N = m.shape
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    times = np.ascontiguousarray(times, dtype=np.float64).reshape(-1)
    P, K = theta.shape[0], times.shape[0]
    if theta.shape != (P, M) or x0.shape != (P, N):
        raise ValueError("theta must be [P][M] and x0 [P][N]")
    if K < 1:
        raise ValueError("need at least one observation time")
    kw.setdefault("nthreads", min(16, os.cpu_count() or 1))
    o = options(**kw)
    xg = np.empty((P, K, N), np.int32)
    x = np.empty((P, N), np.int32)
    r = np.zeros((P, M), np.int32) if r0 is None else np.array(r0, dtype=np.int32, copy=True)
    G = np.zeros((P, M), np.float64) if G0 is None else np.array(G0, dtype=np.float64, copy=True)
    if r0 is not None or G0 is not None:
        o.accumulate = 1
    st = np.zeros(P, STATS_DTYPE)
    rc = lib().orc_simulate_grid(N, M, _ptr(m), _ptr(p), P, _ptr(theta), _ptr(x0), K,
                                 _ptr(times), C.byref(o), _ptr(xg), _ptr(x), _ptr(r), _ptr(G),
                                 _ptr(st))
    if rc != 0:
        raise ValueError(f"oracle rejected the network, options or times (code {rc})")
    return {"x_grid": xg, "x": x, "r": r, "G": G, "stats": st}


def philox(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().orc_philox(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def uniform_f64(w):
    w = np.ascontiguousarray(w, dtype=np.uint32).reshape(-1, 2)
    out = np.empty(w.shape[0], np.float64)
    lib().orc_uniform_f64(w.shape[0], _ptr(w), _ptr(out))
    return out


def uniform_f32(w):
    w = np.ascontiguousarray(w, dtype=np.uint32).reshape(-1)
    out = np.empty(w.shape[0], np.float32)
    lib().orc_uniform_f32(w.shape[0], _ptr(w), _ptr(out))
    return out


def _unary(name, x, dt):
    x = np.ascontiguousarray(x, dtype=dt).reshape(-1)
    out = np.empty_like(x)
    getattr(lib(), name)(x.shape[0], _ptr(x), _ptr(out))
    return out


def exp_f64(x): return _unary("orc_exp_f64", x, np.float64)
def log_f64(x): return _unary("orc_log_f64", x, np.float64)
def exp_f32(x): return _unary("orc_exp_f32", x, np.float32)
def log_f32(x): return _unary("orc_log_f32", x, np.float32)
def lfact(k): return _unary("orc_lfact", k, np.float64)


def poisson(lam, pid, e, site, *, seed=160807058, stream=0, lambda_thr=15.0, precision="fp64"):
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
    n = lam.shape[0]
    pid = np.ascontiguousarray(np.broadcast_to(pid, n), dtype=np.uint32)
    e = np.ascontiguousarray(np.broadcast_to(e, n), dtype=np.uint32)
    site = np.ascontiguousarray(np.broadcast_to(site, n), dtype=np.uint32)
    out = np.empty(n, np.int64)
    lib().orc_poisson(n, _ptr(lam), _ptr(pid), _ptr(e), _ptr(site), seed, stream,
                      float(lambda_thr), PRECISIONS.get(precision, precision), _ptr(out))
    return out


def ptrs_log_density(k, lam, *, precision="fp64"):
    """(factor, rhs) of the PTRS acceptance test: log p(k; lam) = rhs - log(factor)."""
    k, lam = np.broadcast_arrays(np.asarray(k, np.float64), np.asarray(lam, np.float64))
    k = np.ascontiguousarray(k).reshape(-1)
    lam = np.ascontiguousarray(lam).reshape(-1)
    n = k.shape[0]
    fac, rhs = np.empty(n), np.empty(n)
    lib().orc_ptrs_log_density(n, _ptr(k), _ptr(lam), PRECISIONS.get(precision, precision),
                               _ptr(fac), _ptr(rhs))
    return fac, rhs


def exponential(pid, e, *, seed=160807058, stream=0, precision="fp64"):
    pid = np.ascontiguousarray(pid, dtype=np.uint32).reshape(-1)
    n = pid.shape[0]
    e = np.ascontiguousarray(np.broadcast_to(e, n), dtype=np.uint32)
    out = np.empty(n, np.float64)
    lib().orc_exponential(n, _ptr(pid), _ptr(e), seed, stream,
                          PRECISIONS.get(precision, precision), _ptr(out))
    return out


def tau_select(m, p, theta, x, **kw):
    """Per-state decision quantities; see ``orc_tau_select`` in lx_oracle.cpp."""
    m, p = _net_arrays(m, p)
    M, N = m.shape
    x = np.ascontiguousarray(x, dtype=np.int32).reshape(-1, N)
    Q = x.shape[0]
    theta = np.ascontiguousarray(np.broadcast_to(np.asarray(theta, np.float64).reshape(-1, M),
                                                 (Q, M)))
    o = options(**kw)
    a = np.empty((Q, M), np.float64)
    crit = np.empty((Q, M), np.int32)
    eq = np.empty((Q, M), np.int32)
    tau = np.empty((Q, 2), np.float64)
    act = np.empty(Q, np.int32)
    rc = lib().orc_tau_select(N, M, _ptr(m), _ptr(p), Q, _ptr(theta), _ptr(x), C.byref(o),
                              _ptr(a), _ptr(crit), _ptr(eq), _ptr(tau), _ptr(act))
    if rc != 0:
        raise ValueError("invalid network")
    return {"a": a, "crit": crit, "eq": eq, "tau_ex": tau[:, 0], "tau_im": tau[:, 1],
            "action": act}


def implicit(m, p, theta, x, tau, Pj, jc, **kw):
    """Implicit-leap Newton solve on fixed inputs; see ``orc_implicit``."""
    m, p = _net_arrays(m, p)
    M, N = m.shape
    x = np.ascontiguousarray(x, dtype=np.int32).reshape(-1, N)
    Q = x.shape[0]
    theta = np.ascontiguousarray(np.broadcast_to(np.asarray(theta, np.float64).reshape(-1, M),
                                                 (Q, M)))
    tau = np.ascontiguousarray(np.broadcast_to(tau, Q), dtype=np.float64)
    Pj = np.ascontiguousarray(Pj, dtype=np.int64).reshape(Q, M)
    jc = np.ascontiguousarray(np.broadcast_to(jc, Q), dtype=np.int32)
    o = options(**kw)
    y = np.empty((Q, N), np.float64)
    k = np.empty((Q, M), np.int64)
    ok = np.empty(Q, np.int32)
    it = np.empty(Q, np.int32)
    rc = lib().orc_implicit(N, M, _ptr(m), _ptr(p), Q, _ptr(theta), _ptr(x), _ptr(tau), _ptr(Pj),
                            _ptr(jc), C.byref(o), _ptr(y), _ptr(k), _ptr(ok), _ptr(it))
    if rc != 0:
        raise ValueError("invalid network")
    return {"y": y, "k": k, "ok": ok.astype(bool), "iters": it}


SITE_RESAMPLE = 0x40000002
SITE_GAMMA = 0x40000010


def gamma(shape, pid, e, j, *, seed=160807058, stream=0):
    """Gamma(shape, 1) drawn at site (pid, e, SITE_GAMMA + j)."""
    shape = np.ascontiguousarray(shape, dtype=np.float64).reshape(-1)
    n = shape.shape[0]
    bc = lambda v: np.ascontiguousarray(np.broadcast_to(v, n), dtype=np.uint32)
    pid, e, j = bc(pid), bc(e), bc(j)
    out = np.empty(n, np.float64)
    lib().orc_gamma(n, _ptr(shape), _ptr(pid), _ptr(e), _ptr(j), seed, stream, _ptr(out))
    return out


def resample(codes, k, *, seed=160807058, stream=0):
    """Ancestors of len(codes) new particles from integer weight codes."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    anc = np.empty(codes.shape[0], np.int32)
    lib().orc_resample(codes.shape[0], _ptr(codes), seed, stream, k, _ptr(anc))
    return anc


def pf_run(m, p, theta, x0, K, dt, obs_species, obs_sd, y, alpha, beta, **kw):
    """Particle filter (see orc_pf_run); returns theta, x, r, G, loglik and ops,
    the algorithmic operation count of its simulations (all particles and
    intervals)."""
    m, p = _net_arrays(m, p)
    M, N = m.shape
    theta = np.array(theta, dtype=np.float64, copy=True)
    x = np.array(x0, dtype=np.int32, copy=True)
    P = theta.shape[0]
    r = np.zeros((P, M), np.int32)
    G = np.zeros((P, M), np.float64)
    ll = np.empty(K, np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    kw.setdefault("nthreads", min(16, os.cpu_count() or 1))
    o = options(**kw)
    rc = lib().orc_pf_run(N, M, _ptr(m), _ptr(p), P, K, float(dt), obs_species, float(obs_sd),
                          _ptr(y), _ptr(alpha), _ptr(beta), _ptr(theta), _ptr(x), _ptr(r),
                          _ptr(G), _ptr(ll), C.byref(o))
    if rc != 0:
        raise ValueError(f"oracle particle filter failed ({rc})")
    return {"theta": theta, "x": x, "r": r, "G": G, "loglik": ll,
            "ops": float(lib().orc_pf_last_ops())}
