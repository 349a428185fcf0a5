"""Seeded synthetic workloads: reaction networks, parameters and initial states.

This module only *generates inputs*: stoichiometry tables, rate constants and
initial copy numbers.  It holds none of the simulation method's arithmetic, so
both the CPU oracle (tests) and the GPU path may use it.

Networks are flat tables: ``m[j][i]`` is the number of molecules of species i
consumed by reaction j (reactant order) and ``p[j][i]`` the number produced.
The paper's own models (auto-regulatory gene network, Ras/cAMP/PKA, the stiff
decaying-dimerizing set) ship as SBML files that are not available; the
networks below are synthetic stand-ins with the shapes of the paper's
examples (Results section).  The decaying-dimerizing set takes the constants
c = (1, 0.002, 0.5, 0.04) from X0 = (10000, 0, 0); ``dimer_stiff`` speeds up
its reversible pair so that implicit leaps occur.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_SIM = 160807058  # default Philox seed of the simulations


@dataclass
class Network:
    name: str
    m: np.ndarray          # [M][N] reactant orders
    p: np.ndarray          # [M][N] product coefficients
    theta: np.ndarray      # [M] nominal rate constants
    x0: np.ndarray         # [N] nominal initial state
    species: tuple = ()
    reactions: tuple = ()

    @property
    def N(self) -> int:
        return int(self.m.shape[1])

    @property
    def M(self) -> int:
        return int(self.m.shape[0])


def _net(name, m, p, theta, x0, species=(), reactions=()):
    return Network(name, np.asarray(m, np.int32), np.asarray(p, np.int32),
                   np.asarray(theta, np.float64), np.asarray(x0, np.int32),
                   tuple(species), tuple(reactions))


def birth_death(k1=10.0, k2=0.1, x0=0) -> Network:
    """0 -> X (k1), X -> 0 (k2)."""
    return _net("birth_death", [[0], [1]], [[1], [0]], [k1, k2], [x0], ("X",),
                ("0->X", "X->0"))


def dimer(x0=(10000, 0, 0)) -> Network:
    """Decaying-dimerizing set: S1->0 (1), 2S1->S2 (0.002), S2->2S1 (0.5), S2->S3 (0.04)."""
    m = [[1, 0, 0], [2, 0, 0], [0, 1, 0], [0, 1, 0]]
    p = [[0, 0, 0], [0, 1, 0], [2, 0, 0], [0, 0, 1]]
    return _net("dimer", m, p, [1.0, 0.002, 0.5, 0.04], x0, ("S1", "S2", "S3"),
                ("S1->0", "2S1->S2", "S2->2S1", "S2->S3"))


def dimer_stiff(scale=1000.0, x0=(10000, 0, 0)) -> Network:
    """The decaying-dimerizing set with the reversible pair ``scale`` times faster.

    With the constants of ``dimer()`` the pair never dominates the step-size
    bound enough for an implicit leap; speeding it up makes the set stiff.
    """
    base = dimer(x0)
    theta = base.theta.copy()
    theta[1] *= scale
    theta[2] *= scale
    return _net("dimer_stiff", base.m, base.p, theta, x0, base.species, base.reactions)


def dimer_rathinam(x0=(400, 798, 0)) -> Network:
    """A stand-in for the stiff decaying-dimerizing model of the paper's
    accuracy comparison (whose SBML file is not available): the reactions of
    ``dimer()`` with c = (1, 10, 1000, 0.1) and X0 = (400, 798, 0), the
    constants as the Rathinam et al. (2003) example is commonly stated --
    recalled, not read from that paper or from this one.  The dimerization
    pair is near partial equilibrium from the start."""
    base = dimer(x0)
    return _net("dimer_rathinam", base.m, base.p, [1.0, 10.0, 1000.0, 0.1], x0, base.species,
                base.reactions)


def isomerisation(kf=1.0, kb=1.0, n_total=1000) -> Network:
    """A -> B (kf), B -> A (kb), all N_total molecules start as A."""
    return _net("isomerisation", [[1, 0], [0, 1]], [[0, 1], [1, 0]], [kf, kb], [n_total, 0],
                ("A", "B"), ("A->B", "B->A"))


def schlogl(theta=(0.03, 1e-4, 200.0, 3.5), x0=250) -> Network:
    """Schloegl model: 2X->3X, 3X->2X, 0->X, X->0 (bistable at these constants)."""
    return _net("schlogl", [[2], [3], [0], [1]], [[3], [2], [1], [0]], theta, [x0], ("X",),
                ("2X->3X", "3X->2X", "0->X", "X->0"))


def telegraph() -> Network:
    """Telegraph gene expression: species (G_off, G_on, mRNA, protein)."""
    m = [[1, 0, 0, 0], [0, 1, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 1, 0], [0, 0, 0, 1]]
    p = [[0, 1, 0, 0], [1, 0, 0, 0], [0, 1, 1, 0], [0, 0, 0, 0], [0, 0, 1, 1], [0, 0, 0, 0]]
    return _net("telegraph", m, p, [0.05, 0.15, 20.0, 1.0, 2.0, 0.1], [1, 0, 0, 0],
                ("G_off", "G_on", "mRNA", "protein"),
                ("on", "off", "transcribe", "mRNA decay", "translate", "protein decay"))


def random_network(seed=4, N=48, M=128, n_pairs=32, frac_uni=0.4, omega=100.0, n_fast=4,
                   fast=(30.0, 1e2), slow=(1e-3, 1e-2)) -> Network:
    """Seeded random stiff mass-action network (large-network workload).

    N species, M reactions, 40 % unimolecular and 60 % bimolecular (2A
    allowed); products are 1-2 species with coefficients 1-2.  Species get
    masses w in {1, 2, 3}; every reaction satisfies w.p <= w.m, so the total
    mass never grows, and ``n_pairs`` reversible pairs conserve it exactly.
    x0 is uniform on {50..500}.

    Rate constants (all within [1e-3, 1e2], bimolecular ones divided by the
    system size ``omega``): the ``n_fast`` reversible pairs with the largest
    flux at x0 (the smaller of the two directions' g) are fast, log-uniform
    on ``fast``; every other reaction is slow, log-uniform on ``slow``.  After
    a short relaxation the fast pairs sit in partial equilibrium and the
    slow reactions bound the leap, so the ensemble runs implicit leaps with
    a 48 x 48 Newton system.
    """
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 4, size=N)
    m = np.zeros((M, N), np.int32)
    p = np.zeros((M, N), np.int32)

    def draw_reactants(bi):
        r = np.zeros(N, np.int32)
        if not bi:
            r[rng.integers(N)] = 1
        else:
            r[rng.integers(N)] += 1
            r[rng.integers(N)] += 1
        return r

    def draw_products(mass, exact):
        for _ in range(5000):
            q = np.zeros(N, np.int32)
            for _s in range(rng.integers(1, 3)):
                q[rng.integers(N)] += rng.integers(1, 3)
            pm = int(w @ q)
            if (exact and pm == mass) or (not exact and pm <= mass):
                return q
        return None

    n_uni = int(round(frac_uni * M))
    kinds = np.array([0] * n_uni + [1] * (M - n_uni))
    rng.shuffle(kinds)
    rows = []
    pairs = []
    # reversible pairs: the reverse reaction consumes exactly the products
    while len(pairs) < n_pairs:
        r = draw_reactants(bool(kinds[len(rows)]))
        q = draw_products(int(w @ r), exact=True)
        if q is None or np.array_equal(q, r) or q.sum() > 2:
            continue
        pairs.append((len(rows), len(rows) + 1))
        rows += [(r, q), (q, r)]
    while len(rows) < M:
        r = draw_reactants(bool(kinds[len(rows)]))
        q = draw_products(int(w @ r), exact=False)
        if q is None or np.array_equal(q, r):
            continue
        rows.append((r, q))
    for j, (r, q) in enumerate(rows):
        m[j], p[j] = r, q
    x0 = rng.integers(50, 501, size=N)
    order = m.sum(axis=1)

    def g0(j):
        out = 1.0
        for i in np.nonzero(m[j])[0]:
            out *= math.comb(int(x0[i]), int(m[j, i]))
        return out / (omega if order[j] >= 2 else 1.0)

    flux = np.array([min(g0(a), g0(b)) for a, b in pairs])
    fast_pairs = set(np.argsort(-flux, kind="stable")[:n_fast].tolist())
    theta = 10.0 ** rng.uniform(np.log10(slow[0]), np.log10(slow[1]), size=M)
    for q, (a, b) in enumerate(pairs):
        if q in fast_pairs:
            theta[[a, b]] = 10.0 ** rng.uniform(np.log10(fast[0]), np.log10(fast[1]), size=2)
    theta = np.where(order >= 2, theta / omega, theta)
    return _net(f"random{N}x{M}", m, p, theta, x0)


def pure_death(N=1, x0=10) -> Network:
    """N independent decays X_i -> 0 at rate 1, every X_i starting at x0."""
    m = np.eye(N, dtype=np.int32)
    return _net(f"death{N}", m, np.zeros_like(m), np.ones(N), np.full(N, x0))


def critical_decay(n_fast=1, n_slow=2) -> Network:
    """``n_fast`` species in a fast birth-death balance around 1000 (0 -> Y,
    1000; Y -> 0, 1) and ``n_slow`` species of 5-8 molecules decaying slowly
    (rates 0.3, 0.05, 0.3, 0.05, ...): the small species are always near
    exhaustion, so their decays are critical reactions, while the fast pairs
    keep the leaps long."""
    N = n_fast + n_slow
    m = np.zeros((2 * n_fast + n_slow, N), np.int32)
    p = np.zeros_like(m)
    theta, x0 = [], []
    for k in range(n_fast):
        p[2 * k, k] = 1
        m[2 * k + 1, k] = 1
        theta += [1000.0, 1.0]
        x0.append(1000)
    for k in range(n_slow):
        m[2 * n_fast + k, n_fast + k] = 1
        theta.append(0.3 if k % 2 == 0 else 0.05)
        x0.append(5 if k % 2 == 0 else 8)
    return _net(f"critical_decay{n_fast}_{n_slow}", m, p, theta, x0)


def mass_action_jacobian_terms(net: Network):
    """The derivatives d g_j / d y_k of a mass-action network as polynomial
    terms -- what a caller supplies as a symbolic Jacobian: for every
    reaction j and reactant species k of it, the expansion of
    C'(y_k, m_kj) prod_{i != k} C(y_i, m_ij), with C(y, 1) = y,
    C(y, 2) = y^2/2 - y/2, C(y, 3) = y^3/6 - y^2/2 + y/3 and their derivatives.
    Returns (rxn [T], wrt [T], coef [T], powers [T][N]) in the order
    (j ascending, k ascending, terms by descending power of y_k, then of the
    other species in ascending order)."""
    poly = {1: {1: 1.0}, 2: {2: 0.5, 1: -0.5}, 3: {3: 1.0 / 6.0, 2: -0.5, 1: 1.0 / 3.0}}
    dpoly = {1: {0: 1.0}, 2: {1: 1.0, 0: -0.5}, 3: {2: 0.5, 1: -1.0, 0: 1.0 / 3.0}}
    rxn, wrt, coef, pows = [], [], [], []
    N = net.N
    for j in range(net.M):
        species = [i for i in range(N) if net.m[j, i] > 0]
        for k in species:
            terms = [(1.0, np.zeros(N, np.int32))]
            for i in species:
                factor = dpoly[int(net.m[j, i])] if i == k else poly[int(net.m[j, i])]
                out = []
                for c, pw in terms:
                    for e in sorted(factor, reverse=True):
                        q = pw.copy()
                        q[i] += e
                        out.append((c * factor[e], q))
                terms = out
            for c, pw in terms:
                rxn.append(j)
                wrt.append(k)
                coef.append(c)
                pows.append(pw)
    return (np.array(rxn, np.int32), np.array(wrt, np.int32), np.array(coef, np.float64),
            np.array(pows, np.int32).reshape(len(pows), N))


# --------------------------------------------------------------------------
# Ensembles: per-particle parameters and initial states.
# --------------------------------------------------------------------------

def stiff_padded(n_pad=45, k_birth=10.0, k_death=0.1, x_pad=100) -> Network:
    """The stiff decaying-dimerizing set plus ``n_pad`` independent birth-death
    species (0 -> X_k, X_k -> 0): 3 + n_pad species, 4 + 2 n_pad reactions.

    The slow birth-death channels bound the implicit step, the fast pair does
    not, so implicit leaps occur; with n_pad = 45 the Newton system is 48 x 48.
    """
    base = dimer_stiff()
    N, M = 3 + n_pad, 4 + 2 * n_pad
    m = np.zeros((M, N), np.int32)
    p = np.zeros((M, N), np.int32)
    m[:4, :3] = base.m
    p[:4, :3] = base.p
    for k in range(n_pad):
        p[4 + 2 * k, 3 + k] = 1      # 0 -> X_k
        m[5 + 2 * k, 3 + k] = 1      # X_k -> 0
    theta = np.concatenate([base.theta, np.tile([k_birth, k_death], n_pad)])
    x0 = np.concatenate([base.x0, np.full(n_pad, x_pad)])
    return _net(f"stiff_padded{n_pad}", m, p, theta, x0)


def tile(net: Network, P: int):
    """Every particle gets the nominal theta and x0: theta [P][M], x0 [P][N]."""
    theta = np.ascontiguousarray(np.broadcast_to(net.theta, (P, net.M)), dtype=np.float64)
    x0 = np.ascontiguousarray(np.broadcast_to(net.x0, (P, net.N)), dtype=np.int32)
    return theta, x0


def gamma_prior_theta(net: Network, P: int, seed: int, shape: float = 2.0):
    """theta_pj ~ Gamma(shape, rate = shape / theta_nom_j): mean theta_nom."""
    rng = np.random.default_rng(seed)
    scale = net.theta / shape
    return rng.gamma(shape, scale, size=(P, net.M)).astype(np.float64)


@dataclass
class Workload:
    name: str
    nets: list
    P: int
    t_end: float
    mode: str
    eps: float = 0.03
    theta: list = field(default_factory=list)   # per network: [P_k][M_k]
    x0: list = field(default_factory=list)      # per network: [P_k][N_k]
    pid: list = field(default_factory=list)     # per network: global particle ids [P_k]


def birth_death_workload(P=1024) -> Workload:
    net = birth_death()
    th, x0 = tile(net, P)
    return Workload("birth-death k1=10 k2=0.1 X0=0 t_end=100", [net], P, 100.0, "explicit",
                    theta=[th], x0=[x0], pid=[np.arange(P, dtype=np.int64)])


def dimer_workload(P=16384) -> Workload:
    net = dimer()
    th, x0 = tile(net, P)
    return Workload("decaying-dimerizing X0=(10000,0,0) t_end=30", [net], P, 30.0, "adaptive",
                    theta=[th], x0=[x0], pid=[np.arange(P, dtype=np.int64)])


def rathinam_workload(P=16384) -> Workload:
    """The stiff decaying-dimerizing set of Rathinam et al. (2003), the
    implicit-leap-heavy workload (timing the Jacobian variants)."""
    net = dimer_rathinam()
    th, x0 = tile(net, P)
    return Workload("stiff decaying-dimerizing (Rathinam 2003) X0=(400,798,0) t_end=4", [net], P,
                    4.0, "adaptive", theta=[th], x0=[x0], pid=[np.arange(P, dtype=np.int64)])


def mixed_set_workload(P=1 << 20, seed=3) -> Workload:
    """Isomerisation / birth-death / Schloegl interleaved 1:1:1 (particle p uses
    network p mod 3), theta from Gamma(2, 2/theta_nom) priors."""
    nets = [isomerisation(), birth_death(), schlogl()]
    th, x0, pid = [], [], []
    for k, net in enumerate(nets):
        ids = np.arange(k, P, 3, dtype=np.int64)
        th.append(gamma_prior_theta(net, len(ids), seed + 100 * k))
        x0.append(np.ascontiguousarray(np.broadcast_to(net.x0, (len(ids), net.N)), np.int32))
        pid.append(ids)
    return Workload("iso/birth-death/Schloegl 1:1:1, Gamma(2,2/theta) priors, t_end=50", nets,
                    P, 50.0, "adaptive", theta=th, x0=x0, pid=pid)


def random_network_workload(P=65536, seed=4, omega=100.0) -> Workload:
    net = random_network(seed=seed, omega=omega)
    th, x0 = tile(net, P)
    return Workload(f"random mass-action N=48 M=128 (omega={omega:g}) t_end=10", [net], P, 10.0,
                    "adaptive", theta=[th], x0=[x0], pid=[np.arange(P, dtype=np.int64)])


def stiff_padded_workload(P=16384, n_pad=45) -> Workload:
    """The stiff padded network (48 species, 94 reactions): about 270
    implicit leaps with 48 x 48 Newton systems per trajectory to t_end 4."""
    net = stiff_padded(n_pad)
    th, x0 = tile(net, P)
    return Workload(f"stiff dimer + {n_pad} birth-death species (N={net.N} M={net.M}) t_end=4",
                    [net], P, 4.0, "adaptive", theta=[th], x0=[x0],
                    pid=[np.arange(P, dtype=np.int64)])


def telegraph_workload(P=1 << 18, seed=5) -> Workload:
    net = telegraph()
    th = gamma_prior_theta(net, P, seed)
    x0 = np.ascontiguousarray(np.broadcast_to(net.x0, (P, net.N)), np.int32)
    return Workload("telegraph gene expression, 50 intervals of 5", [net], P, 5.0, "adaptive",
                    theta=[th], x0=[x0], pid=[np.arange(P, dtype=np.int64)])
