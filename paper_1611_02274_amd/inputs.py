"""Seeded synthetic inputs for batched ODE integration.

This module only draws random numbers and lays them out; it holds none of the
integration arithmetic (no right-hand side, no step, no controller).  Both the
CPU oracle tests and the GPU path take their inputs from here, so it imports
nothing else from this package.

Layout: every per-system array is struct-of-arrays, shape ``[rows, n]``, C
order, so entry ``[j, i]`` (flat ``j*n + i``) is unknown ``j`` of system ``i``:
the column-major storage of the paper's N_ode x N state matrix that puts the
same unknown of consecutive systems side by side (Sec. 3, state layout).

Workloads
---------
* van der Pol oscillators (nonstiff, RKCK): y1' = y2, y2' = mu (1 - y1^2) y2 - y1,
  one parameter ``g = (mu,)`` per system.
* synthetic mass-action networks (moderately stiff, RKC), isothermal and at
  constant volume, standing in for the paper's chemical-kinetics workload
  (Sec. 4.2, species equations and Arrhenius rate coefficients).  Two
  parameters per system: ``g = (T, rho)``.

Network convention (the paper leaves units and reverse rates open):
  3 elements with molar masses (1, 12, 16) g/mol; species are built by summing
  compositions of existing species so that many element-balanced reactions
  exist; every reaction is reversible with 1-2 species per side, element
  balanced; k_f = A T^b exp(-E/T) [cm^3 mol^-1 s^-1], k_r = k_f / K;
  a one-species side is multiplied by the total concentration [M] so every
  rate law is bimolecular.  rho = P W_mix / (R_u T) at P = 1 atm.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

ELEMENT_MASS = (1.0, 12.0, 16.0)          # g/mol
P_ATM = 1.01325e6                         # dyn/cm^2
R_UNIVERSAL = 8.314462618e7               # erg/(mol K)

NETWORK_SEEDS = {9: 109, 13: 113, 32: 132, 53: 153}
NETWORK_SIZES = {9: 19, 13: 27, 32: 133, 53: 325}


@dataclasses.dataclass(frozen=True)
class Network:
    """A reversible mass-action network.

    reac, prod: int32 [n_rx, 2], species indices of the two slots of each side,
    -1 for an empty slot (one-species side).  A repeated index (A + A) is allowed.
    lnA: natural log of the pre-exponential factor; beta: temperature exponent;
    Ea: activation temperature E/R in K; Keq: equilibrium constant (k_f / k_r).
    W: molar masses [n_sp] in g/mol; comp: element counts [n_sp, 3].
    """
    n_sp: int
    n_rx: int
    comp: np.ndarray
    W: np.ndarray
    reac: np.ndarray
    prod: np.ndarray
    lnA: np.ndarray
    beta: np.ndarray
    Ea: np.ndarray
    Keq: np.ndarray
    seed: int = -1
    # synthetic thermodynamics (networks with the energy equation only): per
    # unit mass, e_k(T) = u0_k + (cv0_k + cv1_k T) T, c_v,k(T) = cv0_k + 2 cv1_k T
    u0: np.ndarray | None = None
    cv0: np.ndarray | None = None
    cv1: np.ndarray | None = None

    def stoich(self) -> np.ndarray:
        """nu[k, j] = (count of k among products) - (count among reactants)."""
        nu = np.zeros((self.n_sp, self.n_rx), dtype=np.int64)
        for j in range(self.n_rx):
            for s in self.reac[j]:
                if s >= 0:
                    nu[s, j] -= 1
            for s in self.prod[j]:
                if s >= 0:
                    nu[s, j] += 1
        return nu

    def topology_key(self) -> str:
        """Hash of what a compiled right-hand side depends on (species count and
        the reaction slots); rate parameters and masses are runtime data."""
        h = hashlib.sha1()
        h.update(np.int64(self.n_sp).tobytes())
        h.update(np.ascontiguousarray(self.reac, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.prod, dtype=np.int32).tobytes())
        return h.hexdigest()[:16]


def _draw_species(n_sp: int, rng: np.random.Generator) -> np.ndarray:
    comp = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    if n_sp < 3:
        return np.array(comp[:n_sp], dtype=np.int64)
    guard = 0
    while len(comp) < n_sp:
        a = comp[rng.integers(len(comp))]
        b = comp[rng.integers(len(comp))]
        c = tuple(x + y for x, y in zip(a, b))
        if max(c) <= 3 and c not in comp:
            comp.append(c)
        guard += 1
        if guard > 100000:
            raise RuntimeError("species draw did not terminate")
    return np.array(comp, dtype=np.int64)


def _balanced_candidates(comp: np.ndarray):
    n_sp = len(comp)
    sides = [(a,) for a in range(n_sp)] + [(a, b) for a in range(n_sp) for b in range(a, n_sp)]
    tot = {s: tuple(int(x) for x in comp[list(s)].sum(0)) for s in sides}
    out = []
    for i, R in enumerate(sides):
        for P in sides[i + 1:]:
            if set(R) & set(P):
                continue
            if tot[R] == tot[P]:
                out.append((R, P))
    return out


def make_network(n_sp: int, n_rx: int, seed: int) -> Network:
    """Seeded element-conserving reversible network with every species taking part."""
    rng = np.random.default_rng(seed)
    for _ in range(1000):
        comp = _draw_species(n_sp, rng)
        cands = _balanced_candidates(comp)
        if len(cands) < n_rx:
            continue
        for _ in range(100):
            pick = rng.choice(len(cands), size=n_rx, replace=False)
            used = set()
            for p in pick:
                R, P = cands[p]
                used.update(R)
                used.update(P)
            if len(used) == n_sp:
                break
        else:
            continue
        break
    else:
        raise RuntimeError(f"no network with {n_sp} species / {n_rx} reactions for seed {seed}")
    flip = rng.integers(0, 2, size=n_rx)
    reac = -np.ones((n_rx, 2), dtype=np.int32)
    prod = -np.ones((n_rx, 2), dtype=np.int32)
    for j, p in enumerate(pick):
        R, P = cands[p]
        if flip[j]:
            R, P = P, R
        reac[j, :len(R)] = R
        prod[j, :len(P)] = P
    log10A = rng.uniform(8.0, 14.0, n_rx)
    beta = rng.uniform(-1.0, 1.0, n_rx)
    Ea = rng.uniform(0.0, 2.0e4, n_rx)
    log10K = rng.uniform(-2.0, 2.0, n_rx)
    W = comp @ np.array(ELEMENT_MASS)
    return Network(n_sp=n_sp, n_rx=n_rx, comp=comp, W=W.astype(np.float64),
                   reac=reac, prod=prod, lnA=log10A * np.log(10.0), beta=beta,
                   Ea=Ea, Keq=10.0 ** log10K, seed=seed)


def standard_network(n_sp: int) -> Network:
    """The four fixed networks (9/19, 13/27, 32/133, 53/325)."""
    return make_network(n_sp, NETWORK_SIZES[n_sp], NETWORK_SEEDS[n_sp])


THERMO_SEED_OFFSET = 7000


def thermal_network(n_sp: int) -> Network:
    """A standard network with seeded synthetic thermodynamics for the energy
    equation (per unit mass, erg/g): cv0 = (R_u / W) U[1.5, 3.5], cv1 = cv0
    U[0, 1e-4] / K, u0 = (R_u / W) U[-2000, 2000] K."""
    net = standard_network(n_sp)
    rng = np.random.default_rng(THERMO_SEED_OFFSET + n_sp)
    rw = R_UNIVERSAL / net.W
    cv0 = rw * rng.uniform(1.5, 3.5, n_sp)
    cv1 = cv0 * rng.uniform(0.0, 1e-4, n_sp)
    u0 = rw * rng.uniform(-2000.0, 2000.0, n_sp)
    return dataclasses.replace(net, u0=u0, cv0=cv0, cv1=cv1)


def thermal_inputs(net: Network, n: int, seed: int, T_range=(1000.0, 2500.0)):
    """(y0 [N + 1, n] = (T0, Y0), g [1, n] = (rho)) with T0 ~ U[T_range],
    Y0 ~ Dirichlet(1), rho from (T0, Y0) at 1 atm (held constant: constant volume)."""
    Y, g2 = kinetics_inputs(net, n, seed, T_range)
    y0 = np.ascontiguousarray(np.concatenate([g2[:1], Y]))
    return y0, np.ascontiguousarray(g2[1:2])


def density(net: Network, T: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Ideal-gas density at 1 atm for mass fractions Y [n_sp, n]: an input
    parameter per system, held constant during integration."""
    wmix = 1.0 / (Y / net.W[:, None]).sum(axis=0)
    return P_ATM * wmix / (R_UNIVERSAL * T)


def kinetics_inputs(net: Network, n: int, seed: int, T_range=(1000.0, 2500.0), rng=None):
    """(y0 [n_sp, n], g [2, n]) with T ~ U[T_range], Y0 ~ Dirichlet(1), rho from (T, Y0)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    T = rng.uniform(T_range[0], T_range[1], n)
    Y = np.ascontiguousarray(rng.dirichlet(np.ones(net.n_sp), n).T)
    g = np.ascontiguousarray(np.stack([T, density(net, T, Y)]))
    return Y, g


def vdp_inputs(n: int, seed: int, mu_range=(0.5, 2.0)):
    """(y0 [2, n], g [1, n]): mu ~ U[mu_range] (default [0.5, 2]; [300, 3000] is
    stiff: RKC steps of 10 to 60 stages), y0 ~ U[-2, 2]^2."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(mu_range[0], mu_range[1], n)
    y0 = rng.uniform(-2.0, 2.0, (2, n))
    return np.ascontiguousarray(y0), np.ascontiguousarray(mu[None, :])


# Seed of the synthetic seven-body base configuration of the Pleiades workload
# (the problem's own initial conditions are not part of the paper).
PLEIADES_BASE_SEED = 716


def pleiades_base(seed: int = PLEIADES_BASE_SEED) -> np.ndarray:
    """A seeded seven-body configuration [28]: bodies near a ring (angle
    2 pi i / 7 + U[-0.3, 0.3], radius U[1.5, 4]) moving tangentially with
    speed U[0.5, 1.5] * sqrt(28 / r) / 2; layout (x_1..7, y_1..7, x'_1..7, y'_1..7)."""
    rng = np.random.default_rng(seed)
    ang = 2.0 * np.pi * np.arange(7) / 7.0 + rng.uniform(-0.3, 0.3, 7)
    rad = rng.uniform(1.5, 4.0, 7)
    v = rng.uniform(0.5, 1.5, 7) * np.sqrt(28.0 / rad) * 0.5
    return np.concatenate([rad * np.cos(ang), rad * np.sin(ang), -v * np.sin(ang), v * np.cos(ang)])


def pleiades_inputs(n: int, seed: int, rel: float = 1e-2):
    """(y0 [28, n], None): the base configuration with every component of every
    system multiplied by 1 + rel * U[-1, 1] (the paper's randomly perturbed
    initial conditions, Sec. 4.1)."""
    rng = np.random.default_rng(seed)
    f = 1.0 + rel * rng.uniform(-1.0, 1.0, (28, n))
    return np.ascontiguousarray(pleiades_base()[:, None] * f), None


# ---------------------------------------------------------------- workloads
@dataclasses.dataclass
class Workload:
    name: str
    method: str            # "rkck" | "rkc"
    problem: str           # "vdp" | "pleiades" | "net9" | "net13" | "net32" | "net53"
    n: int
    t0: float
    t1: float
    rtol: float
    atol: float
    seed: int
    T_range: tuple = (1000.0, 2500.0)
    # keyword arguments of the integration call the benchmark times (schedule,
    # cost order); tests that check the benchmark's launch use the same
    launch: dict = dataclasses.field(default_factory=dict)
    # [t0, t1] integrated in this many equal global steps, each a restart
    global_steps: int = 1


WORKLOADS = {
    "vdp4096_rkck": Workload("vdp4096_rkck", "rkck", "vdp", 4096, 0.0, 10.0, 1e-8, 1e-10, 1,
                             launch=dict(schedule=1)),
    "net13_rkc": Workload("net13_rkc", "rkc", "net13", 1 << 18, 0.0, 1e-6, 1e-8, 1e-12, 2002,
                          (1000.0, 2500.0), launch=dict(schedule=1, cost_order=1)),
    "net53_rkc": Workload("net53_rkc", "rkc", "net53", 1 << 20, 0.0, 1e-6, 1e-8, 1e-12, 3003,
                          (900.0, 2800.0)),
    "net53_rkck": Workload("net53_rkck", "rkck", "net53", 1 << 20, 0.0, 1e-6, 1e-8, 1e-12, 3003,
                           (900.0, 2800.0)),
    # the 32-species network at the same size (group kernels, 16 lanes per system)
    "net32_rkc": Workload("net32_rkc", "rkc", "net32", 1 << 20, 0.0, 1e-6, 1e-8, 1e-12, 3203,
                          (900.0, 2800.0)),
    "net32_rkck": Workload("net32_rkck", "rkck", "net32", 1 << 20, 0.0, 1e-6, 1e-8, 1e-12, 3203,
                           (900.0, 2800.0)),
    # ten global steps of 0.1 over [0, 1], each a restart (Sec. 4.1); eps = 1e-10
    "pleiades_rkck": Workload("pleiades_rkck", "rkck", "pleiades", 1 << 18, 0.0, 1.0, 1e-10, 0.0,
                              6006, launch=dict(schedule=3), global_steps=10),
    # the energy equation: ten global steps of 1e-6 s, each a restart (Sec. 4.2)
    "net13_thermal_rkc": Workload("net13_thermal_rkc", "rkc", "net13_thermal", 1 << 18, 0.0,
                                  1e-5, 1e-8, 1e-12, 8008, (1000.0, 2500.0),
                                  launch=dict(schedule=1, cost_order=1), global_steps=10),
    # the largest compiled network with the energy equation (53 species + T, the
    # size of Sec. 4.2's mechanism), one global step of 1e-6 s on the group kernels
    "net53_thermal_rkc": Workload("net53_thermal_rkc", "rkc", "net53_thermal", 1 << 18, 0.0,
                                  1e-6, 1e-8, 1e-12, 8053, (1000.0, 2500.0),
                                  launch=dict(schedule=3)),
    "net13_adjoint": Workload("net13_adjoint", "rkc", "net13", 1 << 16, 0.0, 1e-6, 1e-8, 1e-12,
                              5005, (1000.0, 2500.0)),
    "net13_adjoint_rkck": Workload("net13_adjoint_rkck", "rkck", "net13", 1 << 16, 0.0, 1e-6,
                                   1e-8, 1e-12, 5005, (1000.0, 2500.0)),
}


def network_of(problem: str) -> Network:
    return standard_network(int(problem[3:]))


def workload_inputs(w: Workload, n: int | None = None):
    """Inputs of a workload; ``n`` smaller than ``w.n`` gives the first ``n``
    systems of a draw of size ``n`` with the same seed (a smaller case of the
    same distribution, not a prefix of the full draw)."""
    n = w.n if n is None else n
    if w.problem == "vdp":
        return vdp_inputs(n, w.seed)
    if w.problem == "pleiades":
        return pleiades_inputs(n, w.seed)
    if w.problem.endswith("_thermal"):
        return thermal_inputs(thermal_network(int(w.problem[3:-8])), n, w.seed, w.T_range)
    return kinetics_inputs(network_of(w.problem), n, w.seed, w.T_range)


def adjoint_weights(n_eq: int, n: int, seed: int) -> np.ndarray:
    """Loss weights w ~ N(0, 1) [n_eq, n], drawn after the workload's inputs."""
    rng = np.random.default_rng(seed + 1)
    return np.ascontiguousarray(rng.standard_normal((n_eq, n)))


def ragged_inputs(n_total: int = 1_000_000, seed: int = 4004, T_range=(800.0, 3000.0)):
    """Interleaved batch over the 9/13/32/53-species networks:
    slot_net[i] in {0..3} (a seeded permutation of equal shares) and, per
    network, (y0, g) for the systems assigned to it in slot order."""
    rng = np.random.default_rng(seed)
    sizes = (9, 13, 32, 53)
    share = np.repeat(np.arange(4, dtype=np.int32), n_total // 4)
    share = np.concatenate([share, np.arange(n_total - share.size, dtype=np.int32) % 4])
    slot_net = rng.permutation(share).astype(np.int32)
    per_net = []
    for k, n_sp in enumerate(sizes):
        cnt = int((slot_net == k).sum())
        per_net.append(kinetics_inputs(standard_network(n_sp), cnt, seed, T_range, rng=rng))
    return slot_net, per_net


def slot_map_codes(slot_net: np.ndarray) -> np.ndarray:
    """Slot map of the interleaved batch form: code (network << 28 | index of the
    system within its network's block), systems numbered in slot order."""
    slot_net = np.asarray(slot_net, dtype=np.int32)
    local = np.zeros(slot_net.size, dtype=np.int32)
    for k in np.unique(slot_net):
        sel = slot_net == k
        local[sel] = np.arange(int(sel.sum()), dtype=np.int32)
    return (slot_net.astype(np.int32) << 28) | local


def linear_problem_matrix(eigs, seed: int = 0) -> np.ndarray:
    """A dense matrix with the given real eigenvalues and a random orthogonal
    eigenbasis (symmetric, so the spectral radius is max |eig|)."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((len(eigs), len(eigs))))
    return np.ascontiguousarray(q @ np.diag(np.asarray(eigs, dtype=np.float64)) @ q.T)

