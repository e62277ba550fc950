"""Algorithmic FP64 work of an integration, from its per-system statistics.

Counting convention: every add, subtract and multiply of the method's own
arithmetic counts 1 (a fused multiply-add counts 2); division by a constant
counts as the multiply by its reciprocal; other divisions, square roots, exp,
log and pow are special operations and are not counted as flops.  These are
the operations the method must perform as written in the paper, not the
instructions a kernel happens to issue.

Per-unit counts (N unknowns, NR reactions, S = reactant+product slots in use):
  right-hand side  van der Pol: 5;  mass action: 5N - 1 + 5NR + S;
                   Pleiades: 378 (21 pairs: two differences, squared distance 3,
                   d2 sqrt(d2) 1; 42 ordered pairs x 2 coordinates: m_j dx, times
                   1/r, accumulate 3; x_j - x_i is the pair's difference negated --
                   the 21 square roots and reciprocals are special operations)
  rate setup       mass action: 5NR per system (plus 2NR exp/div specials)
  RKCK attempt     56N + 5 beyond its right-hand sides (stage arguments 30N,
                   k_i = h f 6N, fifth-order sum 8N, error sum 9N, scale 3N)
  RKC attempt      (s - 1)(9N + 42) + 11N + 10 beyond its right-hand sides
                   (stage recursion 9N, coefficients 42 per stage, w_1 2N,
                   error estimate and weights 9N, controller 10)
  power method     6N per call + 6N per iteration beyond its right-hand sides
  RKC first step   7N
  adjoint VJP      van der Pol: 15;  mass action: 21NR + 8N (J^T u and the
                   ln A contributions)
  adjoint step     s VJPs + (s - 1)(10N + 4) + 4N + 1 per accepted step of s
                   stages (the transposed recursion), beyond the forward
                   integration; recomputation from checkpoints is not counted
"""
from __future__ import annotations

import numpy as np

ST_ACCEPT, ST_REJECT, ST_RHS, ST_SR_CALLS, ST_POW_ITERS, ST_MAX_STAGES = range(6)


PLEIADES = "pleiades"      # stands for the Pleiades problem where a network is expected


class Thermal:
    """A network with the energy equation: the isothermal right-hand side plus,
    per evaluation, the rate coefficients' arguments lnA + b lnT - E (1/T)
    (3 NR flops; NR exp and one log are special) and the energy sum
    (e_k: 4, sum: 2, c_v,k and its sum: 4 per species; 1 more for the scale)."""

    def __init__(self, net):
        self.net = net


def rhs_flops(net=None) -> int:
    if net is None:
        return 5
    if isinstance(net, Thermal):
        return rhs_flops(net.net) + 3 * net.net.n_rx + 10 * net.net.n_sp + 1
    if isinstance(net, str) and net == PLEIADES:
        return 21 * 6 + 42 * 2 * 3

    slots = int((np.asarray(net.reac) >= 0).sum() + (np.asarray(net.prod) >= 0).sum())
    return 5 * net.n_sp - 1 + 5 * net.n_rx + slots


def setup_flops(net=None) -> int:
    return 0 if net is None or isinstance(net, (str, Thermal)) else 5 * net.n_rx


def per_system(method: str, stats: np.ndarray, n_eq: int, net=None) -> np.ndarray:
    """Algorithmic flops of each system from stats [6, n] (int)."""
    st = np.asarray(stats, dtype=np.float64)
    acc, rej, rhs, sr, pw = st[ST_ACCEPT], st[ST_REJECT], st[ST_RHS], st[ST_SR_CALLS], st[ST_POW_ITERS]
    att = acc + rej
    F = rhs_flops(net)
    N = n_eq
    total = rhs * F + setup_flops(net)
    if method == "rkck":
        total = total + att * (56 * N + 5)
    else:
        started = rhs > 0
        stage_sum = np.where(started, rhs - 2 - pw - att, 0.0)    # sum over attempts of (s - 1)
        total = (total + stage_sum * (9 * N + 42) + att * (11 * N + 10) + pw * 6 * N +
                 sr * 6 * N + np.where(started, 7 * N, 0))
    return total


def total(method: str, stats, n_eq: int, net=None) -> float:
    return float(per_system(method, stats, n_eq, net).sum())


def vjp_flops(net=None) -> int:
    return 15 if net is None else 21 * net.n_rx + 8 * net.n_sp


def adjoint_reverse(n_eq: int, net, n_steps, stage_sum) -> float:
    """Flops of the reverse sweep: n_steps accepted steps whose stage counts sum
    to stage_sum (totals over all systems)."""
    V = vjp_flops(net)
    N = n_eq
    return float(stage_sum * V + (stage_sum - n_steps) * (10 * N + 4) + n_steps * (4 * N + 1))


def adjoint_reverse_rkck(n_eq: int, net, n_steps) -> float:
    """Flops of the RKCK reverse sweep over n_steps accepted steps (total over
    all systems): per step six VJPs, kbar_i = c_i lambda (6N), u = h kbar_i
    (6N), ybar += zbar (6N) and kbar_j += b_ij zbar over the 15 couplings (30N
    fused pairs counted as 2 flops each: 30N)."""
    return float(n_steps * (6 * vjp_flops(net) + 48 * n_eq))
