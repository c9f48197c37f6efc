"""Damped optimality-criteria (DOC) method for the VTS problem (Section 5,
Algorithm 4).  Test infrastructure, like the rest of oracle/: plain FP64,
the state equation solved by a sparse direct solve.

One iteration, from a feasible rho (sum rho = V, bounds):
  u = K(rho)^{-1} f;
  bisection on alpha in [0, 10000] while (hi - lo)/(hi + lo) > tau:
      rho+_i(alpha) = min(max(rho_i (u^T K_i u)^q / alpha, lo_i), hi_i),
      alpha becomes the lower end if sum rho+ > V, else the upper end;
  stop if ||rho+ - rho||_inf <= eps, else rho = rho+.
tau = 0.1 eps and q = 0.5 as in the text after Algorithm 4.  rho+ of the
last bisection midpoint is the new iterate.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import fe, kkt


@dataclass
class DocResult:
    rho: np.ndarray
    u: np.ndarray
    alpha: float
    iterations: int
    converged: bool
    history: List[dict] = field(default_factory=list)


def oc_update(rho, uKu, lo, hi, V, q=0.5, tau=1e-4, alpha_hi=1e4):
    """One bisection of Algorithm 4: (rho+, alpha, bisection steps)."""
    a_lo, a_hi = 0.0, alpha_hi
    steps = 0
    rho_new, alpha = rho, 0.5 * (a_lo + a_hi)
    g = uKu ** q
    while (a_hi - a_lo) / (a_hi + a_lo) > tau:
        alpha = 0.5 * (a_hi + a_lo)
        rho_new = np.minimum(np.maximum(rho * g / alpha, lo), hi)
        if rho_new.sum() > V:
            a_lo = alpha
        else:
            a_hi = alpha
        steps += 1
    return rho_new, alpha, steps


def doc_solve(problem, eps=1e-3, q=0.5, max_iter=1000, alpha_hi=1e4, rho0=None,
              iterations=None) -> DocResult:
    """Algorithm 4 from rho0 (default V/m); with `iterations` set, exactly
    that many iterations are taken (no stopping test)."""
    from .pbm import VTS
    P = VTS(problem)
    g = P.grid
    rho = np.full(g.m, P.V / g.m) if rho0 is None else np.array(rho0, dtype=np.float64)
    tau = 0.1 * eps
    hist = []
    u = np.zeros(g.n_dof)
    alpha = 0.0
    n = iterations if iterations is not None else max_iter
    converged = False
    for k in range(n):
        u = kkt.solve_state(g, P.Ke, rho, P.f)
        uKu = 2.0 * fe.element_energies(g, P.Ke, u)
        rho_new, alpha, steps = oc_update(rho, uKu, P.rho_lo, P.rho_hi, P.V, q, tau, alpha_hi)
        change = float(np.max(np.abs(rho_new - rho)))
        hist.append(dict(change=change, alpha=alpha, bisection=steps,
                         compliance=0.5 * float(P.f @ u)))
        if iterations is None and change <= eps:
            converged = True
            break
        rho = rho_new
    return DocResult(rho=rho, u=u, alpha=alpha, iterations=len(hist), converged=converged,
                     history=hist)
