"""Result checks that need no PBM: compliance, KKT residual, duality
certificate (Section 1 problem (1.1); Section 2, Theorem 2 eq. (2.5) and the
gap (2.6)).

Compliance of a density rho is c(rho) = 1/2 f^T K(rho)^{-1} f (problem (1.1)
with u eliminated).  For every feasible rho_hat and every (u, alpha),
weak duality (Theorem 2) gives
      q(u, alpha) <= c* <= c(rho_hat),
where q is the objective of the unconstrained dual (2.5).  q is concave and
piecewise linear in alpha with breakpoints e_i = 1/2 u^T K_i u, so its
maximum over alpha is attained at one of the e_i.

KKT residual (the paper defines none for PBM; the reading used here):
  r_eq   = ||K(rho) u - f|| / ||f||
  r_vol  = |sum rho - V| / V
  r_box  = max(0, max(rho_lo - rho), max(rho - rho_hi)) / max(rho_hi)
  r_stat = max_i |rho_i - Proj_[lo_i, hi_i](rho_i + (e_i - lam)/lam)| / hi_i
with e_i from u and lam the volume multiplier (= alpha of the dual).
r_stat vanishes iff e_i = lam where lo < rho < hi, e_i <= lam at the lower
and e_i >= lam at the upper bound (stationarity of the Lagrangian (2.3)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fe


def solve_state(grid: fe.Grid, Ke, rho, f, tol=1e-13):
    """u = K(rho)^{-1} f on the free DOFs (sparse direct)."""
    K = fe.assemble_K_free(grid, Ke, rho).tocsc()
    u = np.zeros(grid.n_dof)
    u[grid.free] = spla.spsolve(K, f[grid.free])
    return u


def compliance(grid: fe.Grid, Ke, rho, f) -> float:
    u = solve_state(grid, Ke, rho, f)
    return 0.5 * float(f @ u)


def dual_lower_bound(grid: fe.Grid, Ke, f, V, rho_lo, rho_hi, u):
    """max over alpha of q(u, alpha), eq. (2.5); returns (value, alpha)."""
    e = fe.element_energies(grid, Ke, u)
    fu = float(f @ u)
    best, best_a = -np.inf, None
    # evaluate at every breakpoint; vectorised over the sorted e
    order = np.argsort(e)
    es = e[order]
    lo, hi = rho_lo[order], rho_hi[order]
    # for alpha = es[k]: elements with e < alpha use lo*(alpha-e), e >= alpha hi*(alpha-e)
    c_lo = np.concatenate([[0.0], np.cumsum(lo)])
    c_loe = np.concatenate([[0.0], np.cumsum(lo * es)])
    c_hi = np.concatenate([np.cumsum((hi)[::-1])[::-1], [0.0]])
    c_hie = np.concatenate([np.cumsum((hi * es)[::-1])[::-1], [0.0]])
    k = np.arange(es.size)
    a = es
    val = (-a * V + fu + a * c_lo[k] - c_loe[k] + a * c_hi[k] - c_hie[k])
    j = int(np.argmax(val))
    best, best_a = float(val[j]), float(a[j])
    return best, best_a


def project_feasible(rho, V, rho_lo, rho_hi, iters=200):
    """Closest-in-shift feasible density: clip(rho + theta, lo, hi) with
    sum = V, theta by bisection."""
    a, b = -1.0 - np.max(rho), 1.0 + np.max(rho_hi)
    for _ in range(iters):
        t = 0.5 * (a + b)
        if np.clip(rho + t, rho_lo, rho_hi).sum() > V:
            b = t
        else:
            a = t
    return np.clip(rho + 0.5 * (a + b), rho_lo, rho_hi)


def certificate(grid: fe.Grid, Ke, f, V, rho_lo, rho_hi, rho, u):
    """(lower, upper, (upper-lower)/upper) bracketing the optimal compliance."""
    lb, _ = dual_lower_bound(grid, Ke, f, V, rho_lo, rho_hi, u)
    rh = project_feasible(rho, V, rho_lo, rho_hi)
    ub = compliance(grid, Ke, rh, f)
    return lb, ub, (ub - lb) / ub


def kkt_residual(grid: fe.Grid, Ke, f, V, rho_lo, rho_hi, rho, u, lam):
    """Dictionary of the four terms and their max (see module docstring)."""
    r = fe.apply_K(grid, Ke, rho, u) - f
    r_eq = float(np.linalg.norm(r) / np.linalg.norm(f))
    r_vol = float(abs(rho.sum() - V) / V)
    r_box = float(max(0.0, np.max(rho_lo - rho), np.max(rho - rho_hi)) / np.max(rho_hi))
    e = fe.element_energies(grid, Ke, u)
    proj = np.clip(rho + (e - lam) / lam, rho_lo, rho_hi)
    r_stat = float(np.max(np.abs(rho - proj) / rho_hi))
    return dict(r_eq=r_eq, r_vol=r_vol, r_box=r_box, r_stat=r_stat,
                kkt=max(r_eq, r_vol, r_box, r_stat))
