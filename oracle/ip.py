"""Primal-dual interior point (IP) method for the VTS problem (Section 4,
Algorithm 3), written out step by step.  Test infrastructure, like the rest
of oracle/: plain FP64; the reduced system (eq. S_IP) is assembled and
solved by MINRES with one multigrid V-cycle, or by a supplied direct solve.

Variables (u, alpha, rho, nu_lo, nu_hi), barrier parameters (r, s).  The
Newton residual of Section 4.1 (all-DOF layout, fixed DOFs masked):
    res_1 = K(rho) u - f               res_2 = sum rho - V
    res_3 = e(u) + alpha + nu_lo - nu_hi,   e_i = 1/2 u^T K_i u
    res_4 = (rho - rho_lo) nu_lo - r   res_5 = (rho_hi - rho) nu_hi - s
and its Jacobian, eq. (gradres), in the unknowns (u, alpha, rho, nu_lo,
nu_hi).

Readings of the paper used here:
  * the nu_hi term of the residual belongs to res_5, as the perturbed
    complementarity conditions and the Jacobian state (it is printed in the
    res_4 row);
  * every increment is the Newton step J d = -res of that residual and
    Jacobian.  Eliminating (nu_lo, nu_hi) and then rho gives, with
    R_lo = diag(rho - rho_lo), R_hi = diag(rho_hi - rho),
    N_lo = diag(nu_lo), N_hi = diag(nu_hi), W = (R_lo^-1 N_lo + R_hi^-1 N_hi)^-1
    and X = res_3 - R_lo^-1 res_4 + R_hi^-1 res_5:
        S [du; dalpha] = -[res_1; res_2] - [B; e^T] W X          (eq. S_IP)
        drho = W (B^T du + dalpha e + X)
    The printed right-hand side and the printed Delta rho formula each carry
    a sign pattern of the res_3, res_4, res_5 terms that disagrees with the
    Jacobian and with each other; the Jacobian decides;
  * in the Delta nu_hi formula the term (N_lo - N_hi) rho is read as
    (N_lo - N_hi) Delta rho, which is what the sum of the res_4 and res_5
    rows of the Newton system gives;
  * the KKT conditions of Section 4.1 read e_i + alpha + nu_lo - nu_hi = 0,
    so alpha tends to minus the volume multiplier lambda (= the alpha of the
    dual (2.1) that PBM computes); the gap (2.6) is evaluated at (u, -alpha);
  * the step lengths of nu_lo and nu_hi are capped at 1 like that of
    (u, rho) (a full Newton step at most; the printed formulas state the
    cap for kappa_u only), and a step length over an empty set is 1;
  * MINRES stops, keeping its current iterate, when the V-cycle loses
    positive definiteness in floating point on these ill-conditioned
    systems (the paper does not say what its solver does then).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import fe


@dataclass
class IPOptions:
    """Parameters of Algorithm 3 and of its MINRES rule (Section 6.2), the
    paper's values.  max_minres is larger than for PBM: the reduced IP
    systems become ill-conditioned as the barrier parameters go to zero (the
    weights W of interior elements grow like 1/r) and the paper reports
    several hundred MINRES steps in the last IP iterations."""
    eps_ip: float = 1e-5
    sigma_r: float = 0.2
    sigma_s: float = 0.2
    r0: float = 1e-2
    s0: float = 1e-2
    step_frac: float = 0.9
    eps_mr0: float = 1e-2
    eps_mr_min: float = 1e-9
    max_iter: int = 300
    max_minres: int = 3000


@dataclass
class IPState:
    u: np.ndarray
    alpha: float
    rho: np.ndarray
    nu_lo: np.ndarray
    nu_hi: np.ndarray

    def copy(self):
        return IPState(self.u.copy(), float(self.alpha), self.rho.copy(),
                       self.nu_lo.copy(), self.nu_hi.copy())


def initial_state(n_dof: int, m: int, V: float) -> IPState:
    """Initial point stated before Algorithm 3: u = 0, alpha = 1,
    rho = V/m, nu_lo = nu_hi = e."""
    return IPState(np.zeros(n_dof), 1.0, np.full(m, V / m), np.ones(m), np.ones(m))


@dataclass
class Residual:
    res1: np.ndarray        # all-DOF, masked
    res2: float
    res3: np.ndarray
    res4: np.ndarray
    res5: np.ndarray
    e: np.ndarray
    be: np.ndarray          # m x 24, b_i = K_i u on element i's DOFs


def residual(P, st: IPState, r: float, s: float) -> Residual:
    """The Newton residual of Section 4.1 with the nu_hi term in res_5."""
    g = P.grid
    e = fe.element_energies(g, P.Ke, st.u)
    be = fe.element_forces(g, P.Ke, st.u)
    res1 = fe.apply_K(g, P.Ke, st.rho, st.u) - P.f
    res2 = float(st.rho.sum() - P.V)
    res3 = e + st.alpha + st.nu_lo - st.nu_hi
    res4 = (st.rho - P.rho_lo) * st.nu_lo - r
    res5 = (P.rho_hi - st.rho) * st.nu_hi - s
    return Residual(res1, res2, res3, res4, res5, e, be)


def residual_vector(P, st: IPState, r: float, s: float) -> np.ndarray:
    """(res_1 on free DOFs, res_2, res_3, res_4, res_5) as one vector."""
    R = residual(P, st, r, s)
    return np.concatenate([R.res1[P.free], [R.res2], R.res3, R.res4, R.res5])


def jacobian_dense(P, st: IPState) -> np.ndarray:
    """Eq. (gradres) on (free u, alpha, rho, nu_lo, nu_hi); tiny grids only."""
    g = P.grid
    n, m = P.n, g.m
    be = fe.element_forces(g, P.Ke, st.u)
    B = fe.element_force_matrix(g, be).toarray()
    K = fe.assemble_K_free(g, P.Ke, st.rho).toarray()
    I = np.eye(m)
    one = np.ones((m, 1))
    J = np.zeros((n + 1 + 3 * m,) * 2)
    a, r0, l0, h0 = n, n + 1, n + 1 + m, n + 1 + 2 * m
    J[:n, :n] = K
    J[:n, r0:l0] = B
    J[a, r0:l0] = 1.0
    J[r0:l0, :n] = B.T
    J[r0:l0, a:a + 1] = one
    J[r0:l0, l0:h0] = I
    J[r0:l0, h0:] = -I
    J[l0:h0, r0:l0] = np.diag(st.nu_lo)
    J[l0:h0, l0:h0] = np.diag(st.rho - P.rho_lo)
    J[h0:, r0:l0] = -np.diag(st.nu_hi)
    J[h0:, h0:] = np.diag(P.rho_hi - st.rho)
    return J


def weights(P, st: IPState, R: Residual):
    """W = (R_lo^-1 N_lo + R_hi^-1 N_hi)^-1 and X = res_3 - R_lo^-1 res_4 +
    R_hi^-1 res_5 (per element)."""
    dlo = st.rho - P.rho_lo
    dhi = P.rho_hi - st.rho
    W = 1.0 / (st.nu_lo / dlo + st.nu_hi / dhi)
    X = R.res3 - R.res4 / dlo + R.res5 / dhi
    return W, X


def reduced_system(P, st: IPState, R: Residual):
    """S of eq. (S_IP) on (free u, alpha) and the right-hand side of
    eq. (IP_system):  S = [[K(rho) + B W B^T, B W e], [e^T W B^T, e^T W e]],
    rhs = -[res_1; res_2] - [B; e^T] W X."""
    g = P.grid
    W, X = weights(P, st, R)
    K = fe.assemble_K_free(g, P.Ke, st.rho)
    B = fe.element_force_matrix(g, R.be)
    Suu = (K + B @ sp.diags(W) @ B.T).tocsr()
    c = B @ W
    S = sp.bmat([[Suu, sp.csr_matrix(c[:, None])],
                 [sp.csr_matrix(c[None, :]), sp.csr_matrix([[W.sum()]])]], format="csr")
    WX = W * X
    rhs = np.concatenate([-R.res1[P.free] - B @ WX, [-R.res2 - WX.sum()]])
    return S, rhs, W, X


def increments(P, st: IPState, R: Residual, du: np.ndarray, dalpha: float):
    """Eq. (Delta_rho), then eq. (Delta_onu) and eq. (Delta_unu) in this
    order; du in the all-DOF layout.  Returns (drho, dnu_lo, dnu_hi)."""
    g = P.grid
    W, X = weights(P, st, R)
    t = np.einsum("ei,ei->e", R.be, g.mask(du)[g.dofs]) + dalpha     # B^T du + dalpha e
    drho = W * (t + X)
    dlo = st.rho - P.rho_lo
    dnh = (dlo * t - (st.nu_lo - st.nu_hi) * drho
           - (R.res4 + R.res5 - dlo * R.res3)) / (P.rho_hi - P.rho_lo)
    dnl = dnh - t - R.res3
    return drho, dnl, dnh


def _ratio_min(num, den, mask):
    return float(np.min(num[mask] / den[mask])) if np.any(mask) else math.inf


def step_lengths(P, st: IPState, drho, dnl, dnh, frac=0.9):
    """The step lengths of Algorithm 3: kappa_u = kappa_rho keeps rho
    strictly inside the bounds, kappa_nu_lo and kappa_nu_hi keep the
    multipliers positive, all at most 1."""
    up = _ratio_min(P.rho_hi - st.rho, drho, drho > 0)
    dn = _ratio_min(P.rho_lo - st.rho, drho, drho < 0)
    k_u = min(frac * up, frac * dn, 1.0)
    k_l = min(frac * _ratio_min(-st.nu_lo, dnl, dnl < 0), 1.0)
    k_h = min(frac * _ratio_min(-st.nu_hi, dnh, dnh < 0), 1.0)
    return k_u, k_l, k_h


def gap(P, u: np.ndarray, lam: float, e: np.ndarray) -> float:
    """delta(u, lambda) of eq. (2.6)."""
    a = lam - e
    return float(-0.5 * P.f @ u + lam * P.V - np.sum(np.minimum(P.rho_lo * a, P.rho_hi * a)))


def res_ip(P, st: IPState, R: Residual) -> float:
    """Feasibility measure of eq. (ip_res)."""
    m = P.grid.m
    return (np.linalg.norm(R.res1) / np.linalg.norm(P.f) + abs(R.res2) / P.V
            + np.linalg.norm(R.res3) / (np.linalg.norm(st.nu_lo) + np.linalg.norm(st.nu_hi))
            + abs(R.res4.sum()) / m + abs(R.res5.sum()) / m)


def interior(P, st: IPState) -> bool:
    """rho strictly inside its bounds and both multipliers positive."""
    return bool(np.all(st.rho > P.rho_lo) and np.all(st.rho < P.rho_hi)
                and np.all(st.nu_lo > 0) and np.all(st.nu_hi > 0))


def complementarity_max(P, st: IPState) -> float:
    """d of the MINRES rule for IP (Section 6.2)."""
    return float(max(np.max(np.abs((st.rho - P.rho_lo) * st.nu_lo)),
                     np.max(np.abs((P.rho_hi - st.rho) * st.nu_hi))))


@dataclass
class IPResult:
    state: IPState
    iterations: int
    converged: bool
    minres: int
    history: List[dict] = field(default_factory=list)
    status: str = "ok"      # "ok", "max_iter" or "boundary"


class Solver:
    """Algorithm 3.  `linsolve(S, rhs, eps)` may be replaced (tests use a
    direct solve); the default is MINRES preconditioned by one V-cycle."""

    def __init__(self, problem, opts: Optional[IPOptions] = None, linsolve=None):
        from . import pbm
        self.P = pbm.VTS(problem)
        self.opts = opts or IPOptions()
        self.levels_count = problem.levels
        self._linsolve = linsolve
        o = self.opts
        self.r, self.s = o.r0, o.s0
        self.eps_mr = o.eps_mr0
        self.r_plus = self.s_plus = None

    def linsolve(self, S, rhs):
        from . import mg, minres
        if self._linsolve is not None:
            return self._linsolve(S, rhs, self.eps_mr), 0
        h = mg.Hierarchy(self.P.grid, S, self.levels_count)
        x, its, _ = minres.minres(lambda v: S @ v, rhs, h.vcycle, self.eps_mr,
                                  self.opts.max_minres, stop_on_indefinite=True)
        return x, its

    def _plus(self, st: IPState):
        P, o = self.P, self.opts
        m = P.grid.m
        self.r_plus = o.sigma_r * float(st.nu_lo @ (st.rho - P.rho_lo)) / m
        self.s_plus = o.sigma_s * float(st.nu_hi @ (P.rho_hi - st.rho)) / m

    def step(self, st: IPState):
        """One pass of the loop of Algorithm 3; returns (state, record)."""
        P, o = self.P, self.opts
        if self.r_plus is None:
            self._plus(st)
        R = residual(P, st, self.r, self.s)
        S, rhs, _, _ = reduced_system(P, st, R)
        dy, its = self.linsolve(S, rhs)
        du = np.zeros(P.grid.n_dof)
        du[P.free] = dy[:-1]
        da = float(dy[-1])
        drho, dnl, dnh = increments(P, st, R, du, da)
        r_used, s_used = self.r, self.s
        self.r, self.s = self.r_plus, self.s_plus
        k_u, k_l, k_h = step_lengths(P, st, drho, dnl, dnh, o.step_frac)
        new = IPState(st.u + k_u * du, st.alpha + da, st.rho + k_u * drho,
                      st.nu_lo + k_l * dnl, st.nu_hi + k_h * dnh)
        if not interior(P, new):
            # rounding put a variable on its bound: the barrier terms are no
            # longer defined and the iteration cannot continue
            return new, dict(r=r_used, s=s_used, kappa_u=k_u, kappa_nu_lo=k_l,
                             kappa_nu_hi=k_h, minres=its, eps_mr=self.eps_mr,
                             converged=False, interior=False)
        R1 = residual(P, new, self.r, self.s)
        obj = 0.5 * float(P.f @ new.u)
        delta = gap(P, new.u, -new.alpha, R1.e)
        rip = res_ip(P, new, R1)
        ratio = delta / obj if obj != 0 else math.inf
        converged = (o.eps_ip > ratio > -0.1 * o.eps_ip) and rip < 10 * o.eps_ip
        rec = dict(gap=delta, objective=obj, ratio=ratio, res_ip=rip, r=r_used, s=s_used,
                   kappa_u=k_u, kappa_nu_lo=k_l, kappa_nu_hi=k_h, minres=its,
                   eps_mr=self.eps_mr, converged=converged, interior=True)
        self._plus(new)
        d = complementarity_max(P, new)
        cand = max(100.0 * d, o.eps_mr_min)
        if cand < self.eps_mr:
            self.eps_mr = cand
        return new, rec

    def solve(self, st: Optional[IPState] = None, iterations: Optional[int] = None) -> IPResult:
        """Algorithm 3 from the initial point (or st); with `iterations`
        set, exactly that many passes (no stopping test)."""
        P, o = self.P, self.opts
        if st is None:
            st = initial_state(P.grid.n_dof, P.grid.m, P.V)
        hist = []
        n = iterations if iterations is not None else o.max_iter
        converged = False
        status = "ok" if iterations is not None else "max_iter"
        for _ in range(n):
            st, rec = self.step(st)
            hist.append(rec)
            if not rec["interior"]:
                status = "boundary"
                break
            if iterations is None and rec["converged"]:
                converged, status = True, "ok"
                break
        return IPResult(st, len(hist), converged, sum(h["minres"] for h in hist), hist,
                        status)
