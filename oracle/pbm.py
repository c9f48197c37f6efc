"""PBM applied to the dual VTS problem (Section 3.2), written out step by step.

Variables xi = (u, alpha, nu_lo, nu_hi); multipliers (rho, mu_lo, mu_hi);
penalties (p, q_lo, q_hi).  All displacement-sized vectors live in the
all-DOF layout with zeros at fixed DOFs; the linear algebra of the reduced
system runs on the free DOFs plus the scalar alpha (size n+1).

Readings of the paper used here:
  * the constant term of res_3 in eq. (3.10) is taken as -rho_lo (the sign
    that differentiating eq. (3.9) gives; it is printed as +rho_lo);
  * the mu_lo update of Algorithm 1 uses phi'(-nu_lo/q_lo), as eq. (3.4)
    and the definition of h_lo prescribe;
  * the 2x2 per-element inverse of the (nu_lo, nu_hi) block and the Schur
    complement are evaluated in the closed forms derived below, which are
    algebraically identical to eq. (3.12) and its inverse formula but avoid
    the cancellation rho''^2 - rho''^2 when the penalties are small.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import fe
from .penalty import phi, dphi, d2phi, phi_diff


# ----------------------------------------------------------------------------
# options and state
# ----------------------------------------------------------------------------
@dataclass
class Options:
    """Parameters of Algorithms 1 and 2.  beta, gamma, p_min, eps_nwt0 and the
    MINRES rule are the values stated after Algorithm 1 and in Section 6.2.
    eps_pbm, eps_nwt_min and eps_nwt_final are tighter than the paper's
    (1e-5..1e-6, 1e-3, 10 eps_pbm) so that the result meets a KKT residual of
    1e-6.  The floor of the energy-constraint penalties p is relative to the
    energy scale of the problem: p >= p_min |alpha| (alpha, the volume
    multiplier, equals the common element energy of the optimum), instead of
    the paper's absolute 1e-8; the floor of q_lo, q_hi is q_min |alpha| with
    the paper's q_min = 1e-8.  The constraint functions e_i - alpha + nu_lo -
    nu_hi scale with the square of the load, and an absolute floor makes
    the method's behaviour depend on that scale; the multiplier method
    converges for any positive floor, the Schur weights grow like rho/p, so a
    moderate floor keeps the Newton systems within reach of the Gauss-Seidel
    multigrid, while a small q keeps weakly active bound multipliers
    converging quickly.  `paper_options()` returns the paper's values."""
    beta: float = 0.3
    gamma: float = 0.3
    p_min: float = 1e-3                       # floor of p / |alpha|; paper: 1e-8 absolute
    p_min_relative: bool = True               # False: p_min, q_min are absolute floors
    q_min: float = 1e-8                       # floor of q_lo, q_hi (the paper's value)
    eps_pbm: float = 1e-8
    eps_nwt0: float = 1.0
    eps_nwt_min: float = 1e-5
    eps_nwt_final: Optional[float] = 5e-7     # None -> 10 * eps_pbm
    eps_stat: Optional[float] = 5e-7          # None -> gap test only
    accept_stall: float = 1e-6                # final-Newton stall accepted below this res
    eps_mr0: Optional[float] = None           # None -> 1e-4 sqrt(n)
    eps_mr_min: float = 1e-9
    armijo_c1: float = 1e-4
    armijo_min: float = 2.0 ** -30
    max_outer: int = 500
    max_newton: int = 100
    max_minres: int = 500
    final_res4: bool = True                   # final Newton also tests res_4
    stall_steps: int = 10                     # final Newton: stop after this many steps without progress
    final_state_solve: bool = True            # u <- K(rho)^-1 f for the returned rho
    kkt_tol: float = 1e-6                     # > 0: success iff the KKT residual is below it


# outer-loop resumptions after a final KKT check that misses kkt_tol (R31)
KKT_RESUMES = 3


def p_floor(o: "Options", alpha: float) -> float:
    """Floor of the penalty parameters p after an outer iteration."""
    if o.p_min_relative and alpha != 0.0:
        return o.p_min * abs(alpha)
    return o.p_min


def q_floor(o: "Options", alpha: float) -> float:
    """Floor of the penalty parameters q_lo, q_hi after an outer iteration
    (relative to the same energy scale as p when p_min_relative is set)."""
    if o.p_min_relative and alpha != 0.0:
        return o.q_min * abs(alpha)
    return o.q_min


def paper_options(eps_pbm: float = 1e-5) -> "Options":
    """The parameter values of the paper's experiments (Section 7)."""
    return Options(eps_pbm=eps_pbm, eps_nwt_min=1e-3, eps_nwt_final=None,
                   final_res4=False, eps_stat=None, accept_stall=0.0, p_min=1e-8,
                   p_min_relative=False, q_min=1e-8, final_state_solve=False, kkt_tol=0.0)


@dataclass
class State:
    u: np.ndarray
    alpha: float
    nu_lo: np.ndarray
    nu_hi: np.ndarray
    rho: np.ndarray
    mu_lo: np.ndarray
    mu_hi: np.ndarray
    p: np.ndarray
    q_lo: np.ndarray
    q_hi: np.ndarray

    def copy(self):
        return State(self.u.copy(), float(self.alpha), self.nu_lo.copy(),
                     self.nu_hi.copy(), self.rho.copy(), self.mu_lo.copy(),
                     self.mu_hi.copy(), self.p.copy(), self.q_lo.copy(),
                     self.q_hi.copy())


def initial_state(n_dof: int, m: int, V: float) -> State:
    """Initial point stated after Algorithm 1: u = 0, alpha = 1,
    nu_lo = nu_hi = e, rho_i = V/m, mu_lo = mu_hi = e, p = q = e."""
    one = np.ones(m)
    return State(np.zeros(n_dof), 1.0, one.copy(), one.copy(),
                 np.full(m, V / m), one.copy(), one.copy(), one.copy(),
                 one.copy(), one.copy())


class VTS:
    """Problem data: grid, K_e, load, volume, bounds (problem (1.1))."""

    def __init__(self, problem):
        self.pr = problem
        self.grid = fe.Grid(problem.nx, problem.ny, problem.nz, problem.fixed)
        self.Ke = fe.element_stiffness(problem.E, problem.nu, problem.h)
        self.f = self.grid.mask(problem.f)
        self.V = float(problem.V)
        m = self.grid.m
        self.rho_lo = np.broadcast_to(np.asarray(problem.rho_lo, float), (m,)).copy()
        self.rho_hi = np.broadcast_to(np.asarray(problem.rho_hi, float), (m,)).copy()
        self.free = self.grid.free
        self.n = self.free.size


# ----------------------------------------------------------------------------
# evaluation of the augmented Lagrangian, its derivatives, eq. (3.9)-(3.11)
# ----------------------------------------------------------------------------
@dataclass
class Eval:
    e: np.ndarray
    be: np.ndarray          # m x 24, b_i = K_i u on element i's DOFs
    s: np.ndarray
    t_lo: np.ndarray
    t_hi: np.ndarray
    rho1: np.ndarray        # rho'
    rho2: np.ndarray        # rho''
    mu_lo1: np.ndarray
    mu_lo2: np.ndarray
    mu_hi1: np.ndarray
    mu_hi2: np.ndarray
    g1: np.ndarray          # all-DOF, masked
    g2: float
    g3: np.ndarray
    g4: np.ndarray


def evaluate(P: VTS, st: State) -> Eval:
    """Section 3.2: s_i, the weights rho', rho'', mu', mu'' and the gradient
    (res_1, ..., res_4) of eq. (3.10) with the constant of res_3 = -rho_lo."""
    g = P.grid
    e = fe.element_energies(g, P.Ke, st.u)
    be = fe.element_forces(g, P.Ke, st.u)
    s = (e - st.alpha + st.nu_lo - st.nu_hi) / st.p
    t_lo = -st.nu_lo / st.q_lo
    t_hi = -st.nu_hi / st.q_hi
    rho1 = st.rho * dphi(s)
    rho2 = st.rho / st.p * d2phi(s)
    mu_lo1 = st.mu_lo * dphi(t_lo)
    mu_lo2 = st.mu_lo / st.q_lo * d2phi(t_lo)
    mu_hi1 = st.mu_hi * dphi(t_hi)
    mu_hi2 = st.mu_hi / st.q_hi * d2phi(t_hi)
    g1 = fe.apply_K(g, P.Ke, rho1, st.u) - P.f
    g2 = P.V - rho1.sum()
    g3 = -P.rho_lo + rho1 - mu_lo1
    g4 = P.rho_hi - rho1 - mu_hi1
    return Eval(e, be, s, t_lo, t_hi, rho1, rho2, mu_lo1, mu_lo2, mu_hi1,
                mu_hi2, g1, g2, g3, g4)


def lagrangian(P: VTS, st: State) -> float:
    """Augmented Lagrangian, eq. (3.9)."""
    e = fe.element_energies(P.grid, P.Ke, st.u)
    s = (e - st.alpha + st.nu_lo - st.nu_hi) / st.p
    return (st.alpha * P.V - P.f @ st.u - P.rho_lo @ st.nu_lo + P.rho_hi @ st.nu_hi
            + np.sum(st.rho * st.p * phi(s))
            + np.sum(st.mu_lo * st.q_lo * phi(-st.nu_lo / st.q_lo))
            + np.sum(st.mu_hi * st.q_hi * phi(-st.nu_hi / st.q_hi)))


def lagrangian_change(P: VTS, st: State, ev: Eval, du: np.ndarray, dalpha: float,
                      dnl: np.ndarray, dnh: np.ndarray, kappa: float) -> float:
    """L(xi + kappa dxi) - L(xi) of eq. (3.9) along the Newton direction
    dxi = (du, dalpha, dnl, dnh), as the Armijo rule of Algorithm 2 needs it.

    Every term is formed as a change along the ray, never as the difference
    of two large totals: the element energy is quadratic in u, so exactly
        e_i(u + kappa du) - e_i(u) = kappa b_i^T du_i + kappa^2 e_i(du),
    with b_i = K_i u from the evaluation at xi; the arguments of phi change
    by that amount (and by the alpha and nu steps) over p or q; phi's change
    is taken from its branch-wise difference formula; the linear terms of
    (3.9) change by kappa times their directional part.  Near the optimum
    the decrease kappa * slope is far below the rounding of e_i(u), phi and
    f^T u, and forming the two totals lets that rounding decide the Armijo
    test."""
    g = P.grid
    c1 = np.einsum("ei,ei->e", ev.be, du[g.dofs])
    c2 = fe.element_energies(g, P.Ke, du)
    s0 = (ev.e - st.alpha + st.nu_lo - st.nu_hi) / st.p
    ds = kappa * (c1 + kappa * c2 - dalpha + dnl - dnh) / st.p
    lin = kappa * (dalpha * P.V - P.f @ du - P.rho_lo @ dnl + P.rho_hi @ dnh)
    pen = np.sum(st.rho * st.p * phi_diff(s0, ds))
    pen += np.sum(st.mu_lo * st.q_lo * phi_diff(-st.nu_lo / st.q_lo, -kappa * dnl / st.q_lo))
    pen += np.sum(st.mu_hi * st.q_hi * phi_diff(-st.nu_hi / st.q_hi, -kappa * dnh / st.q_hi))
    return float(lin + pen)


def res_pbm(P: VTS, ev: Eval) -> float:
    """Feasibility measure of eq. (3.15): ||res1||/||f|| + |res2|/V +
    ||res3||/(||rho_lo|| + ||rho_hi||)."""
    return (np.linalg.norm(ev.g1) / np.linalg.norm(P.f) + abs(ev.g2) / P.V
            + np.linalg.norm(ev.g3) / (np.linalg.norm(P.rho_lo) + np.linalg.norm(P.rho_hi)))


def res4_term(P: VTS, ev: Eval) -> float:
    return np.linalg.norm(ev.g4) / (np.linalg.norm(P.rho_lo) + np.linalg.norm(P.rho_hi))


# ----------------------------------------------------------------------------
# the reduced Newton system, eqs. (3.11)-(3.14)
# ----------------------------------------------------------------------------
def nu_block(ev: Eval):
    """Per element, the 2x2 block [[H33_ii, H34_ii], [H34_ii, H44_ii]] =
    [[r''+ml'', -r''], [-r'', r''+mh'']] has determinant
    det = r''(ml''+mh'') + ml'' mh'' (the r''^2 terms cancel exactly) and
    inverse (1/det) [[r''+mh'', r''], [r'', r''+ml'']]."""
    r2, l2, h2 = ev.rho2, ev.mu_lo2, ev.mu_hi2
    det = r2 * (l2 + h2) + l2 * h2
    return det


def schur_weights(ev: Eval):
    """Closed form of eq. (3.12).  Element i couples (u, alpha) to its two nu
    unknowns through c_i [1, -1] with c_i = rho''_i [b_i; -1].  Subtracting
    c_i [1,-1] A_i^{-1} [1,-1]^T c_i^T = rho''^2 (ml''+mh'')/det c c^T from
    the rho''_i [b;-1][b;-1]^T part of H leaves weight
        w_i = rho'' ml'' mh'' / det  ( = 1/(1/rho'' + 1/ml'' + 1/mh'') ),
    and the right-hand side term H_{y nu} A^{-1} (res3, res4) becomes
        z_i [b_i; -1],  z_i = rho''(mh'' res3_i - ml'' res4_i)/det."""
    det = nu_block(ev)
    w = ev.rho2 * ev.mu_lo2 * ev.mu_hi2 / det
    z = ev.rho2 * (ev.mu_hi2 * ev.g3 - ev.mu_lo2 * ev.g4) / det
    return w, z, det


def schur_matrix(P: VTS, ev: Eval) -> sp.csr_matrix:
    """S of eq. (3.12) on (free u, alpha):
        S = [[K(rho') + B diag(w) B^T, -B w], [-(B w)^T, sum w]]."""
    g = P.grid
    w, _, _ = schur_weights(ev)
    K1 = fe.assemble_K_free(g, P.Ke, ev.rho1)
    B = fe.element_force_matrix(g, ev.be)
    Suu = (K1 + B @ sp.diags(w) @ B.T).tocsr()
    c = -(B @ w)
    S = sp.bmat([[Suu, sp.csr_matrix(c[:, None])],
                 [sp.csr_matrix(c[None, :]), sp.csr_matrix([[w.sum()]])]], format="csr")
    return S


def reduced_rhs(P: VTS, ev: Eval) -> np.ndarray:
    """rhs of eq. (3.13): [-res1 + B z; -res2 - sum z] (free DOFs, alpha)."""
    _, z, _ = schur_weights(ev)
    Bz = fe.scatter(P.grid, z[:, None] * ev.be)
    ru = (-ev.g1 + Bz)[P.free]
    return np.concatenate([ru, [-ev.g2 - z.sum()]])


def schur_apply(P: VTS, ev: Eval, x_free: np.ndarray, beta: float):
    """y = S [x; beta] without assembling S (used by parity tests)."""
    g = P.grid
    w, _, _ = schur_weights(ev)
    x = np.zeros(g.n_dof)
    x[P.free] = x_free
    t = np.einsum("ei,ei->e", ev.be, x[g.dofs]) - beta
    yu = fe.apply_K(g, P.Ke, ev.rho1, x) + fe.scatter(g, (w * t)[:, None] * ev.be)
    return yu[P.free], float(-(w * t).sum())


def delta_nu(ev: Eval, tau: np.ndarray):
    """Eq. (3.14): with tau_i = b_i^T du - dalpha,
        (dnl, dnh) = -A_i^{-1} (res3 + r'' tau, res4 - r'' tau),
    multiplied out (the r''^2 tau terms cancel exactly)."""
    r2, l2, h2 = ev.rho2, ev.mu_lo2, ev.mu_hi2
    det = nu_block(ev)
    dnl = -((r2 + h2) * ev.g3 + r2 * ev.g4 + r2 * h2 * tau) / det
    dnh = -(r2 * ev.g3 + (r2 + l2) * ev.g4 - r2 * l2 * tau) / det
    return dnl, dnh


def full_hessian(P: VTS, ev: Eval) -> np.ndarray:
    """Dense Hessian of eq. (3.11) on (free u, alpha, nu_lo, nu_hi); for tiny
    grids only (pins the reduction)."""
    g = P.grid
    n, m = P.n, g.m
    B = fe.element_force_matrix(g, ev.be).toarray()          # n x m
    r1, r2 = ev.rho1, ev.rho2
    K1 = fe.assemble_K_free(g, P.Ke, r1).toarray()
    N = n + 1 + 2 * m
    H = np.zeros((N, N))
    H[:n, :n] = (B * r2) @ B.T + K1                            # H11
    H[:n, n] = -(B @ r2)                                       # H12
    H[:n, n + 1:n + 1 + m] = B * r2                            # H13
    H[:n, n + 1 + m:] = -(B * r2)                              # H14
    H[n, n] = r2.sum()                                         # H22
    H[n, n + 1:n + 1 + m] = -r2                                # H23
    H[n, n + 1 + m:] = r2                                      # H24
    idx_l = np.arange(n + 1, n + 1 + m)
    idx_h = np.arange(n + 1 + m, N)
    H[idx_l, idx_l] = r2 + ev.mu_lo2                           # H33
    H[idx_l, idx_h] = -r2                                      # H34
    H[idx_h, idx_h] = r2 + ev.mu_hi2                           # H44
    iu = np.triu_indices(N, 1)
    H[(iu[1], iu[0])] = H[iu]
    return H


def full_gradient(P: VTS, ev: Eval) -> np.ndarray:
    return np.concatenate([ev.g1[P.free], [ev.g2], ev.g3, ev.g4])


def schur_literal(P: VTS, ev: Eval) -> np.ndarray:
    """S of eq. (3.12) computed literally as H_yy - H_ynu H_nunu^{-1} H_nuy
    with a dense inverse (tiny grids, well-scaled data only)."""
    H = full_hessian(P, ev)
    k = P.n + 1
    return H[:k, :k] - H[:k, k:] @ np.linalg.solve(H[k:, k:], H[k:, :k])


# ----------------------------------------------------------------------------
# gap and dual objective, eq. (2.6) and the objective of (2.1)
# ----------------------------------------------------------------------------
def duality_gap(P: VTS, st: State, e: Optional[np.ndarray] = None) -> float:
    """delta(u, alpha) of eq. (2.6)."""
    if e is None:
        e = fe.element_energies(P.grid, P.Ke, st.u)
    a = st.alpha - e
    return float(-0.5 * P.f @ st.u + st.alpha * P.V
                 - np.sum(np.minimum(P.rho_lo * a, P.rho_hi * a)))


def dual_objective(P: VTS, st: State) -> float:
    """d(u, alpha, nu_lo, nu_hi): objective of problem (2.1)."""
    return float(st.alpha * P.V - P.f @ st.u - P.rho_lo @ st.nu_lo + P.rho_hi @ st.nu_hi)


def update_multipliers(st: State, ev: Eval, beta: float, rho_only=False):
    """Algorithm 1, multiplier step: rho+ = rho phi'(s), mu_lo+ = mu_lo
    phi'(-nu_lo/q_lo), mu_hi+ = mu_hi phi'(-nu_hi/q_hi), each clipped into
    [beta x, x/beta]."""
    def clip(x, xp):
        return np.minimum(np.maximum(xp, beta * x), x / beta)
    rho = clip(st.rho, st.rho * dphi(ev.s))
    if rho_only:
        return rho, st.mu_lo, st.mu_hi
    mu_lo = clip(st.mu_lo, st.mu_lo * dphi(ev.t_lo))
    mu_hi = clip(st.mu_hi, st.mu_hi * dphi(ev.t_hi))
    return rho, mu_lo, mu_hi


def stationarity(P: VTS, rho: np.ndarray, e: np.ndarray, alpha: float) -> float:
    """Estimate of the KKT stationarity/box terms for a candidate density:
    max_i |rho_i - Proj_[lo,hi](rho_i + (e_i - alpha)/alpha)| / hi_i, with e
    from the current u (an addition to Algorithm 1's gap test, used so that
    the final density meets a KKT residual target)."""
    proj = np.clip(rho + (e - alpha) / alpha, P.rho_lo, P.rho_hi)
    return float(np.max(np.abs(rho - proj) / P.rho_hi))


# ----------------------------------------------------------------------------
# Algorithm 2 (PBM NEWTON) and Algorithm 1 (PBM)
# ----------------------------------------------------------------------------
@dataclass
class Log:
    newton: list = field(default_factory=list)
    outer: list = field(default_factory=list)


class Solver:
    """Oracle PBM solver.  `linsolve(S, rhs, eps)` may be replaced (tests use
    a direct solve); the default is MINRES preconditioned by one V-cycle.

    The problem-specific steps (evaluation, Schur matrix, right-hand side,
    gap, the split of a Newton solution, the final checks) are the class
    attributes and small methods below; the multi-load solver replaces them
    and keeps Algorithms 1 and 2 as written here."""

    problem_class = VTS
    evaluate = staticmethod(evaluate)
    schur_matrix = staticmethod(schur_matrix)
    reduced_rhs = staticmethod(reduced_rhs)
    lagrangian_change = staticmethod(lagrangian_change)
    res_pbm = staticmethod(res_pbm)
    duality_gap = staticmethod(duality_gap)
    dual_objective = staticmethod(dual_objective)

    def __init__(self, problem, opts: Optional[Options] = None, linsolve=None):
        from . import mg, minres
        self.P = self.problem_class(problem)
        self.opts = opts or Options()
        self.levels_count = problem.levels
        self.mg = mg
        self.minres = minres
        self._linsolve = linsolve
        n = self.P.n
        self.eps_mr = (self.opts.eps_mr0 if self.opts.eps_mr0 is not None
                       else 1e-4 * math.sqrt(n))
        self.res_prev = None
        self.log = Log()
        self.status = "ok"
        self.progress = None                  # optional callback(outer index, outer log entry)

    # one linear solve of eq. (3.13)
    def linsolve(self, ev, S, rhs):
        if self._linsolve is not None:
            return self._linsolve(S, rhs, self.eps_mr), 0
        h = self.hierarchy(S)
        x, its, _ = self.minres.minres(lambda v: S @ v, rhs, h.vcycle,
                                       self.eps_mr, self.opts.max_minres)
        return x, its

    def hierarchy(self, S):
        return self.mg.Hierarchy(self.P.grid, S, self.levels_count)

    def initial(self) -> State:
        P = self.P
        return initial_state(P.grid.n_dof, P.grid.m, P.V)

    def split(self, dy):
        """(du in the all-DOF layout, dalpha) from a solution of (3.13)."""
        P = self.P
        du = np.zeros(P.grid.n_dof)
        du[P.free] = dy[:-1]
        return du, float(dy[-1])

    def tau(self, ev, du, da):
        """tau_i = b_i^T du_i - dalpha of eq. (3.14)."""
        return np.einsum("ei,ei->e", ev.be, du[self.P.grid.dofs]) - da

    def slope(self, ev, du, da, dnl, dnh):
        """Directional derivative of (3.9) along the Newton direction."""
        return float(ev.g1 @ du + ev.g2 * da + ev.g3 @ dnl + ev.g4 @ dnh)

    def final_checks(self, st):
        """The state of the returned density and the KKT residual."""
        P, o = self.P, self.opts
        if o.final_state_solve and np.min(P.rho_lo) > 0:
            # the primal pair of problem (1.1): the state of the returned density
            # (with a zero lower bound K(rho) may be singular on a void region,
            # where the state equation leaves u free; the dual iterate is then
            # the displacement that meets the optimality conditions)
            from .kkt import solve_state
            st.u = solve_state(P.grid, P.Ke, st.rho, P.f)
        from .kkt import kkt_residual
        return kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho,
                            st.u, st.alpha)

    def newton(self, st: State, eps_nwt: float, final=False):
        """Algorithm 2.  The MINRES tolerance rule of Section 6.2 compares
        res_PBM of consecutive steps of this call.  Status "newton_limit" if
        max_newton steps do not meet eps_nwt; "stalled" once stall_steps
        steps in a row bring no new best value below 0.9 times the best so
        far (the outer loop accepts a stalled call before the final one)."""
        P, o = self.P, self.opts
        ev = self.evaluate(P, st)
        self.res_prev = None
        best, since = np.inf, 0
        for it in range(o.max_newton):
            S = self.schur_matrix(P, ev)
            rhs = self.reduced_rhs(P, ev)
            tries = 0
            while True:
                dy, mr_its = self.linsolve(ev, S, rhs)
                du, da = self.split(dy)
                tau = self.tau(ev, du, da)
                dnl, dnh = delta_nu(ev, tau)
                slope = self.slope(ev, du, da, dnl, dnh)
                if slope < 0 or tries >= 1 or self._linsolve is not None:
                    break
                # a non-descent direction: tighten the MINRES tolerance once
                self.eps_mr = max(0.1 * self.eps_mr, o.eps_mr_min)
                tries += 1
            if slope >= 0:
                self.status = "nondescent"
                return st, ev
            kappa = 1.0
            while self.lagrangian_change(P, st, ev, du, da, dnl, dnh, kappa) > \
                    o.armijo_c1 * kappa * slope:
                kappa *= 0.5
                if kappa < o.armijo_min:
                    self.status = "linesearch"
                    return st, ev
            new = st.copy()
            new.u = st.u + kappa * du
            new.alpha = st.alpha + kappa * da
            new.nu_lo = st.nu_lo + kappa * dnl
            new.nu_hi = st.nu_hi + kappa * dnh
            st = new
            ev = self.evaluate(P, st)
            res = self.res_pbm(P, ev)
            r4 = res4_term(P, ev)
            self.log.newton.append(dict(res=res, res4=r4, kappa=kappa,
                                        minres=mr_its, eps_mr=self.eps_mr))
            if self.res_prev is not None and res > 0.9 * self.res_prev:
                self.eps_mr = max(0.1 * self.eps_mr, o.eps_mr_min)
            self.res_prev = res
            crit = res + r4 if (final and o.final_res4) else res
            if crit < eps_nwt:
                break
            if crit < 0.9 * best:
                best, since = crit, 0
            else:
                since += 1
            if o.stall_steps > 0 and since >= o.stall_steps:
                self.status = "stalled"
                return st, ev
        else:
            self.status = "newton_limit"
        return st, ev

    def solve(self, st: Optional[State] = None):
        P, o = self.P, self.opts
        if st is None:
            st = self.initial()
        eps_nwt = o.eps_nwt0
        eps_stat = o.eps_stat
        k, resumes = 0, 0
        while True:
            st, eps_nwt, k = self._outer_loop(st, eps_nwt, eps_stat, k)
            self._final(st)
            st = self.state
            if self.status == "kkt" and resumes < KKT_RESUMES and k < o.max_outer:
                # the returned state misses the KKT target (the final Newton
                # call moved the stationarity term past it): the outer loop
                # goes on from that state with half the stationarity target
                resumes += 1
                eps_stat = 0.5 * eps_stat
                self.status = "ok"
                continue
            return st

    def _outer_loop(self, st, eps_nwt, eps_stat, k0):
        """Outer iterations of Algorithm 1 from index k0 until its stopping
        test (gap ratio, and this library's stationarity term below
        eps_stat) holds; returns (state, eps_nwt, iterations so far)."""
        P, o = self.P, self.opts
        stat_best, stat_since = 0.0, -1
        k = k0
        while k < o.max_outer:
            k += 1
            st, ev = self.newton(st, eps_nwt)
            if self.status == "stalled":
                # a call before the final one that stalls is taken as the
                # minimizer (the rounding floor of res_PBM lies above its
                # tolerance); the multiplier update and the tests go on
                self.status = "ok"
            delta = self.duality_gap(P, st, ev.e)
            d = self.dual_objective(P, st)
            ratio = abs(delta / d)
            self.log.outer.append(dict(gap=delta, dual=d, ratio=ratio, eps_nwt=eps_nwt,
                                       sum_rho=float(st.rho.sum())))
            rho_n, mul_n, muh_n = update_multipliers(st, ev, o.beta)
            stat = stationarity(P, rho_n, ev.e, st.alpha) if eps_stat else 0.0
            self.log.outer[-1]["stat"] = stat
            if self.progress is not None:
                self.progress(k - 1, self.log.outer[-1])
            stat_ok = stat < (eps_stat or 1.0)
            if ratio < o.eps_pbm and not stat_ok and o.stall_steps > 0 and \
                    stat < 10.0 * (eps_stat or 1.0):
                # the stationarity test is an addition to Algorithm 1's gap test:
                # once the gap test holds and the term, within 10x of its target,
                # stops decreasing (no new value below 0.9 x its best for
                # stall_steps outer iterations), the loop ends and the final
                # Newton call and the KKT check decide
                if stat_since < 0 or stat < 0.9 * stat_best:
                    stat_best, stat_since = stat, 0
                else:
                    stat_since += 1
                    stat_ok = stat_since >= o.stall_steps
            if self.status != "ok" or (ratio < o.eps_pbm and stat_ok):
                break
            st.rho, st.mu_lo, st.mu_hi = rho_n, mul_n, muh_n
            st.p = np.maximum(o.gamma * st.p, p_floor(o, st.alpha))
            st.q_lo = np.maximum(o.gamma * st.q_lo, q_floor(o, st.alpha))
            st.q_hi = np.maximum(o.gamma * st.q_hi, q_floor(o, st.alpha))
            eps_nwt = max(min(100.0 * ratio, eps_nwt), o.eps_nwt_min)
        self._last_ev = ev
        return st, eps_nwt, k

    def _final(self, st):
        """The final Newton call of Algorithm 1, the last rho update and the
        result checks; sets self.state and self.status."""
        P, o = self.P, self.opts
        ev = self._last_ev
        eps_final = o.eps_nwt_final if o.eps_nwt_final is not None else 10.0 * o.eps_pbm
        self.kkt = None
        if self.status == "ok":
            st, ev = self.newton(st, eps_final, final=True)
            stalled = self.status != "ok"   # every Newton failure mode here is a stall
            if stalled and o.kkt_tol <= 0 and self.res_prev is not None and \
                    self.res_prev < o.accept_stall:
                self.status = "ok"          # near-optimal stall accepted
            if self.status == "ok" or (stalled and o.kkt_tol > 0):
                st.rho, _, _ = update_multipliers(st, ev, o.beta, rho_only=True)
                self.kkt = self.final_checks(st)
                if o.kkt_tol > 0:
                    self.status = "ok" if self.kkt["kkt"] <= o.kkt_tol else "kkt"
        else:
            st.rho, _, _ = update_multipliers(st, ev, o.beta, rho_only=True)
        self.state = st
