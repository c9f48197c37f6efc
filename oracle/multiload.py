"""PBM for the multi-load VTS problem, written out step by step.

ORACLE: test infrastructure.  Only tests, the smoke check and the CPU
baseline of the benchmark may import this module.

The multi-load problem minimises the sum of the compliances of k load cases
f_1, ..., f_k over one density (an extension of problem (1.1) of Section 1,
which has one load):
    min_rho  sum_l 1/2 f_l^T u_l   s.t.  K(rho) u_l = f_l (l = 1..k),
             sum rho <= V,  rho_lo <= rho <= rho_hi.
Reading used here: this is problem (1.1) itself for the stacked displacement
U = (u_1, ..., u_k), the stacked load F = (f_1, ..., f_k) and the element
matrices blockdiag(K_i, ..., K_i); K(rho) acts on each load case alone.  So
the duality theory of Section 2 and the PBM of Section 3.2 carry over with
  e_i(U)  = sum_l 1/2 u_l^T K_i u_l          (the element energy of all cases)
  b_i     = (K_i u_1; ...; K_i u_k)           (24k entries per element)
  res_1   = (K(rho') u_l - f_l)_l,   F^T U = sum_l f_l^T u_l,
and Algorithms 1 and 2 unchanged (this module supplies only the steps that
see U; the loop is the single-load solver's).  The Newton system (3.12) is
    S = [[I_k (x) K(rho') + B diag(w) B^T, -B w], [-(B w)^T, sum w]]
with B = (B_1; ...; B_k) the stacked element-force matrix: its rank-one
element terms couple the load cases.

Layout: U is a (k, n_dof) array in the all-DOF layout of each case; the
reduced system runs on the stacked free DOFs (u_1[free], ..., u_k[free])
followed by alpha (size k n + 1).  The multigrid is the single-load one of
Section 6 with a node block holding the node's 3k DOFs over all load cases
and the trilinear prolongation acting on each case (oracle/mg.py, nload).

Pins (tests/test_oracle_multiload.py): one load case reproduces the
single-load oracle exactly; cases (f, c f) reproduce the single-load solve
for the load sqrt(1 + c^2) f (same density, multiplier and iteration
counts); a zero second case changes nothing; the gradient and the Schur
matrix against finite differences of the augmented Lagrangian written from
its definition; the optimal compliance of a tiny two-case problem against a
general-purpose constrained minimisation of the primal.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe, pbm
from .penalty import phi, dphi, d2phi, phi_diff


def _load_cases(problem) -> np.ndarray:
    cases = problem.extra.get("load_cases")
    if cases is None:
        return problem.f[None, :].copy()
    return np.asarray(cases, dtype=np.float64)


class MultiVTS(pbm.VTS):
    """Problem data with k load cases: F is (k, n_dof), masked."""

    def __init__(self, problem):
        super().__init__(problem)
        self.F = np.stack([self.grid.mask(fl) for fl in _load_cases(problem)])
        self.k = self.F.shape[0]
        self.f = self.F.sum(axis=0)          # informative only; F is the load


def initial_state(P: MultiVTS) -> pbm.State:
    """The initial point of Algorithm 1 with U = 0."""
    st = pbm.initial_state(P.grid.n_dof, P.grid.m, P.V)
    st.u = np.zeros((P.k, P.grid.n_dof))
    return st


def energies(P: MultiVTS, U: np.ndarray) -> np.ndarray:
    """e_i(U) = sum_l 1/2 u_l^T K_i u_l."""
    return sum(fe.element_energies(P.grid, P.Ke, U[l]) for l in range(P.k))


def forces(P: MultiVTS, U: np.ndarray) -> np.ndarray:
    """b_i = K_i u_l per case: (k, m, 24)."""
    return np.stack([fe.element_forces(P.grid, P.Ke, U[l]) for l in range(P.k)])


def evaluate(P: MultiVTS, st: pbm.State) -> pbm.Eval:
    """Section 3.2 on the stacked problem: s_i from the summed energies, the
    same weights, res_1 per case (a (k, n_dof) array), res_2..res_4 as for one
    load."""
    e = energies(P, st.u)
    be = forces(P, st.u)
    s = (e - st.alpha + st.nu_lo - st.nu_hi) / st.p
    t_lo = -st.nu_lo / st.q_lo
    t_hi = -st.nu_hi / st.q_hi
    rho1 = st.rho * dphi(s)
    rho2 = st.rho / st.p * d2phi(s)
    mu_lo1 = st.mu_lo * dphi(t_lo)
    mu_lo2 = st.mu_lo / st.q_lo * d2phi(t_lo)
    mu_hi1 = st.mu_hi * dphi(t_hi)
    mu_hi2 = st.mu_hi / st.q_hi * d2phi(t_hi)
    g1 = np.stack([fe.apply_K(P.grid, P.Ke, rho1, st.u[l]) - P.F[l] for l in range(P.k)])
    g2 = P.V - rho1.sum()
    g3 = -P.rho_lo + rho1 - mu_lo1
    g4 = P.rho_hi - rho1 - mu_hi1
    return pbm.Eval(e, be, s, t_lo, t_hi, rho1, rho2, mu_lo1, mu_lo2, mu_hi1,
                    mu_hi2, g1, g2, g3, g4)


def lagrangian(P: MultiVTS, st: pbm.State) -> float:
    """Augmented Lagrangian (3.9) of the stacked problem, from its definition."""
    e = energies(P, st.u)
    s = (e - st.alpha + st.nu_lo - st.nu_hi) / st.p
    FU = float(np.sum(P.F * st.u))
    return (st.alpha * P.V - FU - P.rho_lo @ st.nu_lo + P.rho_hi @ st.nu_hi
            + np.sum(st.rho * st.p * phi(s))
            + np.sum(st.mu_lo * st.q_lo * phi(-st.nu_lo / st.q_lo))
            + np.sum(st.mu_hi * st.q_hi * phi(-st.nu_hi / st.q_hi)))


def tau(P: MultiVTS, ev: pbm.Eval, dU: np.ndarray, da: float) -> np.ndarray:
    """tau_i = b_i^T dU_i - dalpha (sum over the load cases)."""
    dofs = P.grid.dofs
    return sum(np.einsum("ei,ei->e", ev.be[l], dU[l][dofs]) for l in range(P.k)) - da


def lagrangian_change(P: MultiVTS, st: pbm.State, ev: pbm.Eval, dU: np.ndarray,
                      dalpha: float, dnl: np.ndarray, dnh: np.ndarray, kappa: float) -> float:
    """L(xi + kappa dxi) - L(xi) along the ray, term by term as for one load:
    e_i(U + kappa dU) - e_i(U) = kappa b_i^T dU_i + kappa^2 e_i(dU)."""
    c1 = tau(P, ev, dU, 0.0)
    c2 = energies(P, dU)
    s0 = (ev.e - st.alpha + st.nu_lo - st.nu_hi) / st.p
    ds = kappa * (c1 + kappa * c2 - dalpha + dnl - dnh) / st.p
    lin = kappa * (dalpha * P.V - float(np.sum(P.F * dU)) - P.rho_lo @ dnl + P.rho_hi @ dnh)
    pen = np.sum(st.rho * st.p * phi_diff(s0, ds))
    pen += np.sum(st.mu_lo * st.q_lo * phi_diff(-st.nu_lo / st.q_lo, -kappa * dnl / st.q_lo))
    pen += np.sum(st.mu_hi * st.q_hi * phi_diff(-st.nu_hi / st.q_hi, -kappa * dnh / st.q_hi))
    return float(lin + pen)


def res_pbm(P: MultiVTS, ev: pbm.Eval) -> float:
    """Eq. (3.15) on the stacked problem: ||res_1|| / ||F|| over all cases."""
    return (np.linalg.norm(ev.g1) / np.linalg.norm(P.F) + abs(ev.g2) / P.V
            + np.linalg.norm(ev.g3) / (np.linalg.norm(P.rho_lo) + np.linalg.norm(P.rho_hi)))


def force_matrix(P: MultiVTS, ev: pbm.Eval) -> sp.csr_matrix:
    """B = (B_1; ...; B_k): (k n) x m, column i the stacked free entries of b_i."""
    return sp.vstack([fe.element_force_matrix(P.grid, ev.be[l]) for l in range(P.k)]).tocsr()


def schur_matrix(P: MultiVTS, ev: pbm.Eval) -> sp.csr_matrix:
    """S of eq. (3.12) on (stacked free U, alpha)."""
    w, _, _ = pbm.schur_weights(ev)
    K1 = fe.assemble_K_free(P.grid, P.Ke, ev.rho1)
    B = force_matrix(P, ev)
    Suu = (sp.kron(sp.identity(P.k), K1) + B @ sp.diags(w) @ B.T).tocsr()
    c = -(B @ w)
    return sp.bmat([[Suu, sp.csr_matrix(c[:, None])],
                    [sp.csr_matrix(c[None, :]), sp.csr_matrix([[w.sum()]])]], format="csr")


def reduced_rhs(P: MultiVTS, ev: pbm.Eval) -> np.ndarray:
    """rhs of eq. (3.13): [(-res1_l + B_l z)_l; -res2 - sum z]."""
    _, z, _ = pbm.schur_weights(ev)
    parts = []
    for l in range(P.k):
        Bz = fe.scatter(P.grid, z[:, None] * ev.be[l])
        parts.append((-ev.g1[l] + Bz)[P.free])
    return np.concatenate(parts + [[-ev.g2 - z.sum()]])


def schur_apply(P: MultiVTS, ev: pbm.Eval, X: np.ndarray, beta: float):
    """S [X; beta] for X in the all-DOF layout (k, n_dof), without assembly:
    per case K(rho') x_l + scatter(w t b_{i,l}), t_i = sum_l b_{i,l}^T x_l - beta;
    returns the (k, n_dof) part (zero at fixed DOFs) and the alpha entry."""
    g = P.grid
    w, _, _ = pbm.schur_weights(ev)
    t = tau(P, ev, X, beta)
    Y = np.stack([g.mask(fe.apply_K(g, P.Ke, ev.rho1, X[l])
                         + fe.scatter(g, (w * t)[:, None] * ev.be[l])) for l in range(P.k)])
    return Y, float(-(w * t).sum())


def duality_gap(P: MultiVTS, st: pbm.State, e: Optional[np.ndarray] = None) -> float:
    """delta(U, alpha) of eq. (2.6) with F^T U."""
    if e is None:
        e = energies(P, st.u)
    a = st.alpha - e
    return float(-0.5 * np.sum(P.F * st.u) + st.alpha * P.V
                 - np.sum(np.minimum(P.rho_lo * a, P.rho_hi * a)))


def dual_objective(P: MultiVTS, st: pbm.State) -> float:
    """Objective of problem (2.1) with F^T U."""
    return float(st.alpha * P.V - np.sum(P.F * st.u) - P.rho_lo @ st.nu_lo
                 + P.rho_hi @ st.nu_hi)


# ----------------------------------------------------------------------------
# result checks (problem (1.1) on the stacked displacement)
# ----------------------------------------------------------------------------
def solve_states(P: MultiVTS, rho: np.ndarray) -> np.ndarray:
    """U = (K(rho)^{-1} f_l)_l on the free DOFs (sparse direct)."""
    K = fe.assemble_K_free(P.grid, P.Ke, rho).tocsc()
    lu = spla.splu(K)
    U = np.zeros((P.k, P.grid.n_dof))
    for l in range(P.k):
        U[l, P.free] = lu.solve(P.F[l, P.free])
    return U


def compliance(P: MultiVTS, rho: np.ndarray) -> float:
    """sum_l 1/2 f_l^T K(rho)^{-1} f_l."""
    return 0.5 * float(np.sum(P.F * solve_states(P, rho)))


def dual_lower_bound(P: MultiVTS, U: np.ndarray) -> float:
    """max over alpha of the unconstrained dual of eq. (2.5) on the stacked
    problem, q(U, alpha) = F^T U - alpha V + sum_i min(lo_i d_i, hi_i d_i)
    with d_i = alpha - e_i(U).  q is concave and piecewise linear in alpha
    with breakpoints e_i, so its maximum is attained at one of them; with the
    energies sorted, the elements below a breakpoint take lo, the rest hi."""
    e = energies(P, U)
    FU = float(np.sum(P.F * U))
    order = np.argsort(e)
    es, lo, hi = e[order], P.rho_lo[order], P.rho_hi[order]
    c_lo = np.concatenate([[0.0], np.cumsum(lo)])
    c_loe = np.concatenate([[0.0], np.cumsum(lo * es)])
    c_hi = np.concatenate([np.cumsum(hi[::-1])[::-1], [0.0]])
    c_hie = np.concatenate([np.cumsum((hi * es)[::-1])[::-1], [0.0]])
    j = np.arange(es.size)
    val = FU - es * P.V + es * c_lo[j] - c_loe[j] + es * c_hi[j] - c_hie[j]
    return float(np.max(val))


def kkt_residual(P: MultiVTS, rho: np.ndarray, U: np.ndarray, lam: float) -> dict:
    """The four terms of the single-load KKT residual on the stacked problem:
    equilibrium of every case relative to ||F||, volume, box, stationarity
    with the summed energies."""
    r = np.stack([fe.apply_K(P.grid, P.Ke, rho, U[l]) - P.F[l] for l in range(P.k)])
    r_eq = float(np.linalg.norm(r) / np.linalg.norm(P.F))
    r_vol = float(abs(rho.sum() - P.V) / P.V)
    r_box = float(max(0.0, np.max(P.rho_lo - rho), np.max(rho - P.rho_hi)) / np.max(P.rho_hi))
    e = energies(P, U)
    proj = np.clip(rho + (e - lam) / lam, P.rho_lo, P.rho_hi)
    r_stat = float(np.max(np.abs(rho - proj) / P.rho_hi))
    return dict(r_eq=r_eq, r_vol=r_vol, r_box=r_box, r_stat=r_stat,
                kkt=max(r_eq, r_vol, r_box, r_stat))


class Solver(pbm.Solver):
    """Algorithms 1 and 2 of the single-load solver on the stacked problem."""

    problem_class = MultiVTS
    evaluate = staticmethod(evaluate)
    schur_matrix = staticmethod(schur_matrix)
    reduced_rhs = staticmethod(reduced_rhs)
    lagrangian_change = staticmethod(lagrangian_change)
    res_pbm = staticmethod(res_pbm)
    duality_gap = staticmethod(duality_gap)
    dual_objective = staticmethod(dual_objective)

    def __init__(self, problem, opts: Optional[pbm.Options] = None, linsolve=None):
        super().__init__(problem, opts, linsolve)
        if self.opts.eps_mr0 is None:
            # the rule of Section 6.2 with n the number of unknowns of the system
            import math
            self.eps_mr = 1e-4 * math.sqrt(self.P.k * self.P.n)

    def hierarchy(self, S):
        return self.mg.Hierarchy(self.P.grid, S, self.levels_count, nload=self.P.k)

    def initial(self) -> pbm.State:
        return initial_state(self.P)

    def split(self, dy):
        P = self.P
        dU = np.zeros((P.k, P.grid.n_dof))
        for l in range(P.k):
            dU[l, P.free] = dy[l * P.n:(l + 1) * P.n]
        return dU, float(dy[-1])

    def tau(self, ev, du, da):
        return tau(self.P, ev, du, da)

    def slope(self, ev, du, da, dnl, dnh):
        return float(np.sum(ev.g1 * du) + ev.g2 * da + ev.g3 @ dnl + ev.g4 @ dnh)

    def final_checks(self, st):
        P, o = self.P, self.opts
        if o.final_state_solve and np.min(P.rho_lo) > 0:
            st.u = solve_states(P, st.rho)
        return kkt_residual(P, st.rho, st.u, st.alpha)
