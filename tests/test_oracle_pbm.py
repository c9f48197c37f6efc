"""Pins of the oracle's penalty function, augmented-Lagrangian derivatives
and Schur reduction (Section 3) -- finite differences and dense solves."""
import numpy as np
import pytest

import workloads as W
from oracle import pbm, fe
from oracle.penalty import phi, dphi, d2phi


# ---------------------------------------------------------------- phi, eq. (3.8)
def test_phi_axioms():
    assert phi(0.0) == 0.0                    # (phi 1)
    assert dphi(0.0) == 1.0                   # (phi 2)
    assert dphi(1e6) > 1e5                    # (phi 3), b = +inf
    assert 0 < dphi(-1e9) < 1e-9              # (phi 4)
    t = np.linspace(-50, 20, 20001)
    assert np.all(np.diff(phi(t)) > 0)        # strictly increasing
    assert np.all(d2phi(t) > 0)               # strictly convex


def test_phi_is_C2_at_tau_hat():
    th = -0.5
    for f in (phi, dphi, d2phi):
        assert abs(f(th) - f(th - 1e-12)) < 1e-10
    assert np.isclose(phi(th), -3.0 / 8.0)
    assert np.isclose(dphi(th), 0.5)
    assert np.isclose(d2phi(th), 1.0)


def test_phi_derivatives_by_finite_differences():
    t = np.array([-40.0, -3.0, -0.7, -0.51, -0.49, 0.0, 0.3, 5.0])
    h = 1e-6
    assert np.allclose((phi(t + h) - phi(t - h)) / (2 * h), dphi(t), rtol=1e-7)
    assert np.allclose((dphi(t + h) - dphi(t - h)) / (2 * h), d2phi(t), rtol=1e-6)
    # the log branch with t_hat = -1/2: phi = -1/4 log(-2t) - 3/8
    tl = np.array([-7.0, -1.0, -0.6])
    assert np.allclose(phi(tl), -0.25 * np.log(-2 * tl) - 0.375, rtol=1e-15)


def test_phi_diff_matches_plain_difference_and_first_order():
    from oracle.penalty import phi_diff
    t = np.array([-40.0, -3.0, -0.7, -0.51, -0.49, -0.3, 0.0, 0.3, 5.0])
    for dt in (0.4, -0.2, 1e-3, -1e-3):
        assert np.allclose(phi_diff(t, dt), phi(t + dt) - phi(t), rtol=1e-12, atol=1e-15)
    # tiny steps on each branch: the change is phi'(t) dt to second order
    dt = 1e-12
    assert np.allclose(phi_diff(t, dt), dphi(t) * dt, rtol=1e-9, atol=0)


# ------------------------------------------------------------- helpers
def _tiny(rho_lo=1e-3, seed=0):
    pr = W.cantilever_edge(2, 1, 1, 1, vol_frac=0.4, rho_lo=rho_lo)
    P = pbm.VTS(pr)
    rng = np.random.default_rng(seed)
    m = P.grid.m
    st = pbm.State(u=P.grid.mask(0.3 * rng.standard_normal(P.grid.n_dof)),
                   alpha=0.2 + 0.1 * rng.random(),
                   nu_lo=0.2 * rng.random(m), nu_hi=0.2 * rng.random(m),
                   rho=rng.uniform(0.2, 0.8, m), mu_lo=rng.uniform(0.5, 1.5, m),
                   mu_hi=rng.uniform(0.5, 1.5, m), p=rng.uniform(0.2, 1.0, m),
                   q_lo=rng.uniform(0.2, 1.0, m), q_hi=rng.uniform(0.2, 1.0, m))
    return P, st


def _pack(P, st):
    return np.concatenate([st.u[P.free], [st.alpha], st.nu_lo, st.nu_hi])


def _unpack(P, st, x):
    n, m = P.n, P.grid.m
    s2 = st.copy()
    s2.u = np.zeros(P.grid.n_dof)
    s2.u[P.free] = x[:n]
    s2.alpha = x[n]
    s2.nu_lo = x[n + 1:n + 1 + m]
    s2.nu_hi = x[n + 1 + m:]
    return s2


def _L(P, st, x):
    return pbm.lagrangian(P, _unpack(P, st, x))


# ------------------------------------------------- gradient eq. (3.10)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_finite_differences(seed):
    P, st = _tiny(seed=seed)
    x0 = _pack(P, st)
    g = pbm.full_gradient(P, pbm.evaluate(P, st))
    h = 1e-6
    fd = np.array([(_L(P, st, x0 + h * e) - _L(P, st, x0 - h * e)) / (2 * h)
                   for e in np.eye(x0.size)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_res3_constant_sign():
    # with rho_lo large the printed "+rho_lo" would be off by 2 rho_lo
    P, st = _tiny(rho_lo=0.05)
    ev = pbm.evaluate(P, st)
    x0 = _pack(P, st)
    n, m, h = P.n, P.grid.m, 1e-6
    i = n + 1                                   # d/d nu_lo_0
    e = np.zeros_like(x0); e[i] = 1.0
    fd = (_L(P, st, x0 + h * e) - _L(P, st, x0 - h * e)) / (2 * h)
    assert abs(ev.g3[0] - fd) < 1e-6
    assert abs((ev.g3[0] + 2 * P.rho_lo[0]) - fd) > 0.09


# ------------------------------------------------- Hessian eq. (3.11)
@pytest.mark.parametrize("seed", [0, 3])
def test_hessian_matches_finite_differences(seed):
    P, st = _tiny(seed=seed)
    x0 = _pack(P, st)
    H = pbm.full_hessian(P, pbm.evaluate(P, st))
    h = 1e-5
    cols = []
    for e in np.eye(x0.size):
        gp = pbm.full_gradient(P, pbm.evaluate(P, _unpack(P, st, x0 + h * e)))
        gm = pbm.full_gradient(P, pbm.evaluate(P, _unpack(P, st, x0 - h * e)))
        cols.append((gp - gm) / (2 * h))
    Hfd = np.array(cols).T
    assert np.allclose(H, Hfd, rtol=1e-5, atol=1e-6)
    assert np.min(np.linalg.eigvalsh(H)) > -1e-10          # convexity


# ------------------------------------------- Schur reduction eqs. (3.12)-(3.14)
@pytest.mark.parametrize("seed", [0, 4, 5])
def test_reduced_system_equals_full_newton_solve(seed):
    P, st = _tiny(seed=seed)
    ev = pbm.evaluate(P, st)
    H = pbm.full_hessian(P, ev)
    g = pbm.full_gradient(P, ev)
    full = np.linalg.solve(H, -g)
    S = pbm.schur_matrix(P, ev).toarray()
    rhs = pbm.reduced_rhs(P, ev)
    y = np.linalg.solve(S, rhs)
    n, m = P.n, P.grid.m
    assert np.allclose(y, full[:n + 1], rtol=1e-10, atol=1e-12)
    du = np.zeros(P.grid.n_dof); du[P.free] = y[:n]
    tau = np.einsum("ei,ei->e", ev.be, du[P.grid.dofs]) - y[n]
    dnl, dnh = pbm.delta_nu(ev, tau)
    assert np.allclose(dnl, full[n + 1:n + 1 + m], rtol=1e-10, atol=1e-12)
    assert np.allclose(dnh, full[n + 1 + m:], rtol=1e-10, atol=1e-12)


def test_schur_closed_form_equals_literal_block_formula():
    P, st = _tiny(seed=6)
    ev = pbm.evaluate(P, st)
    S = pbm.schur_matrix(P, ev).toarray()
    Sl = pbm.schur_literal(P, ev)
    assert np.allclose(S, Sl, rtol=1e-11, atol=1e-12)
    assert np.allclose(S, S.T, atol=1e-13)
    assert np.min(np.linalg.eigvalsh(S)) > 0
    # principal block has the (node-block) sparsity of sum K_i: a nonzero
    # couples two DOFs whose nodes share an element
    g = P.grid
    adj = np.zeros((g.n_dof, g.n_dof), dtype=bool)
    for e in range(g.m):
        adj[np.ix_(g.dofs[e], g.dofs[e])] = True
    adj = adj[np.ix_(g.free, g.free)]
    assert np.all((np.abs(S[:-1, :-1]) > 0) <= adj)
    assert np.all(np.abs(S[-1, :-1]) > 0)          # alpha row full here


def test_schur_apply_matches_matrix():
    P, st = _tiny(seed=7)
    ev = pbm.evaluate(P, st)
    S = pbm.schur_matrix(P, ev)
    x = np.random.default_rng(1).standard_normal(P.n + 1)
    yu, ya = pbm.schur_apply(P, ev, x[:-1], x[-1])
    y = S @ x
    assert np.allclose(yu, y[:-1], rtol=1e-12, atol=1e-12)
    assert np.isclose(ya, y[-1], rtol=1e-12, atol=1e-12)


def test_schur_weight_is_harmonic_combination():
    P, st = _tiny(seed=8)
    ev = pbm.evaluate(P, st)
    w, z, det = pbm.schur_weights(ev)
    assert np.allclose(w, 1.0 / (1.0 / ev.rho2 + 1.0 / ev.mu_lo2 + 1.0 / ev.mu_hi2), rtol=1e-14)


def test_lagrangian_change_matches_difference():
    # the change along the Newton ray (Armijo rule of Algorithm 2) equals the
    # literal difference of eq. (3.9) at the two points
    P, st = _tiny(seed=9)
    ev = pbm.evaluate(P, st)
    rng = np.random.default_rng(2)
    du = P.grid.mask(rng.standard_normal(P.grid.n_dof))
    da = 0.3
    dnl = 0.1 * rng.standard_normal(P.grid.m)
    dnh = 0.1 * rng.standard_normal(P.grid.m)
    for kappa in (1.0, 0.25, 0.01):
        new = st.copy()
        new.u = st.u + kappa * du
        new.alpha += kappa * da
        new.nu_lo = st.nu_lo + kappa * dnl
        new.nu_hi = st.nu_hi + kappa * dnh
        d = pbm.lagrangian_change(P, st, ev, du, da, dnl, dnh, kappa)
        assert np.isclose(d, pbm.lagrangian(P, new) - pbm.lagrangian(P, st), rtol=1e-9, atol=1e-12)


def test_lagrangian_change_is_exact_where_totals_cancel():
    # a tiny step: the change along the ray keeps the first-order term
    # kappa * grad L^T dxi (eq. (3.10)) to near machine precision, while the
    # difference of the two totals of eq. (3.9) loses most of its digits
    P, st = _tiny(seed=9)
    ev = pbm.evaluate(P, st)
    rng = np.random.default_rng(3)
    du = P.grid.mask(rng.standard_normal(P.grid.n_dof))
    da = 0.2
    dnl = 0.1 * rng.standard_normal(P.grid.m)
    dnh = 0.1 * rng.standard_normal(P.grid.m)
    slope = float(ev.g1 @ du + ev.g2 * da + ev.g3 @ dnl + ev.g4 @ dnh)
    kappa = 1e-11
    d = pbm.lagrangian_change(P, st, ev, du, da, dnl, dnh, kappa)
    assert abs(d - kappa * slope) <= 1e-7 * abs(kappa * slope)
    new = st.copy()
    new.u = st.u + kappa * du
    new.alpha += kappa * da
    new.nu_lo = st.nu_lo + kappa * dnl
    new.nu_hi = st.nu_hi + kappa * dnh
    lit = pbm.lagrangian(P, new) - pbm.lagrangian(P, st)
    assert abs(lit - kappa * slope) > 10 * abs(d - kappa * slope)


# --------------------------------------------------------- gap (2.6)
def test_gap_vanishes_only_at_optimum_and_is_nonnegative_when_feasible():
    # for the exact state u(rho) of any feasible rho, delta >= 0 for alpha maximizing (2.5)
    from oracle import kkt
    pr = W.cantilever_edge(4, 2, 2, 2, vol_frac=0.3)
    P = pbm.VTS(pr)
    rho = np.full(P.grid.m, P.V / P.grid.m)
    u = kkt.solve_state(P.grid, P.Ke, rho, P.f)
    lb, a = kkt.dual_lower_bound(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, u)
    st = pbm.initial_state(P.grid.n_dof, P.grid.m, P.V)
    st.u, st.alpha = u, a
    delta = pbm.duality_gap(P, st)
    assert delta >= -1e-12
    assert np.isclose(delta, 0.5 * P.f @ u - lb, rtol=1e-12)
