"""Pins of the multi-load oracle (oracle/multiload.py) against what the
mathematics fixes, independent of its own formulas:
  * one load case: the single-load oracle (Section 3.2, Algorithms 1-2);
  * cases (f, c f): the single-load problem with load sqrt(1 + c^2) f, whose
    iterates are the multi-load ones mapped by x -> (x, c x) / sqrt(1 + c^2)
    (the map commutes with S, the node-block smoother and the prolongation);
  * a zero second case: the single-load problem;
  * the gradient (res_1..res_4) and the Newton system (3.12)-(3.13) against
    central differences of the augmented Lagrangian (3.9) written from its
    definition, the system as the literal Schur complement of the
    difference Hessian;
  * the optimal compliance of a tiny two-case problem against a general
    constrained minimiser of the primal, with the adjoint gradient written
    from the single-load finite-element pieces, and weak duality (Theorem 2).
"""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import workloads as W
from oracle import fe, kkt, mg, pbm
from oracle import multiload as ML


def _two_loads(nx=8, ny=4, nz=4, levels=3, vol_frac=0.3):
    return W.cantilever_two_loads(nx, ny, nz, levels, vol_frac=vol_frac)


def _state(P, seed, k):
    rng = np.random.default_rng(seed)
    m = P.grid.m
    st = ML.initial_state(P)
    st.u = np.stack([P.grid.mask(0.3 * rng.standard_normal(P.grid.n_dof)) for _ in range(k)])
    st.alpha = 0.4
    st.nu_lo = 0.05 * rng.random(m)
    st.nu_hi = 0.05 * rng.random(m)
    st.rho = rng.uniform(0.1, 1.0, m)
    st.mu_lo = rng.uniform(0.5, 1.5, m)
    st.mu_hi = rng.uniform(0.5, 1.5, m)
    st.p = rng.uniform(0.5, 1.5, m)
    st.q_lo = rng.uniform(0.5, 1.5, m)
    st.q_hi = rng.uniform(0.5, 1.5, m)
    return st


def test_one_case_is_the_single_load_problem():
    pr = W.cantilever_edge(8, 4, 4, 3)
    Ps, Pm = pbm.VTS(pr), ML.MultiVTS(pr)
    st = _state(Pm, 3, 1)
    ss = st.copy()
    ss.u = st.u[0].copy()
    es, em = pbm.evaluate(Ps, ss), ML.evaluate(Pm, st)
    assert np.allclose(em.e, es.e, rtol=1e-14, atol=0)
    assert np.allclose(em.g1[0], es.g1, rtol=1e-13, atol=1e-14)
    Sd = (ML.schur_matrix(Pm, em) - pbm.schur_matrix(Ps, es)).toarray()
    assert np.max(np.abs(Sd)) < 1e-12 * abs(pbm.schur_matrix(Ps, es)).max()
    assert np.allclose(ML.reduced_rhs(Pm, em), pbm.reduced_rhs(Ps, es), rtol=1e-12, atol=1e-14)
    assert ML.res_pbm(Pm, em) == pytest.approx(pbm.res_pbm(Ps, es), rel=1e-13)
    assert ML.duality_gap(Pm, st) == pytest.approx(pbm.duality_gap(Ps, ss), rel=1e-13)
    # the whole solve
    a, b = pbm.Solver(pr), ML.Solver(pr)
    sa, sb = a.solve(), b.solve()
    assert a.status == b.status == "ok"
    assert len(a.log.outer) == len(b.log.outer)
    assert len(a.log.newton) == len(b.log.newton)
    assert np.max(np.abs(sa.rho - sb.rho)) < 1e-8
    assert b.kkt["kkt"] < 1e-6


@pytest.mark.parametrize("c", [0.5, 2.0])
def test_proportional_cases_are_one_scaled_load(c):
    """Cases (f, c f): the same density as the single load sqrt(1 + c^2) f,
    the same multiplier alpha and iteration counts, and the summed compliance
    of the cases equals that load's compliance."""
    base = W.cantilever_edge(8, 4, 4, 3)
    s = math.sqrt(1.0 + c * c)
    single = W.with_load_cases(base, [s * base.f], name="scaled")
    single.extra.pop("load_cases")
    single.f = s * base.f
    multi = W.with_load_cases(base, [base.f, c * base.f])
    eps0 = 1e-4 * math.sqrt(pbm.VTS(base).n)
    a = pbm.Solver(single, pbm.Options(eps_mr0=eps0))
    b = ML.Solver(multi, pbm.Options(eps_mr0=eps0))
    sa, sb = a.solve(), b.solve()
    assert a.status == b.status == "ok"
    assert len(a.log.outer) == len(b.log.outer)
    assert len(a.log.newton) == len(b.log.newton)
    mr_a = sum(x["minres"] for x in a.log.newton)
    mr_b = sum(x["minres"] for x in b.log.newton)
    assert abs(mr_a - mr_b) <= 0.02 * mr_a + 2
    assert np.max(np.abs(sa.rho - sb.rho)) < 1e-7
    assert sb.alpha == pytest.approx(sa.alpha, rel=1e-8)
    # the iterate lies on the image of the map: u_2 = c u_1, u_1 = u / s
    assert np.allclose(sb.u[1], c * sb.u[0], rtol=0, atol=1e-8 * np.abs(sb.u).max())
    assert np.allclose(sb.u[0], sa.u / s, rtol=0, atol=1e-7 * np.abs(sa.u).max())
    Pm = ML.MultiVTS(multi)
    assert ML.compliance(Pm, sb.rho) == pytest.approx(
        kkt.compliance(Pm.grid, Pm.Ke, sb.rho, s * Pm.F[0]), rel=1e-10)


def test_zero_second_case_changes_nothing():
    base = W.cantilever_edge(8, 4, 4, 3)
    multi = W.with_load_cases(base, [base.f, np.zeros_like(base.f)])
    eps0 = 1e-4 * math.sqrt(pbm.VTS(base).n)
    a = pbm.Solver(base, pbm.Options(eps_mr0=eps0))
    b = ML.Solver(multi, pbm.Options(eps_mr0=eps0))
    sa, sb = a.solve(), b.solve()
    assert len(a.log.outer) == len(b.log.outer)
    assert len(a.log.newton) == len(b.log.newton)
    assert np.max(np.abs(sa.rho - sb.rho)) < 1e-8
    assert np.max(np.abs(sb.u[1])) == 0.0


def _unknowns(P, st):
    """(stacked free U, alpha, nu_lo, nu_hi) as one vector."""
    return np.concatenate([st.u[l, P.free] for l in range(P.k)]
                          + [[st.alpha], st.nu_lo, st.nu_hi])


def _with(P, st, x):
    out = st.copy()
    n, m = P.n, P.grid.m
    out.u = np.zeros_like(st.u)
    for l in range(P.k):
        out.u[l, P.free] = x[l * n:(l + 1) * n]
    out.alpha = x[P.k * n]
    out.nu_lo = x[P.k * n + 1:P.k * n + 1 + m].copy()
    out.nu_hi = x[P.k * n + 1 + m:].copy()
    return out


def test_gradient_and_schur_system_against_differences_of_the_lagrangian():
    pr = W.cantilever_two_loads(2, 1, 1, 1)
    P = ML.MultiVTS(pr)
    st = _state(P, 11, P.k)
    x0 = _unknowns(P, st)
    N = x0.size

    def L(x):
        return ML.lagrangian(P, _with(P, st, x))

    h = 1e-5
    grad_fd = np.array([(L(x0 + h * ei) - L(x0 - h * ei)) / (2 * h) for ei in np.eye(N)])
    ev = ML.evaluate(P, st)
    grad = np.concatenate([ev.g1[l, P.free] for l in range(P.k)] + [[ev.g2], ev.g3, ev.g4])
    assert np.allclose(grad, grad_fd, rtol=1e-7, atol=1e-8 * np.abs(grad).max())

    def G(x):
        e = ML.evaluate(P, _with(P, st, x))
        return np.concatenate([e.g1[l, P.free] for l in range(P.k)] + [[e.g2], e.g3, e.g4])

    H = np.array([(G(x0 + h * ei) - G(x0 - h * ei)) / (2 * h) for ei in np.eye(N)]).T
    H = 0.5 * (H + H.T)
    k = P.k * P.n + 1
    Hyy, Hyn, Hnn = H[:k, :k], H[:k, k:], H[k:, k:]
    S_lit = Hyy - Hyn @ np.linalg.solve(Hnn, Hyn.T)
    S = ML.schur_matrix(P, ev).toarray()
    assert np.max(np.abs(S - S_lit)) < 1e-6 * np.max(np.abs(S))
    rhs_lit = -grad[:k] + Hyn @ np.linalg.solve(Hnn, grad[k:])
    rhs = ML.reduced_rhs(P, ev)
    assert np.max(np.abs(rhs - rhs_lit)) < 1e-6 * np.max(np.abs(rhs))
    # and S without assembly
    X = np.stack([P.grid.mask(np.random.default_rng(5).standard_normal(P.grid.n_dof))
                  for _ in range(P.k)])
    Y, ya = ML.schur_apply(P, ev, X, 0.7)
    xs = np.concatenate([X[l, P.free] for l in range(P.k)] + [[0.7]])
    ys = S @ xs
    assert np.allclose(np.concatenate([Y[l, P.free] for l in range(P.k)] + [[ya]]), ys,
                       rtol=1e-12, atol=1e-12 * np.abs(ys).max())


def _primal_optimum(pr):
    """min_rho sum_l 1/2 f_l^T K(rho)^{-1} f_l over the volume and box
    constraints by SLSQP, with the adjoint gradient -sum_l e_i(u_l)."""
    g = fe.Grid(pr.nx, pr.ny, pr.nz, pr.fixed)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    F = [g.mask(f) for f in W.load_cases(pr)]
    m = g.m

    def fun(r):
        us = [kkt.solve_state(g, Ke, r, f) for f in F]
        c = sum(0.5 * float(f @ u) for f, u in zip(F, us))
        grad = -sum(fe.element_energies(g, Ke, u) for u in us)
        return c, grad

    r0 = np.full(m, pr.V / m)
    res = so.minimize(fun, r0, jac=True, method="SLSQP",
                      bounds=[(pr.rho_lo, pr.rho_hi)] * m,
                      constraints=[dict(type="eq", fun=lambda r: r.sum() - pr.V,
                                        jac=lambda r: np.ones(m))],
                      options=dict(ftol=1e-14, maxiter=2000))
    assert res.success, res.message
    return float(res.fun), res.x


def test_two_case_optimum_against_a_general_minimiser():
    pr = W.cantilever_two_loads(4, 2, 2, 2, vol_frac=0.4, rho_lo=1e-2)
    c_star, r_star = _primal_optimum(pr)
    sol = ML.Solver(pr)
    st = sol.solve()
    assert sol.status == "ok" and sol.kkt["kkt"] < 1e-6
    P = sol.P
    c_pbm = ML.compliance(P, st.rho)
    assert c_pbm == pytest.approx(c_star, rel=1e-6)
    lb = ML.dual_lower_bound(P, st.u)
    assert lb <= c_star * (1 + 1e-9) and lb == pytest.approx(c_star, rel=1e-6)
    # the two-case design is not either case's own optimum
    for l in range(2):
        one = W.with_load_cases(pr, [W.load_cases(pr)[l]])
        s1 = pbm.Solver(one).solve()
        assert ML.compliance(P, s1.rho) > c_star * 1.01


def test_multiload_vcycle_is_symmetric_positive_and_exact_on_one_level():
    pr = _two_loads()
    P = ML.MultiVTS(pr)
    st = _state(P, 21, P.k)
    ev = ML.evaluate(P, st)
    S = ML.schur_matrix(P, ev)
    H = mg.Hierarchy(P.grid, S, 3, nload=P.k)
    rng = np.random.default_rng(0)
    v, w = rng.standard_normal(S.shape[0]), rng.standard_normal(S.shape[0])
    Mv, Mw = H.vcycle(v), H.vcycle(w)
    assert w @ Mv == pytest.approx(v @ Mw, rel=1e-10)
    assert v @ Mv > 0 and w @ Mw > 0
    H1 = mg.Hierarchy(P.grid, S, 1, nload=P.k)
    assert np.allclose(S @ H1.vcycle(v), v, rtol=0, atol=1e-9 * np.abs(v).max())
    # the node blocks hold all cases of a node: a block sweep with the rank-one
    # coupling of the cases solves a system of one node exactly
    assert H.levels[-1].colors[0][1].shape[1:] == (6, 6)


def test_multiload_vcycle_contracts_and_colours_decouple():
    """The V-cycle with node blocks over all cases, used as an iteration
    z <- z + M^{-1}(r - S z), contracts the error (spectral radius of
    I - M^{-1} S below 1, by power iteration); and within one parity colour
    the stacked S couples no two distinct nodes, so the colour-wise block
    Gauss-Seidel of oracle/mg.py updates each node block exactly."""
    pr = _two_loads()
    P = ML.MultiVTS(pr)
    st = _state(P, 23, P.k)
    ev = ML.evaluate(P, st)
    S = ML.schur_matrix(P, ev).tocsr()
    H = mg.Hierarchy(P.grid, S, 2, nload=P.k)
    e = np.random.default_rng(3).standard_normal(S.shape[0])
    rate = 1.0
    for _ in range(30):
        e2 = e - H.vcycle(S @ e)
        rate = np.linalg.norm(e2) / np.linalg.norm(e)
        e = e2 / np.linalg.norm(e2)
    assert rate < 0.9
    # colour decoupling on the finest level
    lev = H.levels[-1]
    for comp, _ in lev.colors:
        idx = comp[comp >= 0]
        node_of = np.repeat(np.arange(comp.shape[0]), comp.shape[1])[(comp >= 0).ravel()]
        sub = S[idx][:, idx].tocoo()
        assert np.all(node_of[sub.row] == node_of[sub.col])
