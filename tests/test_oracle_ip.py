"""Pins of the oracle interior point method (Section 4, Algorithm 3) against
what the mathematics fixes: the Jacobian against finite differences of the
residual, the reduced step against the full Newton step, the PBM optimum as
a zero of the IP residual, and convergence to the certified optimum."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import ip, kkt, pbm


def direct(S, b, eps):
    return spla.spsolve(S.tocsc(), b)


def interior_state(P, seed):
    """A strictly feasible IP point away from the initial one."""
    rng = np.random.default_rng(seed)
    g = P.grid
    u = np.where(g.fixed == 1, 0.0, rng.uniform(-1, 1, g.n_dof))
    rho = rng.uniform(P.rho_lo + 0.05, P.rho_hi - 0.05)
    return ip.IPState(u, 0.3 - rng.uniform(), rho, rng.uniform(0.1, 2.0, g.m),
                      rng.uniform(0.1, 2.0, g.m))


def flat(P, st):
    return np.concatenate([st.u[P.free], [st.alpha], st.rho, st.nu_lo, st.nu_hi])


def unflat(P, st, x):
    n, m = P.n, P.grid.m
    u = np.zeros(P.grid.n_dof)
    u[P.free] = x[:n]
    return ip.IPState(u, float(x[n]), x[n + 1:n + 1 + m].copy(),
                      x[n + 1 + m:n + 1 + 2 * m].copy(), x[n + 1 + 2 * m:].copy())


@pytest.fixture(scope="module")
def tiny():
    return pbm.VTS(W.cantilever_edge(4, 2, 2, 2, vol_frac=0.3))


def test_jacobian_matches_finite_differences(tiny):
    P = tiny
    st = interior_state(P, 1)
    J = ip.jacobian_dense(P, st)
    x0 = flat(P, st)
    h = 1e-6
    rng = np.random.default_rng(2)
    for j in rng.choice(x0.size, 40, replace=False):
        xp, xm = x0.copy(), x0.copy()
        xp[j] += h
        xm[j] -= h
        col = (ip.residual_vector(P, unflat(P, st, xp), 0.01, 0.02)
               - ip.residual_vector(P, unflat(P, st, xm), 0.01, 0.02)) / (2 * h)
        assert np.max(np.abs(col - J[:, j])) <= 1e-6 * (1 + np.max(np.abs(J[:, j]))), j


@pytest.mark.parametrize("seed", [3, 4])
def test_reduced_step_equals_full_newton_step(tiny, seed):
    P = tiny
    st = interior_state(P, seed)
    r, s = 0.03, 0.01
    J = ip.jacobian_dense(P, st)
    d = np.linalg.solve(J, -ip.residual_vector(P, st, r, s))
    full = unflat(P, ip.IPState(np.zeros_like(st.u), 0.0, 0 * st.rho, 0 * st.rho, 0 * st.rho), d)
    R = ip.residual(P, st, r, s)
    S, rhs, _, _ = ip.reduced_system(P, st, R)
    y = np.linalg.solve(S.toarray(), rhs)
    du = np.zeros(P.grid.n_dof)
    du[P.free] = y[:-1]
    drho, dnl, dnh = ip.increments(P, st, R, du, y[-1])
    for a, b in ((du, full.u), (y[-1], full.alpha), (drho, full.rho), (dnl, full.nu_lo),
                 (dnh, full.nu_hi)):
        a, b = np.atleast_1d(a), np.atleast_1d(b)
        assert np.max(np.abs(a - b)) <= 1e-9 * (1 + np.max(np.abs(b)))
    # S is symmetric positive definite at a strictly feasible point
    assert np.linalg.eigvalsh(S.toarray()).min() > 0


def test_pbm_optimum_is_a_zero_of_the_ip_residual(tiny):
    """The KKT point PBM reaches, with alpha_IP = -alpha_PBM and r = s = 0."""
    P = tiny
    sol = pbm.Solver(P.pr)
    st = sol.solve()
    assert sol.status == "ok" and st.alpha > 0
    R = ip.residual(P, ip.IPState(st.u, -st.alpha, st.rho, st.nu_lo, st.nu_hi), 0.0, 0.0)
    assert np.linalg.norm(R.res1) <= 1e-9 * np.linalg.norm(P.f)
    assert abs(R.res2) <= 1e-9 * P.V
    for v in (R.res3, R.res4, R.res5):
        assert np.max(np.abs(v)) <= 1e-9 * st.alpha


def test_exact_solves_reach_the_certified_optimum():
    """With direct linear solves Algorithm 3 converges to the optimum of
    (1.1): KKT residual and duality certificate at the tolerance asked."""
    pr = W.config(0)
    sol = ip.Solver(pr, ip.IPOptions(eps_ip=1e-10), linsolve=direct)
    res = sol.solve()
    assert res.converged
    P, x = sol.P, res.state
    k = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, x.rho, x.u, -x.alpha)
    assert k["kkt"] <= 1e-8
    lb, ub, rel = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, x.rho, x.u)
    assert rel <= 1e-9
    assert lb * (1 - 1e-9) <= 0.5 * P.f @ x.u <= ub * (1 + 1e-9)


def test_barrier_parameters_are_shifted_by_one_iteration():
    pr = W.config(0)
    sol = ip.Solver(pr, linsolve=direct)
    P = sol.P
    st = ip.initial_state(P.grid.n_dof, P.grid.m, P.V)
    states = [st]
    recs = []
    for _ in range(4):
        st, rec = sol.step(st)
        states.append(st)
        recs.append(rec)
    m = P.grid.m
    assert recs[0]["r"] == 1e-2
    for k in range(1, 4):
        # the system of pass k (at iterate k) uses the measure of iterate k-1
        x = states[k - 1]
        assert recs[k]["r"] == pytest.approx(0.2 * x.nu_lo @ (x.rho - P.rho_lo) / m, rel=1e-14)
        assert recs[k]["s"] == pytest.approx(0.2 * x.nu_hi @ (P.rho_hi - x.rho) / m, rel=1e-14)


def test_multigrid_run_stops_at_the_paper_test():
    """With MINRES and the V-cycle at the paper's tolerances the method
    stops at the paper's test with the compliance of the optimum to the
    accuracy that test asks for."""
    pr = W.config(0)
    mgs = ip.Solver(pr)
    res = mgs.solve()
    assert res.converged
    P, x = mgs.P, res.state
    lb, ub, _ = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, x.rho, x.u)
    c = 0.5 * P.f @ x.u
    assert abs(c - ub) <= 1e-5 * ub and lb <= ub
    k = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, x.rho, x.u, -x.alpha)
    assert k["kkt"] <= 1e-3
    last = res.history[-1]
    assert last["ratio"] < 1e-5 and last["res_ip"] < 1e-4


def test_uniform_strain_bar_has_uniform_optimum():
    """A bar under uniform traction on symmetry rollers: every element has
    the same energy at uniform rho, so rho* = V/m (closed form)."""
    pr = W.bar_rollers(4, 2, 2, 2, vol_frac=0.5)
    # every element is interior here, so nu -> 0 and W -> infinity for all of
    # them: 1e-8 is reached, a much tighter eps_ip makes the Newton systems
    # numerically singular
    sol = ip.Solver(pr, ip.IPOptions(eps_ip=1e-8), linsolve=direct)
    res = sol.solve()
    assert res.converged
    P, x = sol.P, res.state
    assert np.max(np.abs(x.rho - P.V / P.grid.m)) <= 1e-6
    c_uni = kkt.compliance(P.grid, P.Ke, np.full(P.grid.m, P.V / P.grid.m), P.f)
    assert abs(0.5 * P.f @ x.u - c_uni) <= 1e-8 * c_uni


def test_load_scaling():
    """f -> s f leaves rho* unchanged and scales the compliance and the
    multiplier by s^2 (alpha_IP = -lambda)."""
    out = []
    for scale in (1.0, 3.0):
        pr = W.config(0)
        pr.f = pr.f * scale
        sol = ip.Solver(pr, ip.IPOptions(eps_ip=1e-10), linsolve=direct)
        res = sol.solve()
        assert res.converged
        out.append((res.state, 0.5 * sol.P.f @ res.state.u))
    (a, ca), (b, cb) = out
    assert np.max(np.abs(a.rho - b.rho)) <= 1e-6
    assert abs(cb - 9.0 * ca) <= 1e-8 * cb
    assert abs(b.alpha - 9.0 * a.alpha) <= 1e-6 * abs(b.alpha)
