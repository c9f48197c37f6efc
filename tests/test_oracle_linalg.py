"""Pins of the oracle's multigrid and MINRES (Section 6)."""
import numpy as np
import scipy.sparse as sp
import pytest

import workloads as W
from oracle import pbm, fe, mg, minres


def _system(nx=8, ny=4, nz=4, L=3, seed=0, kind="cant"):
    pr = (W.cantilever_edge if kind == "cant" else W.bridge_top)(nx, ny, nz, L)
    P = pbm.VTS(pr)
    rng = np.random.default_rng(seed)
    m = P.grid.m
    st = pbm.initial_state(P.grid.n_dof, m, P.V)
    st.u = P.grid.mask(0.5 * rng.standard_normal(P.grid.n_dof))
    st.rho = rng.uniform(0.05, 1.0, m)
    st.p = np.full(m, 0.1)
    st.q_lo = np.full(m, 0.1)
    st.q_hi = np.full(m, 0.1)
    ev = pbm.evaluate(P, st)
    return P, ev, pbm.schur_matrix(P, ev), L


@pytest.mark.parametrize("kind", ["cant", "bridge"])
def test_vcycle_symmetric_positive(kind):
    P, ev, S, L = _system(kind=kind)
    h = mg.Hierarchy(P.grid, S, L)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, S.shape[0]))
    Mx, My = h.vcycle(x), h.vcycle(y)
    assert abs(x @ My - y @ Mx) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(My)
    for _ in range(5):
        v = rng.standard_normal(S.shape[0])
        assert v @ h.vcycle(v) > 0


def test_galerkin_hierarchy_alpha_identity():
    P, ev, S, L = _system()
    h = mg.Hierarchy(P.grid, S, L)
    for k in range(1, L):
        Pk = h.P[k].toarray()
        assert Pk[-1, -1] == 1.0 and np.all(Pk[-1, :-1] == 0) and np.all(Pk[:-1, -1] == 0)
        # alpha diagonal equal on every level
        assert np.isclose(h.levels[k - 1].S[-1, -1], S[-1, -1], rtol=1e-14)


def test_same_colour_nodes_do_not_couple():
    P, ev, S, L = _system()
    h = mg.Hierarchy(P.grid, S, L)
    for lev in h.levels[1:]:
        A = lev.S.tocsr()
        for comp, _ in lev.colors:
            idx = comp[comp >= 0]
            sub = A[idx][:, idx].toarray()
            own = np.zeros_like(sub, dtype=bool)
            for r in comp:                     # blocks of one node may couple
                ii = [np.nonzero(idx == c)[0][0] for c in r if c >= 0]
                own[np.ix_(ii, ii)] = True
            assert np.all(sub[~own] == 0)


def test_two_level_cycle_contracts_and_gs_converges():
    P, ev, S, _ = _system(L=2)
    h = mg.Hierarchy(P.grid, S, 2)
    b = np.random.default_rng(2).standard_normal(S.shape[0])
    x = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    for _ in range(30):
        x = x + h.vcycle(b - S @ x)
    assert np.linalg.norm(b - S @ x) < 0.1 * r0          # contraction < 1
    # Gauss-Seidel on an SPD matrix decreases the S-norm of the error at
    # every sweep (forward and backward alike)
    lev = h.levels[1]
    Sd = S.toarray()
    xs = np.linalg.solve(Sd, b)
    z = np.zeros_like(b)
    prev = np.sqrt(xs @ Sd @ xs)
    for _ in range(10):
        for sweep in (lev.gs_forward, lev.gs_backward):
            sweep(b, z)
            err = np.sqrt((z - xs) @ Sd @ (z - xs))
            assert err < prev
            prev = err


def test_single_level_is_exact_solve():
    P, ev, S, _ = _system(4, 2, 2, 1)
    h = mg.Hierarchy(P.grid, S, 1)
    b = np.random.default_rng(3).standard_normal(S.shape[0])
    assert np.allclose(S @ h.vcycle(b), b, rtol=1e-10, atol=1e-10)


def _spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1, cond, n)) @ Q.T


def test_minres_equals_dense_solve():
    A = _spd(40, 0)
    M = _spd(40, 1, cond=10)
    Minv = np.linalg.inv(M)
    b = np.random.default_rng(2).standard_normal(40)
    x, its, rel = minres.minres(lambda v: A @ v, b, lambda r: Minv @ r, 1e-14, 200)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)
    assert its < 200


def test_minres_residual_estimate_is_Minv_norm():
    A = _spd(30, 3, cond=50)
    Minv = np.linalg.inv(_spd(30, 4, cond=5))
    b = np.random.default_rng(5).standard_normal(30)
    beta1 = np.sqrt(b @ Minv @ b)
    prev = np.inf
    for k in range(1, 12):
        x, its, rel = minres.minres(lambda v: A @ v, b, lambda r: Minv @ r, 0.0, k)
        r = b - A @ x
        assert np.isclose(np.sqrt(r @ Minv @ r), rel * beta1, rtol=1e-8)
        assert rel <= prev + 1e-15                # monotone
        prev = rel


def test_minres_identity_preconditioner_matches_krylov_optimum():
    # MINRES minimizes ||b - A x|| over the Krylov space K_k(A, b)
    A = _spd(25, 6, cond=100)
    b = np.random.default_rng(7).standard_normal(25)
    k = 6
    Kry = np.array([np.linalg.matrix_power(A, j) @ b for j in range(k)]).T
    Qk, _ = np.linalg.qr(Kry)
    c, *_ = np.linalg.lstsq(A @ Qk, b, rcond=None)
    best = np.linalg.norm(b - A @ Qk @ c)
    x, its, rel = minres.minres(lambda v: A @ v, b, lambda r: r, 0.0, k)
    assert np.isclose(np.linalg.norm(b - A @ x), best, rtol=1e-8)


def test_minres_mg_on_schur_system():
    P, ev, S, L = _system()
    h = mg.Hierarchy(P.grid, S, L)
    b = pbm.reduced_rhs(P, ev)
    x, its, rel = minres.minres(lambda v: S @ v, b, h.vcycle, 1e-10, 300)
    assert np.linalg.norm(S @ x - b) < 1e-8 * np.linalg.norm(b) * 1e2
    assert its < 100
