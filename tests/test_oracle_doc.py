"""Pins of the DOC oracle (Algorithm 4): the bisection keeps the volume,
its objective is monotone, a uniform optimum is a fixed point, and the
converged design approaches the optimum that the PBM oracle certifies."""
import numpy as np
import pytest

import workloads as W
from oracle import doc, fe, kkt, pbm


def test_bisection_volume_and_monotonicity():
    rng = np.random.default_rng(3)
    m = 500
    rho = rng.uniform(0.05, 0.9, m)
    uKu = rng.uniform(0.0, 3.0, m) ** 2
    lo, hi = np.full(m, 1e-3), np.ones(m)
    V = 0.3 * m
    for tau in (1e-3, 1e-5):
        rn, a, steps = doc.oc_update(rho, uKu, lo, hi, V, q=0.5, tau=tau)
        assert abs(rn.sum() - V) <= 3 * tau * V
        assert np.all(rn >= lo) and np.all(rn <= hi)
        assert steps > 5
    # the volume of rho+(alpha) is non-increasing in alpha: bisection is valid
    alphas = np.geomspace(1e-3, 1e3, 200)
    vol = [np.minimum(np.maximum(rho * uKu ** 0.5 / a, lo), hi).sum() for a in alphas]
    assert np.all(np.diff(vol) <= 1e-12)


def test_uniform_optimum_is_a_fixed_point():
    pr = W.bar_rollers(8, 4, 4, 2, vol_frac=0.5)
    r = doc.doc_solve(pr, eps=1e-4)
    assert r.converged and r.iterations == 1
    assert np.max(np.abs(r.rho - pr.V / pr.m)) <= 1e-4


def test_converges_to_the_certified_optimum():
    pr = W.config(0)
    r = doc.doc_solve(pr, eps=1e-5, max_iter=3000)
    assert r.converged
    P = pbm.VTS(pr)
    c_doc = kkt.compliance(P.grid, P.Ke, r.rho, P.f)
    st = pbm.Solver(pr).solve()
    lb, ub, rel = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho, st.u)
    assert rel <= 1e-7
    # DOC's design meets the volume to the bisection tolerance; projected onto
    # the exact volume it is feasible, so weak duality puts its compliance
    # above the dual bound, and DOC's tolerance puts it near the optimum
    assert abs(r.rho.sum() - P.V) <= 1e-5 * P.V
    c_feas = kkt.compliance(P.grid, P.Ke, kkt.project_feasible(r.rho, P.V, P.rho_lo, P.rho_hi),
                            P.f)
    assert c_feas >= lb * (1 - 1e-12)
    assert c_feas <= ub * (1 + 1e-3)
    assert abs(c_doc - c_feas) <= 1e-4 * c_feas
