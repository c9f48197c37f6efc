"""End-to-end pins of the oracle PBM solver (Algorithms 1 and 2) against
results fixed by the mathematics: brute force, a case with a closed-form
optimum, weak duality (Theorem 2) and invariances of problem (1.1)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import pbm, kkt, fe


def _solve(pr, **kw):
    s = pbm.Solver(pr, pbm.Options(**kw))
    st = s.solve()
    assert s.status == "ok"
    return s, st


def _check(s, st):
    P = s.P
    return kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho, st.u, st.alpha)


def test_two_element_brute_force():
    # m = 2: c(r, V - r) is convex in r; golden section to 1e-12
    pr = W.cantilever_edge(2, 1, 1, 1, vol_frac=0.6)
    s, st = _solve(pr)
    P = s.P
    lo = max(P.rho_lo[0], P.V - P.rho_hi[1])
    hi = min(P.rho_hi[0], P.V - P.rho_lo[1])
    c = lambda r: kkt.compliance(P.grid, P.Ke, np.array([r, P.V - r]), P.f)
    g = (math.sqrt(5) - 1) / 2
    a, b = lo, hi
    for _ in range(200):
        x1, x2 = b - g * (b - a), a + g * (b - a)
        if c(x1) < c(x2):
            b = x2
        else:
            a = x1
    cstar = c(0.5 * (a + b))
    assert abs(kkt.compliance(P.grid, P.Ke, st.rho, P.f) - cstar) < 1e-7 * cstar
    assert abs(st.rho[0] - 0.5 * (a + b)) < 1e-5


def test_uniform_strain_bar_has_uniform_optimum():
    pr = W.bar_rollers(4, 2, 2, 2, vol_frac=0.5)
    s, st = _solve(pr)
    P = s.P
    assert np.max(np.abs(st.rho - P.V / P.grid.m)) < 1e-6
    c_uni = kkt.compliance(P.grid, P.Ke, np.full(P.grid.m, P.V / P.grid.m), P.f)
    assert abs(0.5 * P.f @ st.u - c_uni) < 1e-7 * c_uni


@pytest.fixture(scope="module")
def c1():
    return _solve(W.config(0))


def test_config0_kkt_and_duality_certificate(c1):
    s, st = c1
    r = _check(s, st)
    assert r["kkt"] <= 1e-6, r
    P = s.P
    lb, ub, rel = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho, st.u)
    assert rel <= 1e-7
    c = kkt.compliance(P.grid, P.Ke, st.rho, P.f)
    # rho itself is feasible only to the KKT tolerance: its compliance sits
    # within that tolerance of the bracket
    assert lb * (1 - 1e-6) <= c <= ub * (1 + 1e-6)
    # Section 7.1 reports the volume met from above within one permille at
    # the paper's looser tolerances; at KKT 1e-6 it is met to rounding level
    # from either side
    assert -1e-9 * P.V <= st.rho.sum() - P.V <= 1e-3 * P.V


def test_config0_mirror_symmetry(c1):
    s, st = c1
    g = s.P.grid
    r = st.rho.reshape(g.nz, g.ny, g.nx)
    assert np.max(np.abs(r - r[:, ::-1, :])) < 1e-5


def test_load_scaling_invariance(c1):
    s, st = c1
    pr = W.config(0)
    pr.f = 2.0 * pr.f
    s2, st2 = _solve(pr)
    c1v = kkt.compliance(s.P.grid, s.P.Ke, st.rho, s.P.f)
    c2v = kkt.compliance(s2.P.grid, s2.P.Ke, st2.rho, s2.P.f)
    assert abs(c2v - 4 * c1v) < 1e-6 * c2v
    assert np.max(np.abs(st.rho - st2.rho)) < 1e-4


def test_bridge_small_kkt():
    pr = W.bridge_top(8, 4, 4, 2, vol_frac=0.15)
    s, st = _solve(pr)
    assert _check(s, st)["kkt"] <= 1e-6


def test_stored_benchmark_oracle_run_is_certified():
    """The stored oracle run of the 64x32x32 cantilever: its compliance sits
    inside its own weak-duality bracket, the bracket is tight, and the run met
    the KKT target (values written by make_oracle_results.py)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "oracle_cant-64x32x32.json")))
    assert g["status"] == "ok" and g["workload"] == "cant-64x32x32"
    assert g["certificate_lower"] <= g["compliance_exact"] <= g["certificate_upper"]
    assert g["certificate_rel"] <= 1e-7
    assert abs(g["compliance_half_fu"] - g["compliance_exact"]) <= 1e-6 * g["compliance_exact"]
    assert g["kkt"] <= 1e-6
    assert abs(g["sum_rho"] - g["V"]) <= 1e-6 * g["V"]
    # the stored iteration record is that of the totals, and its last outer
    # iteration met the outer tests of the options it was run with
    o = g["options"]
    assert len(g["outer_log"]) == g["outer"] and len(g["newton_log"]) == g["newton"]
    assert sum(d["minres"] for d in g["newton_log"]) == g["minres"]
    last = g["outer_log"][-1]
    assert last["ratio"] < o["eps_pbm"] and last["stat"] < o["eps_stat"]
    assert all(d["ratio"] >= o["eps_pbm"] or d["stat"] >= o["eps_stat"]
               for d in g["outer_log"][:-1])
    # the final Newton call (Algorithm 1, last step) met its tolerance
    assert g["newton_log"][-1]["res"] <= o["eps_nwt_final"]


def test_paper_parameters_reach_the_paper_accuracy():
    """With the parameter values of Section 7 (absolute penalty floors 1e-8,
    eps_PBM = 1e-5) the oracle stops with the gap ratio below 1e-5 and a
    compliance within that accuracy of the certified optimum."""
    pr = W.config(0)
    s = pbm.Solver(pr, pbm.paper_options())
    st = s.solve()
    assert s.status == "ok"
    assert s.log.outer[-1]["ratio"] < 1e-5
    P = s.P
    ref = pbm.Solver(pr).solve()
    lb, ub, rel = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, ref.rho, ref.u)
    c = kkt.compliance(P.grid, P.Ke, kkt.project_feasible(st.rho, P.V, P.rho_lo, P.rho_hi), P.f)
    assert lb * (1 - 1e-12) <= c <= ub * (1 + 1e-4)


def test_missed_final_kkt_check_resumes_the_outer_loop():
    """A 16x8x8 cantilever (V/m = 0.2535, the first request of the serving
    burst) meets the outer stopping test at stationarity 3.7e-7, and the
    final Newton call and rho update leave 1.06e-6 > 1e-6: the outer loop
    resumes with half the stationarity target and the result meets KKT
    1e-6, certified by weak duality (Theorem 2)."""
    frac = float(np.random.default_rng(1).uniform(0.1, 0.4))
    pr = W.cantilever_edge(16, 8, 8, 3, vol_frac=frac)
    s, st = _solve(pr, max_outer=500)
    assert len(s.log.outer) > 13            # the first stop was at 13 outer iterations
    r = _check(s, st)
    assert r["kkt"] <= 1e-6
    P = s.P
    lb, ub, gap = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, st.rho, st.u)
    assert gap < 1e-6
    # without a resumption the same run ends above the target
    t = pbm.Solver(pr, pbm.Options(max_outer=500))
    saved, pbm.KKT_RESUMES = pbm.KKT_RESUMES, 0
    try:
        t.solve()
    finally:
        pbm.KKT_RESUMES = saved
    assert t.status == "kkt" and t.kkt["kkt"] > 1e-6 and len(t.log.outer) == 13
