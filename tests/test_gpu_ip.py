"""Primal-dual interior point method (Algorithm 3) on the GPU against the
oracle: the iterates and the per-iteration records of the first passes, the
converged design, and the error paths."""
import numpy as np
import pytest

import workloads as W
from oracle import ip, kkt, pbm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1904_06556_amd import vts as V  # noqa: E402


def say(*a):
    print("[ip]", *a, flush=True)


CASES = {
    "cant-8x4x4-l3": (lambda: W.config(0), 8),
    "cant-16x8x8-l3": (lambda: W.cantilever_edge(16, 8, 8, 3, vol_frac=0.3), 8),
    # the size and launch configuration that bench.py --ip times
    "cant-64x32x32-l5": (lambda: W.config(1), 3),
}


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", list(CASES))
def test_ip_iterates_match_oracle(case):
    """The first passes, where the systems are still well conditioned: the
    same MINRES counts, barrier parameters and step lengths, and iterates
    equal to rounding."""
    make, passes = CASES[case]
    pr = make()
    say("iterates", case)
    ref = ip.Solver(pr)
    P = ref.P
    st = ip.initial_state(P.grid.n_dof, P.grid.m, P.V)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    ctx.ip_init()
    for k in range(passes):
        g = ctx.ip_step()
        st, h = ref.step(st)
        say(" pass", k, "minres", g["minres_its"], h["minres"], "ratio", g["gap_ratio"])
        assert g["minres_its"] == h["minres"]
        assert g["r"] == pytest.approx(h["r"], rel=1e-12)
        assert g["s"] == pytest.approx(h["s"], rel=1e-12)
        for key in ("kappa_u", "kappa_nu_lo", "kappa_nu_hi"):
            assert g[key] == pytest.approx(h[key], rel=1e-8, abs=1e-12), key
        assert g["gap_ratio"] == pytest.approx(h["ratio"], rel=1e-6, abs=1e-10)
        assert g["res_ip"] == pytest.approx(h["res_ip"], rel=1e-6)
        assert g["compliance"] == pytest.approx(h["objective"], rel=1e-10)
        d = ctx.state_dict()
        assert rel(d["u"], st.u) <= 1e-8
        assert d["alpha"] == pytest.approx(st.alpha, rel=1e-9)
        assert rel(d["rho"], st.rho) <= 1e-9
        assert rel(d["nu_lo"], st.nu_lo) <= 1e-8
        assert rel(d["nu_hi"], st.nu_hi) <= 1e-8
    ctx.close()


def test_ip_solve_reaches_the_optimum():
    pr = W.config(0)
    say("solve", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    s = ctx.ip_solve()
    say(" iterations", s["iterations"], "minres", s["minres_its"], "ratio", s["gap_ratio"])
    assert s["converged"] == 1 and s["status"] == V.VTS_OK
    assert s["gap_ratio"] < 1e-5 and s["res_ip"] < 1e-4
    ref = ip.Solver(pr).solve()
    assert ref.converged
    assert abs(s["iterations"] - ref.iterations) <= 3
    d = ctx.state_dict()
    P = pbm.VTS(pr)
    # alpha is minus the volume multiplier; the optimum is certified by
    # weak duality
    lb, ub, _ = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"])
    assert abs(s["compliance"] - ub) <= 1e-5 * ub
    k = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"],
                         -d["alpha"])
    assert k["kkt"] <= 1e-3
    assert abs(s["compliance"] - 0.5 * P.f @ ref.state.u) <= 1e-5 * ub
    ctx.close()


def test_ip_error_paths():
    pr = W.config(0)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    s = ctx.ip_step(check=False)
    assert s["status"] == V.VTS_ESTATE
    with pytest.raises(V.VtsError):
        ctx.ip_init(sigma_r=1.5)
    with pytest.raises(V.VtsError):
        ctx.ip_init(max_minres=0)
    # a run cut at max_iter reports non-convergence and keeps a strictly
    # feasible iterate
    s = ctx.ip_solve(check=False, max_iter=3)
    assert s["status"] == V.VTS_ENOTCONV and s["iterations"] == 3
    d = ctx.state_dict()
    P = pbm.VTS(pr)
    assert np.all(d["rho"] > P.rho_lo) and np.all(d["rho"] < P.rho_hi)
    assert np.all(d["nu_lo"] > 0) and np.all(d["nu_hi"] > 0)
    # the context still runs PBM afterwards
    ctx.reset()
    r = ctx.pbm_solve()
    assert r["status"] == V.VTS_OK
    ctx.close()
