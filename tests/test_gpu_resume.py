"""The outer loop's resumption after a missed final KKT check (Algorithm 1
stopping test, this library's KKT target) on the GPU against the oracle:
the 16x8x8 serving cantilever at V/m = 0.2535 first stops at 13 outer
iterations with a returned state above KKT 1e-6, resumes, and ends below it
with the oracle's outer and Newton counts, in FP64 and mixed precision."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import kkt, pbm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def _problem():
    frac = float(np.random.default_rng(1).uniform(0.1, 0.4))
    return W.cantilever_edge(16, 8, 8, 3, vol_frac=frac)


@pytest.mark.parametrize("precision", [V.VTS_FP64, V.VTS_MIXED])
def test_resumed_solve_matches_oracle(precision):
    pr = _problem()
    print("resumed solve", pr.name, "precision", precision, flush=True)
    sys.stdout.flush()
    s = pbm.Solver(pr, pbm.Options(max_outer=500))
    so = s.solve()
    assert s.status == "ok" and len(s.log.outer) > 13
    ctx = V.Context.from_problem(pr, precision=precision,
                                 options=V.default_options(max_outer=500))
    res = ctx.pbm_solve()
    d = ctx.state_dict()
    P = pbm.VTS(pr)
    r = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"], d["alpha"])
    assert res["status"] == 0 and r["kkt"] <= 1e-6, r
    assert res["outer"] == len(s.log.outer)
    assert res["newton"] == len(s.log.newton)
    c_or = kkt.compliance(P.grid, P.Ke, so.rho, P.f)
    assert kkt.compliance(P.grid, P.Ke, d["rho"], P.f) == pytest.approx(c_or, rel=1e-6)
    ctx.close()
