"""The two large workloads solved end to end in mixed precision (FP32
multigrid, FP64 MINRES / Newton / multipliers): the 128x64x64 bridge
(1.6 M DOFs) and the 192x96x96 cantilever with three point loads (5.4 M
DOFs).  Checked on the host with the oracle's definitions: the KKT residual
of the returned (rho, u, alpha) (problem (1.1)) and the weak-duality bracket
of Theorem 2 (the dual lower bound of u against 1/2 f^T u), to the KKT
level at which the returned rho is feasible."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fe, kkt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("idx", [2, 3])
def test_large_workload_reaches_kkt_1e6_mixed(idx):
    pr = W.config(idx)
    say("end to end", pr.name)
    opts = V.default_options()
    if pr.extra.get("p_min"):
        opts.p_min = pr.extra["p_min"]
    ctx = V.Context.from_problem(pr, precision=V.VTS_MIXED, options=opts)
    res = ctx.pbm_solve()
    say(" ", {k: res[k] for k in ("status", "outer", "newton", "minres", "kkt", "compliance")})
    assert res["status"] == V.VTS_OK and res["kkt"] <= 1e-6
    d = ctx.state_dict()
    ctx.close()
    g = fe.Grid(pr.nx, pr.ny, pr.nz, pr.fixed)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    f = g.mask(pr.f)
    lo = np.broadcast_to(np.asarray(pr.rho_lo, float), (pr.m,))
    hi = np.broadcast_to(np.asarray(pr.rho_hi, float), (pr.m,))
    r = kkt.kkt_residual(g, Ke, f, pr.V, lo, hi, d["rho"], d["u"], d["alpha"])
    say("  host KKT", r)
    assert r["kkt"] <= 1e-6
    assert abs(r["kkt"] - res["kkt"]) <= 1e-9 + 1e-6 * r["kkt"]
    c = 0.5 * float(f @ d["u"])
    assert abs(c - res["compliance"]) <= 1e-12 * c
    lb, _ = kkt.dual_lower_bound(g, Ke, f, pr.V, lo, hi, d["u"])
    say("  compliance", c, "dual lower bound", lb, "rel gap", (c - lb) / c)
    # weak duality (Theorem 2) bounds the compliance of a feasible rho from
    # below; the returned rho meets its box and volume only to the KKT level
    # (r_box, r_vol <= 1e-6), and the compliance moves by about sum_i e_i
    # |drho_i|, so the bracket holds to that level and no closer
    assert lb <= c * (1 + 1e-6)
    assert abs(c - lb) / c <= 1e-6
