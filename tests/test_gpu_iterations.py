"""The GPU's whole PBM iteration record against the FP64 oracle's, both in
FP64 from the same initial point (Algorithm 1 with Algorithm 2, the eps_NWT
update of Algorithm 1, the eps_MR rule of Section 6.2, the stall stop):
outer iterations, the Newton steps and MINRES iterations of every outer
iteration, the gap ratio |delta/d| of eq. (2.6) after every outer iteration,
and the Newton steps of the final call.  A MINRES solve may end one
iteration apart where it stops within rounding of its test."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import pbm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402

CASES = {
    "cant-8x4x4": lambda: W.config(0),
    "bridge-16x8x8": lambda: W.bridge_top(16, 8, 8, 3, vol_frac=0.15, h=0.25),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_record(pr):
    s = pbm.Solver(pr)
    marks = []                      # Newton steps done after each outer iteration
    s.progress = lambda k, d: marks.append(len(s.log.newton))
    s.solve()
    minres = [d["minres"] for d in s.log.newton]
    outer, start = [], 0
    for end, d in zip(marks, s.log.outer):
        outer.append((end - start, sum(minres[start:end]), d["ratio"]))
        start = end
    final_newton = len(minres) - start
    return s.status, outer, final_newton


@pytest.mark.parametrize("case", list(CASES))
def test_iteration_record_matches_oracle(case):
    pr = CASES[case]()
    say("iteration record", case)
    o_status, o_outer, o_final = _oracle_record(pr)
    assert o_status == "ok"

    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    g_outer = []
    while True:
        st = ctx.pbm_iterate()
        g_outer.append((st["newton_its"], st["minres_its"], st["ratio"]))
        if st["converged"]:
            break
        assert len(g_outer) < len(o_outer), "GPU needs more outer iterations"
    res = ctx.pbm_solve()
    ctx.close()
    g_final = res["newton"] - sum(n for n, _, _ in g_outer)
    say("  oracle outer", [(n, m) for n, m, _ in o_outer], "final Newton", o_final)
    say("  GPU    outer", [(n, m) for n, m, _ in g_outer], "final Newton", g_final)
    assert res["status"] == V.VTS_OK
    assert len(g_outer) == len(o_outer)
    for (gn, gm, gr), (on, om, orr) in zip(g_outer, o_outer):
        assert gn == on
        assert abs(gm - om) <= on                       # at most one per Newton step
        assert abs(gr - orr) <= 1e-3 * abs(orr) + 1e-14
    assert g_final == o_final
