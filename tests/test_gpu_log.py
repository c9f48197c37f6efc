"""The JSON-lines log of a PBM solve (vts_options.log_path): one line per
Newton step of Algorithm 2 and per outer iteration of Algorithm 1, then the
result; the counts and the final values agree with what vts_pbm_solve
returns."""
import json
import sys

import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def test_solve_log_matches_result(tmp_path):
    path = tmp_path / "solve.jsonl"
    pr = W.config(0)
    print("log test", pr.name, path, flush=True)
    sys.stdout.flush()
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64,
                                 options=V.default_options(log_path=str(path)))
    res = ctx.pbm_solve()
    ctx.close()
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    newton = [l for l in lines if l["event"] == "newton"]
    outer = [l for l in lines if l["event"] == "outer"]
    result = [l for l in lines if l["event"] == "result"]
    assert len(result) == 1 and lines[-1]["event"] == "result"
    r = result[0]
    assert (r["status"], r["outer"], r["newton"], r["minres"]) == (
        res["status"], res["outer"], res["newton"], res["minres"])
    assert r["kkt"] == res["kkt"]
    assert len(outer) == res["outer"] and outer[-1]["stop"] == 1
    assert all(o["stop"] == 0 for o in outer[:-1])
    assert len(newton) == res["newton"]
    assert sum(n["minres"] for n in newton) <= res["minres"]
    assert any(n["final"] == 1 for n in newton)
    assert all(0 < n["kappa"] <= 1 for n in newton)
