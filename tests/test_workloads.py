"""The Table 3 and 4 rows the bench compares against (workloads.paper_tables)
agree with the problem sizes in tests/golden/paper_problem_sizes.txt (both
transcribed from the paper; a mismatch is a transcription error), and the
footnote overrides map to the option values Section 7.2 states; the load
cases of the multi-load workloads and the binding's check of their length."""
import os

import numpy as np
import pytest

import workloads as W
from workloads import paper_tables as T

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture():
    rows = {}
    with open(os.path.join(HERE, "golden", "paper_problem_sizes.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, mx, my, mz, l, m, n, src = line.split()
                if src in ("Table3", "Table4"):
                    rows[f"{k}-{mx}-{my}-{mz}-{l}"] = (int(m), int(n))
    return rows


def test_tables_cover_the_families_with_the_fixture_sizes():
    fx = _fixture()
    assert set(fx) == set(T.TABLES)
    for name, (m, n) in fx.items():
        e = T.entry(name)
        assert (e["m"], e["n"]) == (m, n), name
        outer, nwt, mr = e["pbm"]
        assert 0 < outer <= nwt


@pytest.mark.parametrize("name", ["BRIDGE-2-2-2-7", "BRIDGE-4-2-2-7", "BRIDGE-6-2-2-7",
                                  "BRIDGE-8-2-2-7"])
def test_stalled_bridges_carry_their_res_pbm(name):
    assert T.entry(name)["res_pbm"] is not None and 1 in T.entry(name)["flags"]


def test_paper_overrides_follow_footnotes():
    n = T.entry("CANT-8-2-2-7")["n"]
    o = T.paper_overrides("CANT-8-2-2-7", n)
    assert o["beta"] == o["gamma"] == 0.5 and abs(o["eps_mr0"] - 1e-5 * n ** 0.5) < 1e-12
    assert T.paper_overrides("BRIDGE-2-2-2-7", 1) == {"beta": 0.5, "gamma": 0.5}
    o = T.paper_overrides("BRIDGE-6-2-2-7", 4.0)
    assert o["eps_nwt0"] == 0.1 and o["eps_mr0"] == 2e-5
    assert T.paper_overrides("CANT-4-2-2-6", 1.0) == {}


def test_load_cases_of_the_multi_load_workloads():
    pr = W.multi_config(0)
    F = W.load_cases(pr)
    assert F.shape == (2, pr.n_dof)
    assert np.all(F[:, pr.fixed == 1] == 0.0)
    assert np.array_equal(F.sum(axis=0), pr.f)
    # the single-load problems carry their one load
    one = W.cantilever_edge(8, 4, 4, 3)
    assert np.array_equal(W.load_cases(one), one.f[None, :])
    # the point-load cantilever's cases sum to its single load
    pts = W.cantilever_points(16, 8, 8, 3, npoints=3, seed=0)
    assert "load_cases" not in pts.extra
    cases = W.point_cases(pts)
    assert cases.shape == (3, pts.n_dof) and np.array_equal(cases.sum(axis=0), pts.f)
    assert np.all(np.count_nonzero(cases, axis=1) == 1)


def test_binding_checks_the_length_of_the_load_cases():
    from paper_1904_06556_amd import vts as V
    pr = W.cantilever_two_loads(8, 4, 4, 3)
    f = W.load_cases(pr).ravel()
    p, _ = V._problem_struct(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, f, pr.V, 1e-3, 1.0,
                             1.0, 0.3, 1.0, V.VTS_FP64, 2)
    assert p.nload == 2
    with pytest.raises(ValueError):
        V._problem_struct(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, f, pr.V, 1e-3, 1.0,
                          1.0, 0.3, 1.0, V.VTS_FP64, 3)
