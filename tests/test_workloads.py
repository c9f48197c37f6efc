"""The Table 3 and 4 rows the bench compares against (workloads.paper_tables)
agree with the problem sizes in tests/golden/paper_problem_sizes.txt (both
transcribed from the paper; a mismatch is a transcription error), and the
footnote overrides map to the option values Section 7.2 states."""
import os

import pytest

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
