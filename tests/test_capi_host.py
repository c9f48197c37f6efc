"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point that include/vts.h declares, and rejects invalid problems before
touching a device."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import pbm as opbm
from paper_1904_06556_amd import vts as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vts.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vts_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = V.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(V.SIGNATURES), set(names) ^ set(V.SIGNATURES)


def test_default_options_match_oracle_defaults():
    o = V.default_options()
    p = opbm.Options()
    for k in ("beta", "gamma", "p_min", "q_min", "eps_pbm", "eps_nwt0", "eps_nwt_min", "eps_nwt_final",
              "eps_stat", "accept_stall", "eps_mr_min", "armijo_c1", "armijo_min",
              "max_outer", "max_newton", "max_minres"):
        assert getattr(o, k) == pytest.approx(getattr(p, k), rel=0, abs=0), k
    assert bool(o.final_res4) == p.final_res4
    assert bool(o.p_min_relative) == p.p_min_relative
    assert o.stall_steps == p.stall_steps


def test_footprint_grows_with_problem():
    a = V.Context.footprint_bytes(8, 4, 4, 3)
    b = V.Context.footprint_bytes(64, 32, 32, 5)
    c = V.Context.footprint_bytes(64, 32, 32, 5, V.VTS_MIXED)
    assert 0 < a < b and c < b


def _create(pr, **kw):
    return V.Context(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, pr.f, kw.pop("V", pr.V),
                     pr.rho_lo, pr.rho_hi, **kw)


def _expect(status, fn):
    with pytest.raises(V.VtsError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


def test_rejects_not_strictly_feasible_volume():
    pr = W.cantilever_edge(8, 4, 4, 3)
    _expect(V.VTS_EINVAL, lambda: _create(pr, V=pr.m * 1.0))       # V = sum rho_hi
    _expect(V.VTS_EINVAL, lambda: _create(pr, V=pr.m * 1e-3))      # V = sum rho_lo


def test_rejects_missing_supports_and_bad_grids():
    pr = W.cantilever_edge(8, 4, 4, 3)
    pr.fixed[:] = 0
    _expect(V.VTS_EINVAL, lambda: _create(pr))
    pr = W.cantilever_edge(6, 4, 4, 3)                              # 6 not divisible by 4
    _expect(V.VTS_EINVAL, lambda: _create(pr))


def test_rejects_supports_not_nested_across_levels():
    pr = W.cantilever_edge(8, 4, 4, 3)
    pr.fixed[:] = 0
    node = pr.node(1, 1, 1)                                        # odd node: not on coarse grid
    pr.fixed[3 * node:3 * node + 3] = 1
    pr.fixed[:3] = 1
    _expect(V.VTS_EINVAL, lambda: _create(pr))


def test_rejects_non_finite_load():
    pr = W.cantilever_edge(8, 4, 4, 3)
    f = pr.f.copy()
    f[3 * 10 + 1] = np.nan
    pr.f = f
    _expect(V.VTS_EINVAL, lambda: _create(pr))
    f[3 * 10 + 1] = np.inf
    _expect(V.VTS_EINVAL, lambda: _create(pr))


def test_rejects_too_large_coarsest_level():
    pr = W.cantilever_edge(32, 16, 16, 1)
    _expect(V.VTS_EINVAL, lambda: _create(pr))


def test_state_layout_roundtrip_pack():
    d = dict(u=np.arange(6.0), alpha=2.0, nu_lo=[1.0], nu_hi=[2.0], rho=[3.0], mu_lo=[4.0],
             mu_hi=[5.0], p=[6.0], q_lo=[7.0], q_hi=[8.0], eps_nwt=0.5, eps_mr=1e-3)
    b = V.Context.pack_state(d, 6, 1)
    h = V.STATE_HEAD
    assert b.size == h + 6 + 1 + 8 + 2 + 3 and b[h + 6] == 2.0 and b[h + 6 + 1 + 8 + 1] == 1e-3
    assert list(b[:h]) == [V.STATE_MAGIC, V.STATE_VERSION, 6, 1]
    assert list(b[-3:]) == [0, 0, 0]
    d.update(outer=7, newton=11, minres=123)
    assert list(V.Context.pack_state(d, 6, 1)[-3:]) == [7, 11, 123]


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys as _sys
    r = subprocess.run([_sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_product_code_does_not_use_the_oracle():
    """The package never imports oracle/; in bench.py only the cpu_baseline
    legs (functions named cpu_baseline*) do."""
    import ast
    import glob
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def oracle_imports(tree):
        for node in ast.walk(tree):
            if isinstance(node, ast.Import) and any(a.name.split(".")[0] == "oracle"
                                                   for a in node.names):
                yield node
            if isinstance(node, ast.ImportFrom) and (node.module or "").split(".")[0] == "oracle":
                yield node

    for path in glob.glob(os.path.join(root, "paper_1904_06556_amd", "*.py")):
        assert not list(oracle_imports(ast.parse(open(path).read()))), path
    tree = ast.parse(open(os.path.join(root, "bench.py")).read())
    for fn in tree.body:
        if isinstance(fn, ast.FunctionDef) and not fn.name.startswith("cpu_baseline"):
            assert not list(oracle_imports(fn)), fn.name
    assert not [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))
                and list(oracle_imports(n))]


def test_header_is_plain_c99(tmp_path):
    """include/vts.h compiles as ISO C99 (no C++ or torch types cross the ABI)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text('#include "vts.h"\nint main(void) { vts_options o; vts_default_options(&o);'
                   ' return o.max_outer > 0 ? 0 : 1; }\n')
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o",
                        str(tmp_path / "abi.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
