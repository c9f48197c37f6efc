"""GPU parity tests: the HIP path (through the C ABI) against the FP64 oracle
on the same seeded inputs.  Tolerances: operator applications relative 1e-12
(bound 1e-10); one V-cycle in FP64 1e-10; FP32 paths at their rounding
level; final compliance 1e-6 and KKT residual <= 1e-6."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fe, pbm, mg, minres, kkt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


OP_CASES = {
    "cant-8x4x4-l3": lambda: W.cantilever_edge(8, 4, 4, 3),
    "cant-10x6x4-l2": lambda: W.cantilever_edge(10, 6, 4, 2),
    "bridge-16x8x8-l3": lambda: W.bridge_top(16, 8, 8, 3),
    "bridge-32x16x16-l4-h": lambda: W.bridge_top(32, 16, 16, 4, h=0.125),
    "cant-64x32x32-l5": lambda: W.config(1),
}


@pytest.mark.parametrize("case", list(OP_CASES))
def test_apply_K_parity(case):
    pr = OP_CASES[case]()
    say("apply_K", case)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    g = fe.Grid(pr.nx, pr.ny, pr.nz, pr.fixed)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    rho = W.random_rho(pr.m, seed=1)
    x = W.random_vector(pr.n_dof, seed=2)          # fixed entries non-zero: masked on read
    ctx.set_rho(dev(rho))
    y = torch.empty(pr.n_dof, dtype=torch.float64, device="cuda")
    ctx.apply_K(dev(x), y)
    yo = fe.apply_K(g, Ke, rho, x)
    assert rel(host(y), yo) < 1e-12
    assert np.all(host(y)[pr.fixed == 1] == 0)
    # FP32 operator (the mixed-precision multigrid's arithmetic)
    yf = torch.empty(pr.n_dof, dtype=torch.float32, device="cuda")
    ctx.apply_K_f32(dev(x, torch.float32), yf)
    assert rel(host(yf), yo) < 2e-5
    # caller-supplied rho (the context's rho untouched): the same operator
    rho2 = W.random_rho(pr.m, seed=7)
    y2 = torch.empty_like(y)
    ctx.apply_K_rho(dev(rho2), dev(x), y2)
    assert rel(host(y2), fe.apply_K(g, Ke, rho2, x)) < 1e-12
    ctx.apply_K(dev(x), y)
    assert rel(host(y), yo) < 1e-12
    ctx.apply_K_rho_f32(dev(rho2, torch.float32), dev(x, torch.float32), yf)
    assert rel(host(yf), fe.apply_K(g, Ke, rho2, x)) < 2e-5
    # K(c 1) = c sum K_i
    ctx.set_rho(dev(np.full(pr.m, 0.37)))
    ctx.apply_K(dev(x), y)
    y1 = fe.apply_K(g, Ke, np.ones(pr.m), x)
    assert rel(host(y), 0.37 * y1) < 1e-12
    ctx.close()


def test_apply_K_deterministic():
    pr = W.config(1)
    say("determinism", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    ctx.set_rho(dev(W.random_rho(pr.m, seed=3)))
    x = dev(W.random_vector(pr.n_dof, seed=4))
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    ctx.apply_K(x, y1)
    ctx.apply_K(x, y2)
    assert torch.equal(y1, y2)
    ctx.close()


def test_element_energy_parity():
    pr = W.bridge_top(16, 8, 8, 3)
    say("energy", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    g = fe.Grid(pr.nx, pr.ny, pr.nz, pr.fixed)
    u = W.random_vector(pr.n_dof, seed=5, fixed=pr.fixed)
    e = torch.empty(pr.m, dtype=torch.float64, device="cuda")
    ctx.element_energy(dev(u), e)
    assert rel(host(e), fe.element_energies(g, fe.element_stiffness(), u)) < 1e-12
    ctx.close()


# ---------------------------------------------------------------- Newton system
def _state(P, seed, p=0.1):
    rng = np.random.default_rng(seed)
    m = P.grid.m
    st = pbm.initial_state(P.grid.n_dof, m, P.V)
    st.u = P.grid.mask(0.5 * rng.standard_normal(P.grid.n_dof))
    st.alpha = 0.3
    st.nu_lo = 0.05 * rng.random(m)
    st.nu_hi = 0.05 * rng.random(m)
    st.rho = rng.uniform(0.05, 1.0, m)
    st.mu_lo = rng.uniform(0.5, 1.5, m)
    st.mu_hi = rng.uniform(0.5, 1.5, m)
    st.p = np.full(m, p)
    st.q_lo = np.full(m, p)
    st.q_hi = np.full(m, p)
    return st


def _push(ctx, st, eps_mr=1e-3):
    d = dict(u=st.u, alpha=st.alpha, nu_lo=st.nu_lo, nu_hi=st.nu_hi, rho=st.rho,
             mu_lo=st.mu_lo, mu_hi=st.mu_hi, p=st.p, q_lo=st.q_lo, q_hi=st.q_hi,
             eps_nwt=1.0, eps_mr=eps_mr)
    ctx.set_state(V.Context.pack_state(d, ctx.n_dof, ctx.m))


def _sv(P, y_free_alpha):
    """oracle (free DOFs, alpha) -> S-vector (all DOFs, alpha)"""
    out = np.zeros(P.grid.n_dof + 1)
    out[P.free] = y_free_alpha[:-1]
    out[-1] = y_free_alpha[-1]
    return out


SYS_CASES = {
    "cant-8x4x4-l3": lambda: W.cantilever_edge(8, 4, 4, 3),
    "bridge-16x8x8-l3-h": lambda: W.bridge_top(16, 8, 8, 3, h=0.25),
    "cant-12x8x4-l2": lambda: W.cantilever_edge(12, 8, 4, 2),
}


@pytest.fixture(scope="module", params=list(SYS_CASES))
def system(request):
    pr = SYS_CASES[request.param]()
    say("system", request.param)
    P = pbm.VTS(pr)
    st = _state(P, seed=11)
    ev = pbm.evaluate(P, st)
    S = pbm.schur_matrix(P, ev)
    H = mg.Hierarchy(P.grid, S, pr.levels)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    _push(ctx, st)
    ctx.newton_setup()
    yield dict(pr=pr, P=P, st=st, ev=ev, S=S, H=H, ctx=ctx, name=request.param)
    ctx.close()


def test_setup_parity(system):
    P, ev, ctx = system["P"], system["ev"], system["ctx"]
    say("setup parity", system["name"])
    assert rel(host(ctx.vector("energy")), ev.e) < 1e-12
    assert rel(host(ctx.vector("rho1")), ev.rho1) < 1e-12
    w, z, _ = pbm.schur_weights(ev)
    assert rel(host(ctx.vector("w")), w) < 1e-12
    assert rel(host(ctx.vector("g1")), ev.g1) < 1e-11
    rhs = _sv(P, pbm.reduced_rhs(P, ev))
    assert rel(host(ctx.vector("rhs")), rhs) < 1e-11


def test_apply_S_parity(system):
    P, S, ctx = system["P"], system["S"], system["ctx"]
    say("apply_S parity", system["name"])
    xf = np.random.default_rng(21).standard_normal(P.n + 1)
    y = torch.empty(P.grid.n_dof + 1, dtype=torch.float64, device="cuda")
    ctx.apply_S(dev(_sv(P, xf)), y)
    assert rel(host(y), _sv(P, S @ xf)) < 1e-11


def test_vcycle_parity_fp64(system):
    P, H, ctx = system["P"], system["H"], system["ctx"]
    say("V-cycle parity", system["name"])
    r = np.random.default_rng(22).standard_normal(P.n + 1)
    z = torch.empty(P.grid.n_dof + 1, dtype=torch.float64, device="cuda")
    ctx.precondition(dev(_sv(P, r)), z)
    zo = _sv(P, H.vcycle(r))
    assert rel(host(z), zo) < 1e-10
    z2 = torch.empty_like(z)
    ctx.precondition(dev(_sv(P, r)), z2)
    assert torch.equal(z, z2)


def test_minres_parity(system):
    P, S, H, ctx, ev = system["P"], system["S"], system["H"], system["ctx"], system["ev"]
    say("MINRES parity", system["name"])
    rhs = pbm.reduced_rhs(P, ev)
    x, its, relres = minres.minres(lambda v: S @ v, rhs, H.vcycle, 1e-8, 500)
    st = ctx.solve_newton(1e-8)
    assert abs(st["iterations"] - its) <= 1
    dy = host(ctx.vector("dy"))
    assert rel(dy, _sv(P, x)) < 1e-7


def test_newton_step_parity():
    pr = W.cantilever_edge(8, 4, 4, 3)
    say("Newton step parity", pr.name)
    P = pbm.VTS(pr)
    st = _state(P, seed=31, p=0.3)
    solver = pbm.Solver(pr, pbm.Options(eps_mr0=1e-6))
    solver.eps_mr = 1e-6
    new, ev = solver.newton(st.copy(), eps_nwt=1e9)          # exactly one step
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64,
                                 options=V.default_options(eps_mr0=1e-6))
    _push(ctx, st, eps_mr=1e-6)
    ns = ctx.newton_step()
    g = ctx.state_dict()
    assert ns["kappa"] == solver.log.newton[-1]["kappa"]
    assert rel(g["u"], new.u) < 1e-8
    assert abs(g["alpha"] - new.alpha) < 1e-8 * abs(new.alpha)
    assert rel(g["nu_lo"], new.nu_lo) < 1e-7
    assert abs(ns["res_pbm"] - solver.log.newton[-1]["res"]) < 1e-7 * solver.log.newton[-1]["res"]
    ctx.close()


def test_mixed_precision_vcycle_close_to_fp64(system):
    pr, P, H = system["pr"], system["P"], system["H"]
    say("mixed V-cycle", system["name"])
    ctx = V.Context.from_problem(pr, precision=V.VTS_MIXED)
    _push(ctx, system["st"])
    ctx.newton_setup()
    r = np.random.default_rng(23).standard_normal(P.n + 1)
    z = torch.empty(P.grid.n_dof + 1, dtype=torch.float64, device="cuda")
    ctx.precondition(dev(_sv(P, r)), z)
    assert rel(host(z), _sv(P, H.vcycle(r))) < 1e-3
    ctx.close()


# ---------------------------------------------------------------- full PBM
@pytest.mark.parametrize("precision", [V.VTS_FP64, V.VTS_MIXED])
def test_pbm_solve_config0_matches_oracle(precision):
    pr = W.config(0)
    say("PBM solve", pr.name, "precision", precision)
    ctx = V.Context.from_problem(pr, precision=precision)
    res = ctx.pbm_solve()
    d = ctx.state_dict()
    P = pbm.VTS(pr)
    r = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"], d["alpha"])
    assert r["kkt"] <= 1e-6, r
    s = pbm.Solver(pr)
    so = s.solve()
    c_gpu = kkt.compliance(P.grid, P.Ke, d["rho"], P.f)
    c_or = kkt.compliance(P.grid, P.Ke, so.rho, P.f)
    assert abs(c_gpu - c_or) <= 1e-6 * c_or
    assert abs(res["compliance"] - 0.5 * P.f @ so.u) <= 1e-6 * c_or
    ctx.close()


@pytest.mark.parametrize("precision", [V.VTS_FP64, V.VTS_MIXED])
def test_pbm_solve_bridge_matches_oracle(precision):
    """Bridge on the unit-cube coarse box (element side 1/4), the shape of
    the 128x64x64 bridge workload at 3 levels."""
    pr = W.bridge_top(16, 8, 8, 3, vol_frac=0.15, h=0.25)
    say("PBM solve", pr.name, "h", pr.h, "precision", precision)
    ctx = V.Context.from_problem(pr, precision=precision)
    res = ctx.pbm_solve()
    d = ctx.state_dict()
    P = pbm.VTS(pr)
    r = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"], d["alpha"])
    assert r["kkt"] <= 1e-6, r
    so = pbm.Solver(pr).solve()
    c_gpu = kkt.compliance(P.grid, P.Ke, d["rho"], P.f)
    c_or = kkt.compliance(P.grid, P.Ke, so.rho, P.f)
    assert abs(c_gpu - c_or) <= 1e-6 * c_or
    assert abs(res["compliance"] - 0.5 * P.f @ so.u) <= 1e-6 * c_or
    ctx.close()


def test_checkpoint_roundtrip():
    pr = W.config(0)
    say("checkpoint", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    ctx.pbm_iterate()
    s1 = ctx.get_state()
    a = ctx.pbm_iterate()
    s2 = ctx.get_state()
    ctx.set_state(s1)
    b = ctx.pbm_iterate()
    assert np.array_equal(ctx.get_state(), s2)
    assert a["gap"] == b["gap"]
    # resumed in a fresh context: same iterate and the run's counters
    fresh = V.Context.from_problem(pr, precision=V.VTS_FP64)
    fresh.set_state(s1)
    c = fresh.pbm_iterate()
    assert np.array_equal(fresh.get_state(), s2)
    assert c["gap"] == a["gap"]
    d = fresh.state_dict()
    assert d["outer"] == 2 and d["newton"] > 0 and d["minres"] > 0
    fresh.close()
    ctx.close()


@pytest.mark.parametrize("precision", [V.VTS_FP64, V.VTS_MIXED])
def test_benchmark_workload_matches_stored_oracle(precision):
    """The 64x32x32 cantilever in the benchmark's configuration against the
    stored FP64 oracle run (tests/golden/oracle_cant-64x32x32.json, written by
    make_oracle_results.py from oracle/ alone): compliance within 1e-6, inside
    the oracle's weak-duality bracket, KKT <= 1e-6, and the same iteration
    record: outer iterations and Newton steps equal, MINRES iterations within
    2 % (the multigrid's rounding order differs, which moves single MINRES
    counts by one)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "oracle_cant-64x32x32.json")))
    pr = W.config(1)
    say("benchmark workload vs stored oracle", pr.name, "precision", precision)
    opts = V.default_options(eps_mr0=pr.extra["eps_mr0"])
    ctx = V.Context.from_problem(pr, precision=precision, options=opts)
    res = ctx.pbm_solve()
    c_or = gold["compliance_half_fu"]
    assert abs(res["compliance"] - c_or) <= 1e-6 * c_or
    lo, hi = gold["certificate_lower"], gold["certificate_upper"]
    assert lo * (1 - 1e-6) <= res["compliance"] <= hi * (1 + 1e-6)
    d = ctx.state_dict()
    P = pbm.VTS(pr)
    r = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"], d["alpha"])
    assert r["kkt"] <= 1e-6, r
    assert abs(res["alpha"] - gold["alpha"]) <= 1e-5 * abs(gold["alpha"])
    say("  counts", res["outer"], res["newton"], res["minres"], "oracle", gold["outer"],
        gold["newton"], gold["minres"])
    assert (res["outer"], res["newton"]) == (gold["outer"], gold["newton"])
    assert abs(res["minres"] - gold["minres"]) <= 0.02 * gold["minres"]
    ctx.close()


def test_pbm_solve_is_bitwise_repeatable():
    pr = W.config(0)
    say("repeatability", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_MIXED)
    a = ctx.pbm_solve()
    sa = ctx.get_state()
    ctx.reset()
    b = ctx.pbm_solve()
    assert a == b
    assert np.array_equal(sa, ctx.get_state())
    ctx.close()


def test_profile_hook_counts_launches():
    pr = W.config(1)
    say("profile hook", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    ctx.newton_setup()
    n = ctx.n_dof + 1
    r = torch.rand(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    ctx.profile_start("gs_fine")
    for _ in range(3):
        ctx.precondition(r, z)
    p = ctx.profile_stop()
    # 7 forward passes (colour 0 is fused into the input step) + 8 backward
    assert p["launches"] == 3 * 15 and p["total_ms"] > 0 and p["bytes"] > 0
    ctx.profile_start("apply_K")
    x = torch.rand(ctx.n_dof, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ctx.apply_K(x, y)
    p = ctx.profile_stop()
    assert p["launches"] == 1 and p["bytes"] == 16.0 * ctx.n_dof + 8.0 * ctx.m
    ctx.close()


@pytest.mark.parametrize("prec", [V.VTS_FP64, V.VTS_MIXED])
def test_graph_vcycle_equals_direct_launches(prec):
    """V-cycles replayed from captured HIP graphs against the same kernels
    launched one by one: replays of one graph with other device work in
    between, fresh captures for new buffers (and eviction from the graph
    cache), and a whole solve, all bitwise equal."""
    pr = W.cantilever_edge(32, 16, 16, 4, vol_frac=0.2)
    say("graph V-cycle", pr.name, prec)
    g = V.Context.from_problem(pr, precision=prec, options=V.default_options(use_graphs=1))
    e = V.Context.from_problem(pr, precision=prec, options=V.default_options(use_graphs=0))
    for c in (g, e):
        c.newton_setup()
    n = g.n_dof + 1
    gen = torch.Generator(device="cuda").manual_seed(5)
    r = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
    zg, ze = torch.empty_like(r), torch.empty_like(r)
    s = torch.empty_like(r)
    for rep in range(8):
        if rep >= 3:
            # new buffers: a new capture each time, older graphs evicted
            r = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
            zg, ze = torch.empty_like(r), torch.empty_like(r)
        g.precondition(r, zg)
        e.precondition(r, ze)
        g.apply_S(zg, s)              # other work on the stream between replays
        torch.cuda.synchronize()
        assert torch.equal(zg, ze), rep
    ra, rb = g.pbm_solve(), e.pbm_solve()
    assert ra == rb
    assert np.array_equal(g.get_state(), e.get_state())
    # a second solve on the same contexts (graphs rebuilt per Newton step)
    g.reset()
    e.reset()
    assert g.pbm_solve() == e.pbm_solve() == ra
    g.close()
    e.close()


DEGENERATE = {
    "one-element-1x1x1-l1": lambda: W.cantilever_edge(1, 1, 1, 1, vol_frac=0.3),
    "two-elements-2x1x1-l1": lambda: W.cantilever_edge(2, 1, 1, 1, vol_frac=0.6),
    "ragged-7x3x5-l1": lambda: W.cantilever_edge(7, 3, 5, 1, vol_frac=0.25),
}


@pytest.mark.parametrize("precision", [V.VTS_FP64, V.VTS_MIXED])
@pytest.mark.parametrize("case", list(DEGENERATE))
def test_degenerate_grids_solve(case, precision):
    """One level (the multigrid is the coarse solve alone), one and two
    elements, and a grid of odd sizes, against what fixes their optimum:
    m = 1 has rho = V; m = 2 a convex one-dimensional compliance (golden
    section); otherwise the weak-duality bracket."""
    pr = DEGENERATE[case]()
    say("degenerate", case, precision)
    ctx = V.Context.from_problem(pr, precision=precision)
    r = ctx.pbm_solve()
    d = ctx.state_dict()
    ctx.close()
    P = pbm.VTS(pr)
    k = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"], d["u"], d["alpha"])
    assert k["kkt"] <= 1e-6, k
    c = kkt.compliance(P.grid, P.Ke, d["rho"], P.f)
    assert abs(r["compliance"] - c) <= 1e-6 * c
    if P.grid.m == 1:
        assert abs(d["rho"][0] - P.V) <= 1e-9 * P.V
        assert abs(c - kkt.compliance(P.grid, P.Ke, np.array([P.V]), P.f)) <= 1e-9 * c
    elif P.grid.m == 2:
        lo = max(P.rho_lo[0], P.V - P.rho_hi[1])
        hi = min(P.rho_hi[0], P.V - P.rho_lo[1])
        cf = lambda t: kkt.compliance(P.grid, P.Ke, np.array([t, P.V - t]), P.f)
        gr = (np.sqrt(5.0) - 1.0) / 2.0
        a, b = lo, hi
        for _ in range(200):
            x1, x2 = b - gr * (b - a), a + gr * (b - a)
            if cf(x1) < cf(x2):
                b = x2
            else:
                a = x1
        assert abs(c - cf(0.5 * (a + b))) <= 1e-7 * c
    else:
        lb, ub, rel_gap = kkt.certificate(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, d["rho"],
                                          d["u"])
        assert rel_gap <= 1e-6 and lb <= c * (1 + 1e-9)
