"""Several load cases on the GPU (vts_problem.nload) against the multi-load
oracle (oracle/multiload.py) on the same seeded inputs: the evaluation, the
gradient and the reduced right-hand side, the batched K(rho) on k vectors,
the S-apply of the stacked system (3.12), one V-cycle with 3k x 3k node
blocks (FP64, 1e-10), one Newton step, and whole solves (KKT <= 1e-6 from
the returned (rho, U, alpha) on the host, compliance against the oracle's
run), and a checkpoint round trip.  Cases k = 2, 3 and 4 (node blocks of 6, 9
and 12) on 1- to 3-level
hierarchies, the benchmark's two-case 64x32x32 cantilever for the
operators, and the proportional-cases property (f, c f) == one load
sqrt(1 + c^2) f on the GPU itself."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fe, mg, pbm
from oracle import multiload as ML

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def three_loads(nx, ny, nz, levels):
    """The two end-edge cases plus a seeded third case on the top face."""
    pr = W.cantilever_two_loads(nx, ny, nz, levels)
    rng = np.random.default_rng(7)
    third = np.zeros(pr.n_dof)
    top = np.nonzero(np.arange(pr.n_nodes) // ((nx + 1) * (ny + 1)) == nz)[0]
    third[3 * top + 0] = rng.uniform(-1.0, 1.0, top.size)
    return W.with_load_cases(pr, [*W.load_cases(pr), third], name=f"cant3load-{nx}x{ny}x{nz}")


def four_loads(nx, ny, nz, levels):
    """The three cases above plus a seeded fourth on the top face (z)."""
    pr = three_loads(nx, ny, nz, levels)
    rng = np.random.default_rng(8)
    fourth = np.zeros(pr.n_dof)
    top = np.nonzero(np.arange(pr.n_nodes) // ((nx + 1) * (ny + 1)) == nz)[0]
    fourth[3 * top + 2] = rng.uniform(-1.0, 0.0, top.size)
    return W.with_load_cases(pr, [*W.load_cases(pr), fourth], name=f"cant4load-{nx}x{ny}x{nz}")


CASES = {
    "k2-8x4x4-l3": lambda: W.cantilever_two_loads(8, 4, 4, 3),
    "k4-8x4x4-l2": lambda: four_loads(8, 4, 4, 2),
    "k2-8x4x4-l1": lambda: W.cantilever_two_loads(8, 4, 4, 1),
    "k3-8x4x4-l2": lambda: three_loads(8, 4, 4, 2),
    "k2-16x8x8-l3": lambda: W.multi_config(0),
}


def _state(P, seed):
    rng = np.random.default_rng(seed)
    m = P.grid.m
    st = ML.initial_state(P)
    st.u = np.stack([P.grid.mask(0.5 * rng.standard_normal(P.grid.n_dof)) for _ in range(P.k)])
    st.alpha = 0.3
    st.nu_lo = 0.05 * rng.random(m)
    st.nu_hi = 0.05 * rng.random(m)
    st.rho = rng.uniform(0.05, 1.0, m)
    st.mu_lo = rng.uniform(0.5, 1.5, m)
    st.mu_hi = rng.uniform(0.5, 1.5, m)
    st.p = np.full(m, 0.1)
    st.q_lo = np.full(m, 0.1)
    st.q_hi = np.full(m, 0.1)
    return st


def _push(ctx, st, eps_mr=1e-3):
    d = dict(u=st.u.ravel(), alpha=st.alpha, nu_lo=st.nu_lo, nu_hi=st.nu_hi, rho=st.rho,
             mu_lo=st.mu_lo, mu_hi=st.mu_hi, p=st.p, q_lo=st.q_lo, q_hi=st.q_hi,
             eps_nwt=1.0, eps_mr=eps_mr)
    ctx.set_state(V.Context.pack_state(d, ctx.n_vec, ctx.m))


def _stacked_all(P, y):
    """stacked free vector (k n + 1) -> the GPU layout (k n_dof + 1)"""
    out = np.zeros(P.k * P.grid.n_dof + 1)
    for l in range(P.k):
        out[l * P.grid.n_dof + P.free] = y[l * P.n:(l + 1) * P.n]
    out[-1] = y[-1]
    return out


@pytest.mark.parametrize("case", list(CASES))
def test_multiload_setup_operators_and_vcycle(case):
    pr = CASES[case]()
    P = ML.MultiVTS(pr)
    say("multi-load setup", case, "k", P.k, "levels", pr.levels)
    st = _state(P, seed=5)
    ev = ML.evaluate(P, st)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    assert ctx.nload == P.k and ctx.n_vec == P.k * P.grid.n_dof
    _push(ctx, st)
    ctx.newton_setup()
    assert rel(host(ctx.vector("energy")), ev.e) < 1e-12
    assert rel(host(ctx.vector("g1")), ev.g1.ravel()) < 1e-11
    assert rel(host(ctx.vector("rhs")), _stacked_all(P, ML.reduced_rhs(P, ev))) < 1e-11
    # S of the stacked system, matrix-free against the oracle's
    rng = np.random.default_rng(9)
    X = np.stack([P.grid.mask(rng.standard_normal(P.grid.n_dof)) for _ in range(P.k)])
    beta = 0.37
    Yo, yao = ML.schur_apply(P, ev, X, beta)
    y = torch.empty(ctx.n_vec + 1, dtype=torch.float64, device="cuda")
    ctx.apply_S(dev(np.concatenate([X.ravel(), [beta]])), y)
    yh = host(y)
    assert rel(yh[:-1], Yo.ravel()) < 1e-11
    assert abs(yh[-1] - yao) < 1e-11 * max(abs(yao), np.abs(Yo).max())
    # batched K(rho) on the k cases (fixed entries of x non-zero: masked on read)
    rho = W.random_rho(pr.m, seed=3)
    Xr = np.concatenate([W.random_vector(pr.n_dof, seed=4 + l) for l in range(P.k)])
    yk = torch.empty(ctx.n_vec, dtype=torch.float64, device="cuda")
    ctx.apply_K_rho(dev(rho), dev(Xr), yk)
    yko = np.concatenate([fe.apply_K(P.grid, P.Ke, rho, Xr[l * pr.n_dof:(l + 1) * pr.n_dof])
                          for l in range(P.k)])
    assert rel(host(yk), yko) < 1e-12
    # one V-cycle with node blocks over all cases, FP64, bitwise repeatable
    S = ML.schur_matrix(P, ev)
    H = mg.Hierarchy(P.grid, S, pr.levels, nload=P.k)
    r = np.random.default_rng(11).standard_normal(S.shape[0])
    z = torch.empty(ctx.n_vec + 1, dtype=torch.float64, device="cuda")
    ctx.precondition(dev(_stacked_all(P, r)), z)
    err = rel(host(z), _stacked_all(P, H.vcycle(r)))
    say("  V-cycle rel", err)
    assert err < 1e-10
    z2 = torch.empty_like(z)
    ctx.precondition(dev(_stacked_all(P, r)), z2)
    assert torch.equal(z, z2)
    ctx.close()


def test_multiload_newton_step_matches_oracle():
    pr = W.cantilever_two_loads(8, 4, 4, 3)
    say("multi-load Newton step", pr.name)
    P = ML.MultiVTS(pr)
    st = _state(P, seed=31)
    st.p = np.full(P.grid.m, 0.3)
    solver = ML.Solver(pr, pbm.Options(eps_mr0=1e-6))
    solver.eps_mr = 1e-6
    new, ev = solver.newton(st.copy(), eps_nwt=1e9)          # exactly one step
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64,
                                 options=V.default_options(eps_mr0=1e-6))
    _push(ctx, st, eps_mr=1e-6)
    ns = ctx.newton_step()
    g = ctx.state_dict()
    assert abs(ns["minres_its"] - solver.log.newton[-1]["minres"]) <= 1
    assert ns["kappa"] == solver.log.newton[-1]["kappa"]
    assert rel(g["u"], new.u.ravel()) < 1e-8
    assert abs(g["alpha"] - new.alpha) < 1e-8 * abs(new.alpha)
    assert rel(g["nu_lo"], new.nu_lo) < 1e-7
    assert abs(ns["res_pbm"] - solver.log.newton[-1]["res"]) < 1e-7 * solver.log.newton[-1]["res"]
    ctx.close()


@pytest.mark.parametrize("case", ["k2-8x4x4-l3", "k3-8x4x4-l2"])
def test_multiload_solve_matches_oracle(case):
    pr = CASES[case]()
    P = ML.MultiVTS(pr)
    say("multi-load PBM solve", case)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    res = ctx.pbm_solve()
    d = ctx.state_dict()
    U = d["u"].reshape(P.k, P.grid.n_dof)
    r = ML.kkt_residual(P, d["rho"], U, d["alpha"])
    say("  GPU", res["outer"], res["newton"], res["minres"], "kkt", r["kkt"])
    assert res["status"] == 0 and r["kkt"] <= 1e-6, r
    s = ML.Solver(pr)
    so = s.solve()
    say("  oracle", len(s.log.outer), len(s.log.newton),
        sum(x["minres"] for x in s.log.newton), "kkt", s.kkt["kkt"])
    c_gpu = ML.compliance(P, d["rho"])
    c_or = ML.compliance(P, so.rho)
    assert c_gpu == pytest.approx(c_or, rel=1e-6)
    assert res["compliance"] == pytest.approx(0.5 * float(np.sum(P.F * U)), rel=1e-12)
    # weak duality on the GPU's displacement (Theorem 2 on the stacked problem)
    lb = ML.dual_lower_bound(P, U)
    assert lb <= c_or * (1 + 1e-9) and lb == pytest.approx(c_or, rel=1e-6)
    assert res["outer"] == len(s.log.outer)
    assert res["newton"] == len(s.log.newton)
    ctx.close()


def test_proportional_cases_equal_one_scaled_load_on_gpu():
    """Cases (f, c f) and the one load sqrt(1 + c^2) f have the same iterates
    in exact arithmetic (the map x -> (x, c x)/sqrt(1 + c^2) commutes with
    every step), on the benchmark's multi-load grid."""
    c = 0.5
    base = W.cantilever_edge(64, 32, 32, 5, vol_frac=0.2)
    s = math.sqrt(1.0 + c * c)
    multi = W.with_load_cases(base, [base.f, c * base.f])
    say("proportional cases", base.name)
    opts = V.default_options(eps_mr0=1e-4 * math.sqrt(pbm.VTS(base).n))
    a = V.Context(base.nx, base.ny, base.nz, base.levels, base.fixed, s * base.f, base.V,
                  base.rho_lo, base.rho_hi, precision=V.VTS_FP64, options=opts)
    b = V.Context.from_problem(multi, precision=V.VTS_FP64,
                               options=V.default_options(eps_mr0=1e-4 * math.sqrt(pbm.VTS(base).n)))
    ra, rb = a.pbm_solve(), b.pbm_solve()
    say("  one load", ra["outer"], ra["newton"], ra["minres"], " two cases", rb["outer"],
        rb["newton"], rb["minres"])
    assert ra["status"] == rb["status"] == 0
    assert ra["outer"] == rb["outer"] and ra["newton"] == rb["newton"]
    assert abs(ra["minres"] - rb["minres"]) <= 0.02 * ra["minres"] + 2
    da, db = a.state_dict(), b.state_dict()
    assert np.max(np.abs(da["rho"] - db["rho"])) < 1e-6
    assert rb["compliance"] == pytest.approx(ra["compliance"], rel=1e-8)
    U = db["u"].reshape(2, -1)
    assert np.max(np.abs(U[1] - c * U[0])) < 1e-8 * np.abs(U).max()
    a.close()
    b.close()


def test_multiload_full_size_batched_K_sampled_rows():
    """K(rho) on the three point-load cases of the 192x96x96 cantilever, the
    launch the benchmark times: sampled node rows against the definition."""
    pr = W.multi_config(2)
    say("batched K full size", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    rho = W.random_rho(pr.m, seed=1)
    X = np.concatenate([W.random_vector(pr.n_dof, seed=2 + l, fixed=pr.fixed) for l in range(3)])
    y = torch.empty(ctx.n_vec, dtype=torch.float64, device="cuda")
    ctx.apply_K_rho(dev(rho), dev(X), y)
    yh = host(y)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    rng = np.random.default_rng(0)
    nx, ny, nz = pr.nx, pr.ny, pr.nz
    NX, NY = nx + 1, ny + 1
    for n in rng.integers(0, pr.n_nodes, 200):
        i, j, k = n % NX, (n // NX) % NY, n // (NX * NY)
        for l in range(3):
            xl = X[l * pr.n_dof:(l + 1) * pr.n_dof]
            acc = np.zeros(3)
            for ez in (k - 1, k):
                for ey in (j - 1, j):
                    for ex in (i - 1, i):
                        if not (0 <= ex < nx and 0 <= ey < ny and 0 <= ez < nz):
                            continue
                        e = ex + nx * (ey + ny * ez)
                        a = (i - ex) + 2 * (j - ey) + 4 * (k - ez)
                        dofs = [3 * ((ex + (b & 1)) + NX * ((ey + ((b >> 1) & 1)) + NY * (ez + (b >> 2)))) + c
                                for b in range(8) for c in range(3)]
                        acc += rho[e] * (Ke[3 * a:3 * a + 3] @ xl[dofs])
            got = yh[l * pr.n_dof + 3 * n:l * pr.n_dof + 3 * n + 3]
            want = np.where(pr.fixed[3 * n:3 * n + 3] == 1, 0.0, acc)
            assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(acc).max()))
    ctx.close()


def test_multiload_argument_errors():
    pr = W.cantilever_two_loads(8, 4, 4, 3)
    f = W.load_cases(pr).ravel()
    with pytest.raises(V.VtsError) as ei:
        V.Context(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, f, pr.V, precision=V.VTS_MIXED,
                  nload=2)
    assert ei.value.status == V.VTS_EINVAL
    with pytest.raises(V.VtsError) as ei:
        V.Context(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, np.tile(f[:pr.n_dof], 5), pr.V,
                  nload=5)
    assert ei.value.status == V.VTS_EINVAL
    nan = f.copy()
    nan[pr.n_dof + np.nonzero(pr.fixed == 0)[0][0]] = np.nan     # the second case
    with pytest.raises(V.VtsError) as ei:
        V.Context(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, nan, pr.V, nload=2)
    assert ei.value.status == V.VTS_EINVAL
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    with pytest.raises(V.VtsError) as ei:
        ctx.ip_init()
    assert ei.value.status == V.VTS_EINVAL
    with pytest.raises(V.VtsError) as ei:
        ctx.doc_step(q=0.5, tau=1e-4, eps_doc=1e-3, eps_mr=1e-6)
    assert ei.value.status == V.VTS_EINVAL
    # before newton_setup the S-apply is out of order
    x = torch.zeros(ctx.n_vec + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VtsError) as ei:
        ctx.apply_S(x, torch.empty_like(x))
    assert ei.value.status == V.VTS_ESTATE
    ctx.close()


def test_multiload_checkpoint_resumes_bitwise():
    """vts_get_state / vts_set_state carry every case of u: a context resumed
    from a checkpoint takes the same Newton step as the original."""
    pr = W.cantilever_two_loads(8, 4, 4, 3)
    say("multi-load checkpoint", pr.name)
    a = V.Context.from_problem(pr, precision=V.VTS_FP64)
    a.newton_step()
    a.newton_step()
    buf = a.get_state()
    assert buf.size == 4 + a.n_vec + 1 + 8 * a.m + 5
    b = V.Context.from_problem(pr, precision=V.VTS_FP64)
    b.set_state(buf)
    sa, sb = a.newton_step(), b.newton_step()
    assert sa == sb
    assert np.array_equal(a.get_state(), b.get_state())
    a.close()
    b.close()
