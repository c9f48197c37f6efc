"""Parity at the full sizes of the 128x64x64 bridge and the 192x96x96
cantilever, in the launch configuration the library uses for them: sampled
outputs that the oracle computes node by node (K(rho)x, the S-apply), and
properties that hold at any size (V-cycle symmetry and positivity, bitwise
repeatability, MINRES residual reduction)."""
import numpy as np
import pytest

import workloads as W
from oracle import fe, pbm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1904_06556_amd import vts as V  # noqa: E402


def say(*a):
    print("[fullsize]", *a, flush=True)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def sample_nodes(pr, count, seed):
    """Seeded node sample including the grid's corners and edges."""
    NX, NY, NZ = pr.nx + 1, pr.ny + 1, pr.nz + 1
    rng = np.random.default_rng(seed)
    pick = list(rng.integers(0, NX * NY * NZ, size=count))
    for i in (0, NX - 1):
        for j in (0, NY - 1):
            for k in (0, NZ - 1):
                pick.append(i + NX * (j + NY * k))
    return np.unique(np.array(pick, dtype=np.int64))


def adjacent(pr, n):
    """(element index, local node index) of the elements around node n; local
    node a = ax + 2 ay + 4 az as in the oracle's connectivity."""
    NX, NY = pr.nx + 1, pr.ny + 1
    i, j, k = n % NX, (n // NX) % NY, n // (NX * NY)
    out = []
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                ei, ej, ek = i - ax, j - ay, k - az
                if 0 <= ei < pr.nx and 0 <= ej < pr.ny and 0 <= ek < pr.nz:
                    out.append((ei + pr.nx * (ej + pr.ny * ek), ax + 2 * ay + 4 * az))
    return out


def elem_dofs(pr, e):
    NX, NY = pr.nx + 1, pr.ny + 1
    ei, ej, ek = e % pr.nx, (e // pr.nx) % pr.ny, e // (pr.nx * pr.ny)
    nodes = [(ei + (a & 1)) + NX * ((ej + ((a >> 1) & 1)) + NY * (ek + (a >> 2)))
             for a in range(8)]
    return np.array([3 * nd + c for nd in nodes for c in range(3)])


def k_rows(pr, Ke, rho, x, nodes):
    """(K(rho) x) at the sampled nodes, element by element, masked."""
    xm = np.where(pr.fixed == 1, 0.0, x)
    out = np.zeros((len(nodes), 3))
    for r, n in enumerate(nodes):
        for e, a in adjacent(pr, n):
            d = elem_dofs(pr, e)
            out[r] += rho[e] * (Ke[3 * a:3 * a + 3] @ xm[d])
    for c in range(3):
        out[pr.fixed[3 * nodes + c] == 1, c] = 0.0
    return out


CASES = {"bridge-128x64x64": 2, "cant3pt-192x96x96": 3}


@pytest.mark.parametrize("case", list(CASES))
def test_apply_K_sampled(case):
    pr = W.config(CASES[case])
    say("apply_K", case, "n_dof", pr.n_dof)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    rho = W.random_rho(pr.m, seed=7)
    x = W.random_vector(pr.n_dof, seed=8)
    ctx.set_rho(dev(rho))
    y = torch.empty(pr.n_dof, dtype=torch.float64, device="cuda")
    ctx.apply_K(dev(x), y)
    y2 = torch.empty_like(y)
    ctx.apply_K(dev(x), y2)
    assert torch.equal(y, y2)
    nodes = sample_nodes(pr, 300, seed=9)
    ref = k_rows(pr, Ke, rho, x, nodes)
    got = host(y).reshape(-1, 3)[nodes]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale
    # FP32 operator
    yf = torch.empty(pr.n_dof, dtype=torch.float32, device="cuda")
    ctx.apply_K_f32(dev(x, torch.float32), yf)
    gotf = host(yf).reshape(-1, 3)[nodes]
    assert np.max(np.abs(gotf - ref)) <= 2e-5 * scale
    ctx.close()


def _setup_state(ctx, pr, seed):
    """A PBM state away from the initial point: random u, rho, multipliers."""
    rng = np.random.default_rng(seed)
    st = pbm.initial_state(pr.n_dof, pr.m, pr.V)
    st.u = np.where(pr.fixed == 1, 0.0, rng.uniform(-1, 1, pr.n_dof)) * 1e-1
    st.rho = rng.uniform(0.05, 0.9, pr.m)
    st.alpha = 0.7
    st.p = np.full(pr.m, 0.05)
    d = dict(u=st.u, alpha=st.alpha, nu_lo=st.nu_lo, nu_hi=st.nu_hi, rho=st.rho,
             mu_lo=st.mu_lo, mu_hi=st.mu_hi, p=st.p, q_lo=st.q_lo, q_hi=st.q_hi,
             eps_nwt=1.0, eps_mr=1e-3)
    ctx.set_state(V.Context.pack_state(d, ctx.n_dof, ctx.m))
    return st


@pytest.mark.parametrize("case,prec", [("bridge-128x64x64", V.VTS_MIXED),
                                       ("bridge-128x64x64", V.VTS_FP64),
                                       ("cant3pt-192x96x96", V.VTS_MIXED)])
def test_S_and_vcycle_properties(case, prec):
    pr = W.config(CASES[case])
    say("S/V-cycle", case, "precision", prec)
    ctx = V.Context.from_problem(pr, precision=prec)
    st = _setup_state(ctx, pr, seed=3)
    ctx.newton_setup()
    P = pbm.VTS(pr)
    ev = pbm.evaluate(P, st)
    w, _, _ = pbm.schur_weights(ev)
    assert np.max(np.abs(host(ctx.vector("w")) - w)) <= 1e-12 * np.max(np.abs(w))
    nv = pr.n_dof + 1
    rng = np.random.default_rng(4)
    x = rng.standard_normal(nv)
    x[:-1][pr.fixed == 1] = 0.0
    y = torch.empty(nv, dtype=torch.float64, device="cuda")
    ctx.apply_S(dev(x), y)
    ys = host(y)
    # sampled rows of S x: K(rho') x + sum_e w_e b_e (b_e . x_e - beta)
    Ke = P.Ke
    nodes = sample_nodes(pr, 120, seed=5)
    ref = k_rows(pr, Ke, ev.rho1, x[:-1], nodes)
    um = np.where(pr.fixed == 1, 0.0, st.u)
    xm = np.where(pr.fixed == 1, 0.0, x[:-1])
    for r, n in enumerate(nodes):
        for e, a in adjacent(pr, n):
            d = elem_dofs(pr, e)
            b = Ke @ um[d]
            ref[r] += w[e] * b[3 * a:3 * a + 3] * (b @ xm[d] - x[-1])
        for c in range(3):
            if pr.fixed[3 * n + c]:
                ref[r, c] = 0.0
    got = ys[:-1].reshape(-1, 3)[nodes]
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
    # V-cycle: symmetric, positive, repeatable
    a = rng.standard_normal(nv)
    b = rng.standard_normal(nv)
    for v in (a, b):
        v[:-1][pr.fixed == 1] = 0.0
    Ma = torch.empty(nv, dtype=torch.float64, device="cuda")
    Mb = torch.empty_like(Ma)
    Ma2 = torch.empty_like(Ma)
    ctx.precondition(dev(a), Ma)
    ctx.precondition(dev(b), Mb)
    ctx.precondition(dev(a), Ma2)
    assert torch.equal(Ma, Ma2)
    ab, ba = float(np.dot(a, host(Mb))), float(np.dot(host(Ma), b))
    tol = 1e-9 if prec == V.VTS_FP64 else 2e-4
    assert abs(ab - ba) <= tol * np.sqrt(abs(np.dot(a, host(Ma))) * abs(np.dot(b, host(Mb))))
    assert np.dot(a, host(Ma)) > 0 and np.dot(b, host(Mb)) > 0
    # MINRES: the reduced Newton system solved to 1e-6 (M^-1 norm) has a
    # small true residual
    lin = ctx.solve_newton(1e-6)
    dy = ctx.vector("dy")
    Sd = torch.empty(nv, dtype=torch.float64, device="cuda")
    ctx.apply_S(dy, Sd)
    rhs = host(ctx.vector("rhs"))
    res = np.linalg.norm(host(Sd) - rhs) / np.linalg.norm(rhs)
    say("MINRES iterations", lin["iterations"], "true residual", res)
    assert lin["iterations"] < 500 and res < 1e-2
    ctx.close()
