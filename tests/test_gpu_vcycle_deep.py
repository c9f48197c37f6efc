"""One V-cycle of the HIP path against the oracle's (Section 6.1) on deep
hierarchies, where every intermediate level runs the multi-workgroup stored
stencil colour passes, residuals and restrictions of the device path, and the
finest level the matrix-free colour passes: cantilever 32x16x16 on 4 levels,
the 64x32x32 cantilever on 5.  A single-level 12x8x8 cantilever puts the
whole system (about 3000 unknowns) on the dense coarsest solver above the
size of the one-workgroup V-cycle.  FP64 to 1e-10 and bitwise repeatable;
mixed precision to 1e-3 of the FP64 cycle."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import pbm, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _state(P, seed):
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
    st.p = np.full(m, 0.1)
    st.q_lo = np.full(m, 0.1)
    st.q_hi = np.full(m, 0.1)
    return st


def _push(ctx, st):
    d = dict(u=st.u, alpha=st.alpha, nu_lo=st.nu_lo, nu_hi=st.nu_hi, rho=st.rho,
             mu_lo=st.mu_lo, mu_hi=st.mu_hi, p=st.p, q_lo=st.q_lo, q_hi=st.q_hi,
             eps_nwt=1.0, eps_mr=1e-3)
    ctx.set_state(V.Context.pack_state(d, ctx.n_dof, ctx.m))


def _sv(P, y):
    out = np.zeros(P.grid.n_dof + 1)
    out[P.free] = y[:-1]
    out[-1] = y[-1]
    return out


DEEP = {
    "cant-32x16x16-l4": lambda: W.cantilever_edge(32, 16, 16, 4),
    "cant-64x32x32-l5": lambda: W.cantilever_edge(64, 32, 32, 5, vol_frac=0.2),
    "cant-12x8x8-l1": lambda: W.cantilever_edge(12, 8, 8, 1),
}


@pytest.mark.parametrize("case", list(DEEP))
def test_vcycle_deep_hierarchy(case):
    pr = DEEP[case]()
    P = pbm.VTS(pr)
    st = _state(P, seed=41)
    ev = pbm.evaluate(P, st)
    S = pbm.schur_matrix(P, ev)
    H = mg.Hierarchy(P.grid, S, pr.levels)
    say("deep V-cycle", case, "levels", pr.levels, "unknowns", P.n + 1,
        "coarsest", H.levels[0].n + 1)
    r = np.random.default_rng(42).standard_normal(P.n + 1)
    zo = _sv(P, H.vcycle(r))
    for prec, tol in ((V.VTS_FP64, 1e-10), (V.VTS_MIXED, 1e-3)):
        ctx = V.Context.from_problem(pr, precision=prec)
        _push(ctx, st)
        ctx.newton_setup()
        z = torch.empty(P.grid.n_dof + 1, dtype=torch.float64, device="cuda")
        ctx.precondition(dev(_sv(P, r)), z)
        err = rel(host(z), zo)
        say("  precision", prec, "rel", err)
        assert err < tol
        z2 = torch.empty_like(z)
        ctx.precondition(dev(_sv(P, r)), z2)
        assert torch.equal(z, z2)
        ctx.close()
