"""The allocation-free S-apply (vts_apply_S_noalloc, static device workspace)
against vts_apply_S through the C ABI: bitwise equal outputs on two calls in
a row, the second on a smaller problem; out-of-order use is rejected."""
import sys

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_06556_amd import vts as V   # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(pr, seed):
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    ctx.newton_setup()
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = (torch.rand(ctx.n_dof + 1, generator=g, dtype=torch.float64) - 0.5).cuda()
    y_ref = torch.empty_like(x)
    y_new = torch.full_like(x, float("nan"))
    ctx.apply_S(x, y_ref)
    ctx.apply_S_noalloc(x, y_new)
    torch.cuda.synchronize()
    return ctx, y_ref.cpu().numpy(), y_new.cpu().numpy()


def test_noalloc_equals_apply_S_twice_second_smaller():
    big = W.config(1)                              # 64x32x32, several hundred workgroups
    small = W.cantilever_edge(16, 8, 8, 3)
    for pr, seed in ((big, 1), (small, 2)):
        say("apply_S_noalloc", pr.name)
        ctx, ref, new = _pair(pr, seed)
        assert np.array_equal(ref, new), np.max(np.abs(ref - new))
        ctx.close()


def test_noalloc_before_setup_is_state_error():
    pr = W.config(0)
    say("apply_S_noalloc before setup", pr.name)
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
    x = torch.zeros(ctx.n_dof + 1, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(V.VtsError) as ei:
        ctx.apply_S_noalloc(x, y)
    assert ei.value.status == V.VTS_ESTATE
    ctx.close()
