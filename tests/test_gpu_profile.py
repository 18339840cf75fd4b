"""Kernel-family timing (ada_profile_enable / ada_profile_families): the events bracket the launches of
the selected families only, and the timed launches of a routed solve are the ones its route makes."""
import numpy as np
import pytest

from paper_2007_11208_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ada():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_11208_amd import ada as mod
    return mod


def test_profile_families_select_the_timed_launches(ada):
    rng = np.random.default_rng(31)
    n = 700  # six 128-column panels, several workgroups each
    a = W.dense_general(n, rng)
    b = W.rhs_for(a, W.x_true(n, 1, rng))
    A = torch.from_numpy(np.asarray(a)).cuda()
    B = torch.from_numpy(np.asarray(b)).cuda()
    ctx = ada.Context(0)
    ctx.profile_reset()
    ctx.profile(True, families=["panel"])
    _, r = ada.solve(A, B, ctx=ctx)
    torch.cuda.synchronize()
    ctx.profile(False)
    p = ctx.profile_all()
    assert r.route == "lu"
    assert p["panel"][0] == 6 and p["panel"][1] > 0.0, p["panel"]
    assert all(v[0] == 0 for f, v in p.items() if f != "panel"), p
    # every family: the same solve also times its updates and its triangular solves
    ctx.profile_reset()
    ctx.profile(True)
    _, r2 = ada.solve(A, B, ctx=ctx)
    torch.cuda.synchronize()
    ctx.profile(False)
    p2 = ctx.profile_all()
    assert r2.route == "lu" and r2.berr == r.berr
    assert p2["panel"][0] == 6 and p2["gemm"][0] > 0 and p2["trsv"][0] > 0, p2
    # profiling off: nothing accumulates
    ctx.profile_reset()
    ada.solve(A, B, ctx=ctx)
    torch.cuda.synchronize()
    assert all(v[0] == 0 for v in ctx.profile_all().values())
