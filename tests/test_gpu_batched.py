"""GPU parity of the batched solve (many small systems in one launch) against the oracle.

Same bars as the single-system parity tests: class and band widths bit-exact,
route / Cholesky failure / fallback reason exact outside a factor 4 of the rcond
threshold (systems inside it are reported), rcond within a factor 2, the
reported backward error equal to the oracle's on the GPU's x and <= 1e-12 (or
twice the oracle's for inconsistent least-squares systems), x within
32 n kappa eps |x| off the SVD route, SVD rank exact.
"""
import re

import numpy as np
import pytest

import oracle
from paper_2007_11208_amd import workloads as W
from paritycheck import check_berr, near_threshold, note_near_threshold

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
O = oracle.get()


@pytest.fixture(scope="module")
def ada():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_11208_amd import ada as _ada
    _ada.lib()
    return _ada


def check(ada, a, b, x, r, **okw):
    xr, rr = O.solve(a, b, **okw)
    assert r.status == rr["status"] or (rr["info"] == 0 and near_threshold(rr["rcond"])), (r, rr)
    if r.status not in (0, -3):
        return
    assert r.cls == ada.CLASS_NAMES[rr["cls"]], (r, rr)
    assert (r.kl, r.ku) == (rr["kl"], rr["ku"])
    xg = x.reshape(xr.shape)
    if rr["info"] == 0 and near_threshold(rr["rcond"]):
        note_near_threshold(f"n={a.shape[0]}", rr, r)
        if r.status == 0:
            check_berr(r.berr, a, b, xg)
        return
    assert r.route == ada.ROUTE_NAMES[rr["route"]], (r, rr)
    assert r.chol_failed == bool(rr["chol_failed"])
    assert r.fallback == rr["fallback"]
    if rr["fallback"] == 0:
        assert 0.5 * rr["rcond"] <= r.rcond <= 2.0 * rr["rcond"], (r.rcond, rr["rcond"])
    if r.status == 0:
        eta = check_berr(r.berr, a, b, xg)
        assert eta <= max(1e-12, 2.0 * rr["berr"]), (eta, rr["berr"])
        if r.route != "svd":
            kappa = 1.0 / max(rr["rcond"], 1e-300)
            tol = 32 * a.shape[0] * kappa * EPS * max(1.0, np.max(np.abs(xr)))
            assert np.max(np.abs(xg - xr)) <= tol
        else:
            assert r.rank == rr["rank"]


def test_batched_mix(ada):
    cases = W.batched_case(120, k=1, n_hi=192)
    As = [c[1] for c in cases]
    Bs = [c[2] for c in cases]
    xs, rs = ada.solve_batched(As, Bs)
    for (kind, a, b), x, r in zip(cases, xs, rs):
        print(f"{kind} n={a.shape[0]} nrhs={b.shape[1]} -> {r.cls}/{r.route}", flush=True)
        check(ada, a, b, x, r)


def test_batched_special_systems(ada):
    import json, os
    fig1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fig1.json")))
    sys_ = [np.array(fig1[k]["matrix"], dtype=np.float64) for k in ("a", "b", "c")]
    rng = np.random.default_rng(9)
    sys_ += [np.array([[3.0]]), np.array([[0.0, 1.0], [1.0, 0.0]]), W.sym_indefinite(200, rng),
             W.triangular(256, rng, upper=True), W.triangular(256, rng, upper=False, scaled=True),
             W.spd(256, rng), W.dense_general(256, rng), W.banded_dense(256, 3, 2, rng)]
    for name in W.SMALL_CASES:
        a, _ = W.small_case(name)
        if a.shape[0] <= 256:
            sys_.append(a)
    z = W.dense_general(40, rng)
    z[:, 7] = 0.0  # exactly singular: zero pivot -> SVD route
    sys_.append(z)
    Bs = [W.rhs_for(a, W.x_true(a.shape[0], 2, rng)) for a in sys_]
    xs, rs = ada.solve_batched(sys_, Bs)
    for a, b, x, r in zip(sys_, Bs, xs, rs):
        print(f"n={a.shape[0]} -> {r.cls}/{r.route} status={r.status}", flush=True)
        check(ada, a, b, x, r)


def test_batched_same_alone_and_in_the_mix(ada):
    cases = W.batched_case(40, k=2, n_hi=160)
    As = [c[1] for c in cases]
    Bs = [c[2] for c in cases]
    xs, rs = ada.solve_batched(As, Bs)
    for k in (0, 7, 23):
        x1, r1 = ada.solve_batched([As[k]], [Bs[k]])
        assert np.array_equal(x1[0], xs[k])
        assert (r1[0].route, r1[0].rcond, r1[0].berr) == (rs[k].route, rs[k].rcond, rs[k].berr)


def test_batched_errors_and_options(ada):
    rng = np.random.default_rng(4)
    big = W.dense_general(300, rng)
    nanm = W.dense_general(20, rng)
    nanm[3, 4] = np.nan
    ok = W.dense_general(30, rng)
    ill = W.ill_conditioned(64, rng, smin=1e-18)
    As = [big, nanm, ok, ill]
    Bs = [np.ones((300, 1)), np.ones((20, 1)), np.ones((30, 9)), np.ones((64, 1))]
    _, rs = ada.solve_batched(As, Bs)
    assert rs[0].status == ada.ERR_ARG
    assert rs[1].status == ada.ERR_NONFINITE
    assert rs[2].status == ada.ERR_ARG  # nrhs > 8
    assert rs[3].status == 0 and rs[3].route == "svd"
    _, rs2 = ada.solve_batched([ill], [np.ones((64, 1))], no_approx=True)
    assert rs2[0].status == ada.ERR_SINGULAR and rs2[0].fallback != 0
    x3, rs3 = ada.solve_batched([ok], [np.ones((30, 1))], force_general=True)
    assert rs3[0].route == "lu" and rs3[0].kl == -1
    assert np.allclose(ok @ x3[0], 1.0, atol=1e-10)


def test_batched_fp32_refined_mix(ada):
    """FP32 factors + FP64 refinement: same decisions as the FP64 oracle, backward error
    <= 1e-10 (the refined form's bar; the refinement itself stops at sqrt(n) eps)."""
    cases = W.batched_case(120, k=1, n_hi=256)
    As = [c[1] for c in cases]
    Bs = [c[2] for c in cases]
    xs, rs = ada.solve_batched(As, Bs, precision="fp32_ir")
    refined = 0
    for (kind, a, b), x, r in zip(cases, xs, rs):
        xr, rr = O.solve(a, b)
        print(f"{kind} n={a.shape[0]} nrhs={b.shape[1]} -> {r.cls}/{r.route} it={r.refine_iters}", flush=True)
        assert r.status == rr["status"] == 0
        assert r.cls == ada.CLASS_NAMES[rr["cls"]] and (r.kl, r.ku) == (rr["kl"], rr["ku"])
        eta = check_berr(r.berr, a, b, x.reshape(xr.shape))
        if rr["info"] == 0 and near_threshold(rr["rcond"]):
            note_near_threshold(f"{kind} n={a.shape[0]}", rr, r)
            continue
        assert r.route == ada.ROUTE_NAMES[rr["route"]], (r, rr)
        assert r.fallback == rr["fallback"]
        if r.route == "tri":
            assert r.refine_iters == 0
        elif r.route == "svd":
            assert r.refine_iters <= 0  # FP32 never reaches the fallback's systems; FP64 decided
        else:
            refined += r.refine_iters > 0
            assert 0.5 * rr["rcond"] <= r.rcond <= 2.0 * rr["rcond"], (r.rcond, rr["rcond"])
        if r.route != "svd":
            assert eta <= 1e-10, r
            kappa = 1.0 / max(rr["rcond"], 1e-300)
            tol = 32 * a.shape[0] * kappa * EPS * max(1.0, np.max(np.abs(xr)))
            assert np.max(np.abs(x.reshape(xr.shape) - xr)) <= tol
        else:
            assert r.rank == rr["rank"]
    assert refined > 0


def test_batched_fp32_refinement_falls_back_to_fp64(ada):
    """A system FP32 cannot factor usefully (kappa 1e10, or entries beyond the FP32 range) is
    handed to the FP64 route: x and the result equal the FP64 solve's bit for bit."""
    rng = np.random.default_rng(12)
    hard = W.prescribed_spectrum(96, np.logspace(0, -10, 96), rng)
    huge = W.dense_general(50, rng) * 1e40
    spd = W.spd(140, rng)
    ok = W.dense_general(200, rng)
    As = [hard, huge, spd, ok]
    Bs = [W.rhs_for(a, W.x_true(a.shape[0], 3, rng)) for a in As]
    x64, r64 = ada.solve_batched(As, Bs)
    x32, r32 = ada.solve_batched(As, Bs, precision="fp32_ir")
    for k in (0, 1):
        assert r32[k].refine_iters < 0, r32[k]
        assert np.array_equal(x32[k], x64[k])
        assert (r32[k].route, r32[k].rcond, r32[k].berr) == (r64[k].route, r64[k].rcond, r64[k].berr)
    for k in (2, 3):
        assert r32[k].refine_iters > 0 and r32[k].route == r64[k].route
        assert check_berr(r32[k].berr, As[k], Bs[k], x32[k]) <= 1e-10
    with pytest.raises(ValueError):
        ada.make_opts(precision="bf16")


def test_batched_launch_in_a_hip_graph(ada):
    """The batched launch captured into a HIP graph and replayed: every replay, with eager
    work and synchronisations between them, gives the eager run's x and results bit for bit."""
    cases = W.batched_case(64, k=5, n_hi=200)
    batch = ada.Batch([c[1] for c in cases], [c[2] for c in cases])
    batch.run()
    torch.cuda.synchronize()
    x_ref = batch.X.clone()
    r_ref = batch.res.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch.run()
    for rep in range(3):
        batch.X.zero_()
        batch.res.zero_()
        junk = torch.randn(1 << 20, device="cuda:0").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.X, x_ref), f"replay {rep}: x differs"
        assert torch.equal(batch.res, r_ref), f"replay {rep}: results differ"
        del junk


def test_batched_shapes_bit_identical_and_tuned(ada):
    """Every launch shape (ranges of orders, workgroups per compute unit, staging width) gives the same
    bits; the autotuner keeps one of them in its context, and the tuned run matches the oracle."""
    cases = W.batched_case(160, k=5, n_lo=8, n_hi=256)
    As = [c[1] for c in cases]
    Bs = [c[2] for c in cases]
    ctx = ada.Context(0)
    batch = ada.Batch(As, Bs, ctx=ctx)
    assert batch.shape() == {"max_n": [256], "wg_per_cu": [1], "workgroups": [256], "stage_cols": 8}
    batch.run()
    torch.cuda.synchronize()
    x_ref, r_ref = batch.X.clone(), batch.res.clone()
    shapes = [ada.batched_shape((256, 96), (1, 2)),
              ada.batched_shape((256, 128, 64), (1, 1, 2), stage_cols=4),
              ada.batched_shape((256, 64), (1, 1), workgroups=(37, 5)),
              ada.batched_shape((256, 200, 17), (1, 1, 2), workgroups=(1, 300, 512))]
    for sh in shapes:
        print("shape", sh.as_dict(), flush=True)
        batch.set_shape(sh)
        assert batch.shape() == sh.as_dict()
        batch.X.zero_()
        batch.res.zero_()
        batch.run()
        torch.cuda.synchronize()
        assert torch.equal(batch.X, x_ref), sh.as_dict()
        assert torch.equal(batch.res, r_ref), sh.as_dict()
    batch.set_shape(None)
    batch.X.zero_()
    batch.res.zero_()
    tuned, ms = batch.tune()
    torch.cuda.synchronize()
    print("tuned", tuned, f"{ms:.3f} ms", flush=True)
    assert ms > 0 and batch.shape() == tuned
    assert torch.equal(batch.X, x_ref) and torch.equal(batch.res, r_ref)
    # the other precision keeps its default
    b32 = ada.Batch(As[:4], Bs[:4], ctx=ctx, precision="fp32_ir")
    assert b32.shape()["max_n"] == [256] and len(b32.shape()["wg_per_cu"]) == 1
    batch.X.zero_()
    batch.run()
    xs, rs = batch.solutions(), batch.results()
    for (kind, a, b), x, r in zip(cases, xs, rs):
        check(ada, a, b, x, r)
    ctx.close()


def test_batched_shape_rejects(ada):
    ctx = ada.Context(0)
    batch = ada.Batch([np.eye(3)], [np.ones((3, 1))], ctx=ctx)
    bad = [(ada.batched_shape((200,)), "max_n[0] must be 256"),
           (ada.batched_shape((256, 128, 128)), "max_n must decrease"),
           (ada.batched_shape((256, 8)), "max_n must be >= 16"),
           (ada.batched_shape((256, 128), (1, 2)), "max_n <= 96"),
           (ada.batched_shape((256, 64), (1, 3)), "wg_per_cu must be 1 or 2"),
           (ada.batched_shape((256,), workgroups=(257,)), "workgroups out of range"),
           (ada.batched_shape((256,), stage_cols=16), "stage_cols must be 4 or 8")]
    for sh, msg in bad:
        with pytest.raises(ada.AdaError, match=re.escape(msg)):
            batch.set_shape(sh)
    assert batch.shape()["max_n"] == [256]
    ctx.close()
