"""GPU test of ada_solve_noalloc, the solve whose workspace is the library's fixed per-GPU scratch:
its x and result equal ada_solve's (same kernels, caller workspace) bit for bit, on two calls in
a row (the second smaller, so that it runs on what the first left in the scratch), through the C
ABI; a shape beyond the scratch is refused with the sizes in the message."""
import ctypes

import numpy as np
import pytest

from paritycheck import check_berr
from paper_2007_11208_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ada():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_11208_amd import ada as _ada
    _ada.lib()
    return _ada


def T(a):
    return torch.from_numpy(np.asfortranarray(a)).to("cuda:0")


def call_noalloc(ada, A, B, **kw):
    """ada_solve_noalloc through ctypes (column-major device tensors)."""
    n, nrhs = B.shape
    X = torch.full((nrhs, n), float("nan"), dtype=torch.float64, device="cuda:0").t()
    o = ada.make_opts(**kw)
    res = ada.Result()
    torch.cuda.synchronize()
    A, B = ada._colmajor(A), ada._colmajor(B)
    rc = ada.lib().ada_solve_noalloc(ada.context(0).handle, n, nrhs, A.data_ptr(), ada._ld(A), B.data_ptr(),
                                     ada._ld(B), X.data_ptr(), ada._ld(X), ctypes.byref(o), ctypes.byref(res),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, X, res


def same(ada, a, b, **kw):
    A, B = T(a), T(b)
    print(f"noalloc case n={a.shape[0]} nrhs={b.shape[1]} {kw}", flush=True)
    rc, X, res = call_noalloc(ada, A, B, **kw)
    assert rc == 0, ada.last_error()
    x_ref, r_ref = ada.solve(A, B, **kw)
    torch.cuda.synchronize()
    assert torch.equal(X, x_ref), "x differs from ada_solve's"
    r = ada._result(res, rc)
    assert (r.cls, r.kl, r.ku, r.route, r.fallback, r.info, r.rank) == \
        (r_ref.cls, r_ref.kl, r_ref.ku, r_ref.route, r_ref.fallback, r_ref.info, r_ref.rank)
    assert r.rcond == r_ref.rcond and r.berr == r_ref.berr
    assert check_berr(r.berr, a, b, X.cpu().numpy()) <= 1e-12
    return r


def test_noalloc_matches_solve_twice_second_smaller(ada):
    rng = np.random.default_rng(71)
    a1 = W.dense_general(1500, rng)
    b1 = W.rhs_for(a1, W.x_true(1500, 3, rng))
    r1 = same(ada, a1, b1)
    assert r1.route == "lu"
    a2 = W.spd(333, rng)
    b2 = W.rhs_for(a2, W.x_true(333, 2, rng))
    r2 = same(ada, a2, b2)
    assert r2.route == "chol"


def test_noalloc_other_routes(ada):
    rng = np.random.default_rng(72)
    for a in (W.banded_dense(2000, 3, 2, rng), W.triangular(700, rng, upper=False, scaled=True),
              W.ill_conditioned(200, rng, 1e-18)):
        b = W.rhs_for(a, W.x_true(a.shape[0], 1, rng))
        same(ada, a, b)


def test_noalloc_rejects_shapes_beyond_the_scratch(ada):
    n = 4000
    a = np.eye(n)
    rc, _, _ = call_noalloc(ada, T(a), T(np.ones((n, 1))))
    assert rc == ada.ERR_ARG
    msg = ada.last_error()
    assert "ada_solve_noalloc" in msg and str(ada.NOALLOC_SCRATCH_BYTES) in msg
