"""GPU parity of the routes the paper names as future work (Section V), selected with the
extension option: plain symmetric matrices by Bunch-Kaufman LDL^T. The oracle runs the same option.
Tridiagonal matrices take the band route.

Bars: class, band widths, route, Cholesky failure, fallback reason and info exact; rcond within
a factor 2 of the oracle's (same estimator; the GPU's blocked LDL^T sums in another order and
may take another pivot at a near tie, which changes the factors but not the matrix they
represent); backward error <= 1e-12; x within 32 n kappa eps |x| of the oracle's.
Without the option the paper's routes run (LU for these matrices).
"""
import numpy as np
import pytest

import oracle
from paritycheck import check_berr
from paper_2007_11208_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
O = oracle.get()
GiB = 1 << 30


@pytest.fixture(scope="module")
def ada():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_11208_amd import ada as _ada
    _ada.lib()
    return _ada


def T(a):
    return torch.from_numpy(np.asfortranarray(a)).to("cuda:0")


def sym_case(n, rng, diag_scale=1.0):
    a = rng.standard_normal((n, n))
    a[np.diag_indices(n)] *= diag_scale
    return np.asfortranarray(a + a.T)


def check(ada, a, b, ext, oext, layout="dense", kl_in=0, ku_in=0):
    n = b.shape[0]
    print(f"case n={n} nrhs={b.shape[1]} ext={ext} layout={layout}", flush=True)
    x, r = ada.solve(T(a), T(b), extensions=ext, layout=layout, kl_in=kl_in, ku_in=ku_in, raise_on_error=False)
    torch.cuda.synchronize()
    if layout == "band":
        xr, rr = O.solve_band(a, kl_in, ku_in, b, ext=oext)
    else:
        xr, rr = O.solve(a, b, ext=oext)
    assert r.status == rr["status"] == 0, (r.status, ada.last_error())
    assert r.cls == ada.CLASS_NAMES[rr["cls"]] and (r.kl, r.ku) == (rr["kl"], rr["ku"])
    assert r.route == ada.ROUTE_NAMES[rr["route"]], (r, rr)
    assert r.chol_failed == bool(rr["chol_failed"]) and r.fallback == rr["fallback"]
    if rr["fallback"] == 0:
        assert 0.5 * rr["rcond"] <= r.rcond <= 2.0 * rr["rcond"], (r.rcond, rr["rcond"])
        xg = x.cpu().numpy().reshape(xr.shape)
        eta = check_berr(r.berr, a, b, xg, band=(kl_in, ku_in) if layout == "band" else None)
        assert eta <= max(1e-12, 2.0 * rr["berr"]), (eta, rr["berr"])
        kappa = 1.0 / max(rr["rcond"], 1e-300)
        tol = 32 * n * kappa * EPS * max(1.0, float(np.max(np.abs(xr))))
        assert float(np.max(np.abs(xg - xr))) <= tol
    else:
        assert r.info == rr["info"] and r.rank == rr["rank"]
    return r


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 64, 65, 130, 511, 1000, 2050])
def test_ldlt_plain_symmetric(ada, n):
    rng = np.random.default_rng(500 + n)
    # a small diagonal makes most pivots 2x2 (and 1x1 interchanges), across panel edges
    a = sym_case(n, rng, diag_scale=0.05 if n % 2 else 1.0)
    b = W.rhs_for(a, W.x_true(n, 3, rng))
    r = check(ada, a, b, ("sym",), oracle.EXT_SYM)
    if n >= 3:
        assert r.cls == "sym" and r.route == "ldlt"


def test_ldlt_many_rhs_and_ragged_panels(ada):
    rng = np.random.default_rng(7)
    for n in (97, 257, 1501):
        a = sym_case(n, rng, diag_scale=0.01)
        b = W.rhs_for(a, W.x_true(n, 70, rng))
        r = check(ada, a, b, ("sym",), oracle.EXT_SYM)
        assert r.route == "ldlt"


def test_ldlt_after_cholesky_failure(ada):
    """Passes the sympd heuristic, Cholesky fails: LDL^T instead of LU with the option."""
    for n in (300, 1200):
        a = W.sym_indefinite(n, np.random.default_rng(n))
        b = W.rhs_for(a, W.x_true(n, 2, np.random.default_rng(n + 1)))
        r = check(ada, a, b, ("sym",), oracle.EXT_SYM)
        assert r.chol_failed and r.route == "ldlt"
        r0 = check(ada, a, b, (), 0)
        assert r0.chol_failed and r0.route == "lu"


def test_ldlt_zero_pivot_goes_to_svd(ada):
    rng = np.random.default_rng(8)
    n = 90
    a = sym_case(n, rng)
    a[40, :] = 0.0
    a[:, 40] = 0.0
    b = W.rhs_for(a, W.x_true(n, 1, rng))
    r = check(ada, a, b, ("sym",), oracle.EXT_SYM)
    assert r.route == "svd" and r.fallback == 1


def test_not_exactly_symmetric_stays_general(ada):
    rng = np.random.default_rng(9)
    a = sym_case(200, rng)
    a[150, 3] = np.nextafter(a[150, 3], np.inf)
    b = W.rhs_for(a, W.x_true(200, 1, rng))
    r = check(ada, a, b, ("sym",), oracle.EXT_SYM)
    assert r.cls == "general" and r.route == "lu"


def test_paper_routes_without_the_option(ada):
    rng = np.random.default_rng(10)
    a = sym_case(300, rng, 0.05)
    b = W.rhs_for(a, W.x_true(300, 2, rng))
    r = check(ada, a, b, (), 0)
    assert r.cls == "general" and r.route == "lu"


def tridiag_band(n, rng):
    ab = np.zeros((3, n))
    ab[0, 1:] = rng.standard_normal(n - 1)
    ab[1] = rng.standard_normal(n)
    ab[2, :-1] = rng.standard_normal(n - 1)
    return np.asfortranarray(ab)


@pytest.mark.parametrize("n", [12, 13, 100, 5000, 200_000])
def test_tridiagonal_takes_the_band_route(ada, n):
    """Tridiagonal matrices (kl = ku = 1) have no route of their own: the band LU, as the oracle."""
    rng = np.random.default_rng(600 + n)
    ab = tridiag_band(n, rng)
    b = np.asfortranarray(rng.standard_normal((n, 2)))
    r = check(ada, ab, b, (), 0, layout="band", kl_in=1, ku_in=1)
    assert r.route == "band_lu"
    if n <= 5000:
        dense = np.diag(ab[1]) + np.diag(ab[2, :-1], -1) + np.diag(ab[0, 1:], 1)
        r2 = check(ada, np.asfortranarray(dense), b, (), 0)
        assert r2.route == ("band_lu" if r2.cls == "banded" else "lu")


def test_unknown_extension_bits_are_rejected(ada):
    import torch
    A = torch.eye(4, dtype=torch.float64, device="cuda:0")
    B = torch.ones((4, 1), dtype=torch.float64, device="cuda:0")
    o = ada.make_opts()
    o.extensions = 2
    X = torch.empty_like(B)
    ws = ada.workspace_size(4, 1, ada.make_opts())
    work = torch.empty(ws, dtype=torch.uint8, device="cuda:0")
    res = ada.Result()
    import ctypes
    rc = ada.lib().ada_solve(ada.context(0).handle, 4, 1, A.data_ptr(), 4, B.data_ptr(), 4, X.data_ptr(), 4,
                             work.data_ptr(), work.numel(), ctypes.byref(o), ctypes.byref(res), None)
    assert rc == ada.ERR_ARG and "unknown extension bits" in ada.last_error()


def test_batched_rejects_extensions(ada):
    a = np.eye(4)
    bt = ada.Batch([a], [np.ones(4)], extensions=("sym",))
    with pytest.raises(ada.AdaError):
        bt.run()


def test_server_keeps_ldlt_factors(ada):
    rng = np.random.default_rng(11)
    srv = ada.Server(2 * GiB, solve_workers=2)
    try:
        a = sym_case(700, rng, 0.05)
        b = W.rhs_for(a, W.x_true(700, 2, rng))
        rc, r, X, f, _, _ = srv.poll(srv.submit(T(a), T(b), keep=True, extensions=("sym",)))
        assert rc == 0 and f != 0 and r.route == "ldlt", (rc, ada.last_error())
        # a small system with the option takes a solve worker, not the batch (paper routes only)
        s = sym_case(60, rng, 0.05)
        bs = W.rhs_for(s, W.x_true(60, 1, rng))
        rc, rs, _, _, _, _ = srv.poll(srv.submit(T(s), T(bs), extensions=("sym",)))
        assert rc == 0 and rs.route == "ldlt"
        for nr in (1, 4):
            b2 = W.rhs_for(a, W.x_true(700, nr, rng))
            rc, r2, X2, _, _, _ = srv.poll(srv.submit(None, T(b2), reuse=f))
            assert rc == 0 and r2.route == "ldlt"
            xr, rr = O.solve(a, b2, ext=oracle.EXT_SYM)
            kappa = 1.0 / rr["rcond"]
            tol = 32 * 700 * kappa * EPS * max(1.0, float(np.max(np.abs(xr))))
            assert float(np.max(np.abs(X2.cpu().numpy().reshape(xr.shape) - xr))) <= tol
            assert check_berr(r2.berr, a, b2, X2.cpu().numpy()) <= 1e-12
        srv.release(f)
    finally:
        srv.close()
