"""GPU parity of the mixed-precision single solve (FP32 or BF16 trailing updates, FP64
iterative refinement) against the FP64 oracle.

Bars: class, band widths, route, Cholesky failure and fallback reason exact (the
decisions are FP64's); refined x has backward error <= sqrt(n) eps (the refinement's
stopping test; the stated bar for the refined form is 1e-10; BF16 factors are refined by
GMRES preconditioned with them), and x is within
32 n kappa eps |x| of the oracle's; rcond (estimated on the low-precision factors)
within a factor 2 of the oracle's (refined BF16 factors: at most twice the oracle's and at least
the 1e-9 refinement gate, since the BF16 factors' condition can exceed A's by orders of magnitude). A refinement that cannot converge (kappa beyond
what the operand precision supports) hands the system to the FP64 route: the result
then says so (refine_iters < 0) and meets the FP64 bars.
"""
import math

import numpy as np
import pytest

import oracle
from paritycheck import check_berr
from paper_2007_11208_amd import workloads as W

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


def T(a):
    return torch.from_numpy(np.asfortranarray(a)).to("cuda:0")


def spectrum_case(n, kappa, spd, nrhs, seed):
    rng = np.random.default_rng(seed)
    s = np.logspace(0, -math.log10(kappa), n)
    a = W.prescribed_spectrum(n, s, rng, symmetric=spd)
    b = W.rhs_for(a, W.x_true(n, nrhs, rng))
    return a, b


def check(ada, a, b, precision):
    n = a.shape[0]
    x, r = ada.solve(T(a), T(b), precision=precision)
    torch.cuda.synchronize()
    xr, rr = O.solve(a, b)
    print(f"n={n} {precision}: {r.cls}/{r.route} it={r.refine_iters} berr={r.berr:.2e} rcond={r.rcond:.2e}",
          flush=True)
    assert r.status == rr["status"] == 0
    assert r.cls == ada.CLASS_NAMES[rr["cls"]] and (r.kl, r.ku) == (rr["kl"], rr["ku"])
    assert r.route == ada.ROUTE_NAMES[rr["route"]], (r, rr)
    assert r.chol_failed == bool(rr["chol_failed"])
    assert r.fallback == rr["fallback"]
    if rr["fallback"] == 0:
        if precision == "bf16_ir" and r.refine_iters > 0:
            # the estimate is that of the BF16 factors, the LU of a matrix perturbed by about u_BF16 |L||U|:
            # never much above A's, possibly far below it, and at least the refinement gate
            assert 1e-9 <= r.rcond <= 2.0 * rr["rcond"], (r.rcond, rr["rcond"])
        else:
            assert 0.5 * rr["rcond"] <= r.rcond <= 2.0 * rr["rcond"], (r.rcond, rr["rcond"])
        xg = x.cpu().numpy().reshape(xr.shape)
        eta = check_berr(r.berr, a, b, xg)
        if r.refine_iters > 0:
            assert eta <= math.sqrt(n) * EPS
        else:
            assert eta <= max(1e-12, 2.0 * rr["berr"])
        kappa = 1.0 / max(rr["rcond"], 1e-300)
        tol = 32 * n * kappa * EPS * max(1.0, np.max(np.abs(xr)))
        assert np.max(np.abs(xg - xr)) <= tol, (np.max(np.abs(xg - xr)), tol)
    return r


@pytest.mark.parametrize("n,spd", [(300, False), (513, False), (1000, True), (1100, False)])
def test_fp32_refined_well_conditioned(ada, n, spd):
    a, b = spectrum_case(n, 1e2, spd, 3, seed=n)
    r = check(ada, a, b, "fp32_ir")
    assert r.refine_iters > 0, "FP32 factors converge at kappa 1e2"


@pytest.mark.parametrize("spd", [False, True])
def test_fp32_refined_kappa_1e5_nrhs16(ada, spd):
    a, b = spectrum_case(1024, 1e5, spd, 16, seed=77)
    r = check(ada, a, b, "fp32_ir")
    assert r.refine_iters > 0, "FP32 factors converge at kappa 1e5"


@pytest.mark.parametrize("spd", [False, True])
def test_bf16_gmres_refined_kappa_1e2(ada, spd):
    """BF16 factors are too inexact for the plain correction; GMRES preconditioned by them converges."""
    a, b = spectrum_case(768, 1e2, spd, 4, seed=5)
    r = check(ada, a, b, "bf16_ir")
    assert r.refine_iters > 0, "GMRES-based refinement of the BF16 factors converges at kappa 1e2"


@pytest.mark.parametrize("n,kappa,nrhs", [(1024, 1e3, 16), (333, 1e4, 1)])
def test_bf16_gmres_refined_dense(ada, n, kappa, nrhs):
    a, b = spectrum_case(n, kappa, False, nrhs, seed=n + 3)
    r = check(ada, a, b, "bf16_ir")
    assert r.refine_iters > 0


def test_bf16_kappa_1e5_refined_or_fp64(ada):
    """At kappa 1e5 (kappa u_BF16 about 400) fifty GMRES steps reduce the preconditioned residual by
    about 50 only and the refinement stalls: the FP64 route then solves the system, to its bars."""
    a, b = spectrum_case(1024, 1e5, False, 16, seed=1027)
    r = check(ada, a, b, "bf16_ir")
    assert r.refine_iters != 0


@pytest.mark.parametrize("precision", ["fp32_ir", "bf16_ir"])
def test_refinement_beyond_its_range_falls_back_to_fp64(ada, precision):
    """kappa 1e10 is beyond both operand precisions: refinement diverges or stalls, and
    the FP64 route solves the system."""
    a, b = spectrum_case(640, 1e10, False, 2, seed=11)
    r = check(ada, a, b, precision)
    assert r.refine_iters < 0


def test_mixed_leaves_other_routes_in_fp64(ada):
    rng = np.random.default_rng(3)
    for a in (W.triangular(300, rng, upper=False, scaled=True), W.banded_dense(400, 2, 3, rng)):
        b = W.rhs_for(a, W.x_true(a.shape[0], 1, rng))
        r = check(ada, a, b, "fp32_ir")
        assert r.refine_iters == 0 and r.route in ("tri", "band_lu")


def test_mixed_cholesky_failure_goes_to_lu(ada):
    """A symmetric indefinite matrix passes the sympd heuristic; Cholesky fails (in the
    low-precision attempt and again in FP64) and LU solves it, as in FP64."""
    a = W.sym_indefinite(700, np.random.default_rng(21))
    b = W.rhs_for(a, W.x_true(700, 2, np.random.default_rng(22)))
    r = check(ada, a, b, "fp32_ir")
    assert r.chol_failed and r.route == "lu"
