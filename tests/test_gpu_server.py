"""GPU tests of the solve server (continuous batching over an HBM arena).

* Every request's result in a mix of concurrent requests equals the same request's
  result alone (the server then runs it with nothing else in flight), within the
  parity tolerance: class, band widths, route and fallback exact, rcond within a
  factor 2, x within 32 n kappa eps |x|, backward error within the FP64 bars; and
  class and route equal the oracle's.
* Kept factors solve new right-hand sides: x equals the oracle's solve of the same
  system within the same tolerance.
* Admission by footprint: a request larger than the arena is refused; requests that
  fit only one at a time all complete; the arena is empty again afterwards.
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


def same_solution(a, x1, x2, r1, r2):
    assert (r1.cls, r1.kl, r1.ku, r1.route, r1.fallback, r1.status) == (r2.cls, r2.kl, r2.ku, r2.route, r2.fallback,
                                                                         r2.status)
    if r1.route == "svd":
        assert r1.rank == r2.rank
        return
    if r1.fallback == 0:
        assert 0.5 * r2.rcond <= r1.rcond <= 2.0 * r2.rcond
    kappa = 1.0 / max(r2.rcond, 1e-300)
    tol = 32 * a.shape[0] * kappa * EPS * max(1.0, float(np.max(np.abs(x2))))
    assert float(np.max(np.abs(x1 - x2))) <= tol


def test_server_mix_equals_alone(ada):
    systems = [W.serving_system(k, n_hi=700) for k in range(48)]
    srv = ada.Server(2 * GiB, solve_workers=3)
    try:
        tickets = [srv.submit(T(a), T(b)) for _, a, b in systems]
        mix = [srv.poll(t) for t in tickets]
        for (kind, a, b), m in zip(systems, mix):
            rc, r, X, kept, q_us, tot_us = m
            print(f"{kind} n={a.shape[0]} nrhs={b.shape[1]} -> {r.cls}/{r.route} rc={rc} {tot_us / 1e3:.2f} ms",
                  flush=True)
            assert rc == 0 and kept == 0 and tot_us >= q_us >= 0.0
            xr, rr = O.solve(a, b)
            assert r.cls == ada.CLASS_NAMES[rr["cls"]] and r.route == ada.ROUTE_NAMES[rr["route"]], (r, rr)
            eta = check_berr(r.berr, a, b, X.cpu().numpy())
            assert eta <= max(1e-12, 2.0 * rr["berr"])
            t = srv.submit(T(a), T(b))
            rc2, r2, X2, _, _, _ = srv.poll(t)
            assert rc2 == 0
            same_solution(a, X.cpu().numpy(), X2.cpu().numpy(), r, r2)
        used, queued, nkept = srv.usage()
        assert queued == 0 and nkept == 0
    finally:
        srv.close()


def test_server_kept_factors_solve_new_rhs(ada):
    rng = np.random.default_rng(31)
    mats = [W.dense_general(300, rng), W.spd(420, rng), W.triangular(260, rng, upper=False, scaled=True),
            W.banded_dense(500, 3, 2, rng), W.ill_conditioned(100, rng, smin=1e-18), W.dense_general(40, rng),
            W.prescribed_spectrum(350, np.logspace(0, -5, 350), rng, symmetric=True)]
    srv = ada.Server(2 * GiB, solve_workers=2)
    try:
        factors = []
        for a in mats:
            b = W.rhs_for(a, W.x_true(a.shape[0], 2, rng))
            rc, r, X, kept, _, _ = srv.poll(srv.submit(T(a), T(b), keep=True))
            assert rc == 0 and kept != 0, (rc, ada.last_error())
            factors.append((a, r, kept))
        assert srv.usage()[2] == len(mats)
        # several new right-hand sides per factor, submitted together
        pend = []
        for a, r0, f in factors:
            for nr in (1, 5):
                b = W.rhs_for(a, W.x_true(a.shape[0], nr, rng))
                pend.append((a, b, r0, srv.submit(None, T(b), reuse=f)))
        for a, b, r0, t in pend:
            rc, r, X, kept, _, _ = srv.poll(t)
            print(f"reuse n={a.shape[0]} nrhs={b.shape[1]} {r.route} berr={r.berr:.2e}", flush=True)
            assert rc == 0 and kept == 0
            assert (r.cls, r.route, r.rcond) == (r0.cls, r0.route, r0.rcond)
            xr, rr = O.solve(a, b)
            assert r.route == ada.ROUTE_NAMES[rr["route"]]
            eta = check_berr(r.berr, a, b, X.cpu().numpy())
            assert eta <= max(1e-12, 2.0 * rr["berr"])
            if r.route != "svd":
                kappa = 1.0 / max(rr["rcond"], 1e-300)
                tol = 32 * a.shape[0] * kappa * EPS * max(1.0, float(np.max(np.abs(xr))))
                assert float(np.max(np.abs(X.cpu().numpy().reshape(xr.shape) - xr))) <= tol
        # mixed-precision factors are refined on reuse
        a = W.prescribed_spectrum(400, np.logspace(0, -3, 400), rng)
        b = W.rhs_for(a, W.x_true(400, 2, rng))
        rc, r, _, fm, _, _ = srv.poll(srv.submit(T(a), T(b), keep=True, precision="fp32_ir"))
        assert rc == 0 and r.refine_iters > 0
        b2 = W.rhs_for(a, W.x_true(400, 3, rng))
        rc, r2, X2, _, _, _ = srv.poll(srv.submit(None, T(b2), reuse=fm))
        assert rc == 0 and r2.refine_iters > 0
        assert check_berr(r2.berr, a, b2, X2.cpu().numpy()) <= math.sqrt(400) * EPS
        for _, _, f in factors:
            srv.release(f)
        srv.release(fm)
        with pytest.raises(ada.AdaError):
            srv.submit(None, T(b2), reuse=fm)
        assert srv.usage()[2] == 0
    finally:
        srv.close()


def test_server_admission_by_footprint(ada):
    rng = np.random.default_rng(5)
    n = 2048
    a = W.dense_general(n, rng)
    b = W.rhs_for(a, W.x_true(n, 1, rng))
    probe = ada.Request()
    probe.n, probe.nrhs, probe.lda, probe.ldb, probe.ldx = n, 1, n, n, n
    fp = ada.lib().ada_request_footprint(probe)
    assert fp > 0
    reserved_srv = ada.Server(1 * GiB, solve_workers=2)
    reserved = reserved_srv.usage()[0]
    reserved_srv.close()
    # room for one such request at a time (plus change)
    srv = ada.Server(reserved + fp + fp // 2, solve_workers=2)
    try:
        ts = [srv.submit(T(a), T(b)) for _ in range(3)]
        for t in ts:
            rc, r, X, _, q_us, tot_us = srv.poll(t)
            assert rc == 0 and r.route == "lu"
            assert check_berr(r.berr, a, b, X.cpu().numpy()) <= 1e-12
        assert srv.usage()[0] == reserved
        big = W.dense_general(4096, rng)
        with pytest.raises(ada.AdaError) as e:
            srv.submit(T(big), T(np.ones((4096, 1))))
        assert e.value.code == ada.ERR_NOMEM
    finally:
        srv.close()


def test_server_errors_and_pending(ada):
    rng = np.random.default_rng(8)
    srv = ada.Server(1 * GiB, solve_workers=1)
    try:
        bad = W.dense_general(30, rng)
        bad[2, 3] = np.inf
        big = W.dense_general(1500, rng)
        t_bad = srv.submit(T(bad), T(np.ones((30, 1))))
        t_big = srv.submit(T(big), T(np.ones((1500, 1))))
        first = srv.poll(t_big, timeout_us=0)
        rc, r, _, _, _, _ = srv.poll(t_bad)
        assert rc == ada.ERR_NONFINITE
        done = first if first is not None else srv.poll(t_big)
        assert done[0] == 0
        with pytest.raises(ada.AdaError):
            srv.poll(t_big)  # retired
        with pytest.raises(ada.AdaError):
            srv.submit(None, T(np.ones((30, 1))), reuse=12345)
    finally:
        srv.close()
