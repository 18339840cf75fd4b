"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests touch the GPU library. Each pin is chosen so that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a flipped comparison) fails at least one of them; the
planted-mistake test at the end checks that for a set of concrete mutations.
"""
import itertools
import json
import os
from fractions import Fraction

import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

import oracle
from paper_2007_11208_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps
O = oracle.get()
CLS = {"general": oracle.GENERAL, "banded": oracle.BANDED, "tri_upper": oracle.TRI_UPPER,
       "tri_lower": oracle.TRI_LOWER, "sympd": oracle.SYMPD}


def F(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- detection

def test_fig1_worked_examples(o=O):
    g = json.load(open(os.path.join(HERE, "golden", "fig1.json")))
    for key in ("a", "b", "c"):
        e = g[key]
        a = F(e["matrix"])
        d = o.detect(a)
        assert (d["kl"], d["ku"]) == (e["kl"], e["ku"]), key
        assert d["banded"] == e["banded"], key
        assert d["cls"] == CLS[e["class"]], key
        n = a.shape[0]
        mask = np.abs(np.subtract.outer(np.arange(n), np.arange(n)))
        i, j = np.indices((n, n))
        inband = ((i - j) <= e["kl"]) & ((j - i) <= e["ku"])
        assert int(inband.sum()) == e["band_positions"]
    # Fig. 1(c) is sympd: Cholesky succeeds and the adaptive solve takes that route
    c = F(g["c"]["matrix"])
    _, info = o.potrf(c)
    assert info == 0
    x, r = o.solve(c, F(np.ones((5, 1))))
    assert r["route"] == 3 and r["fallback"] == 0


def _expected_widths(a):
    i, j = np.nonzero(a)
    kl = int(max([0] + list(i[i > j] - j[i > j])))
    ku = int(max([0] + list(j[j > i] - i[j > i])))
    return kl, ku


def _band_positions(n, kl, ku):
    i, j = np.indices((n, n))
    return int((((i - j) <= kl) & ((j - i) <= ku)).sum())


def test_band_scan_all_4x4_patterns(o=O):
    """Brute force over all 2^16 zero patterns of a 4x4 matrix."""
    rng = np.random.default_rng(7)
    n = 4
    vals = rng.uniform(0.5, 1.0, (n, n)) * rng.choice([-1.0, 1.0], (n, n))
    sym = np.triu(vals, 1)
    sym = sym + sym.T
    sym[np.diag_indices(n)] = 10.0 + rng.uniform(0, 1, n)
    idx = [(i, j) for j in range(n) for i in range(n)]
    for mask in range(1 << 16):
        pat = np.zeros((n, n), dtype=bool)
        for b, (i, j) in enumerate(idx):
            if mask >> b & 1:
                pat[i, j] = True
        symmetric_pat = bool(np.all(pat == pat.T))
        base = sym if symmetric_pat else vals
        a = F(np.where(pat, base, 0.0))
        d = o.detect(a)
        kl, ku = _expected_widths(a)
        assert (d["kl"], d["ku"]) == (kl, ku), mask
        banded = 4 * _band_positions(n, kl, ku) <= n * n
        if banded:
            cls = oracle.BANDED
        elif not np.any(np.tril(a, -1)):
            cls = oracle.TRI_UPPER
        elif not np.any(np.triu(a, 1)):
            cls = oracle.TRI_LOWER
        elif symmetric_pat and np.all(np.diag(pat)):
            cls = oracle.SYMPD  # symmetric, diagonal 10..11 > 2*max|off| -> every Fig. 4 condition holds
        else:
            cls = oracle.GENERAL  # asymmetric pattern or a missing diagonal entry
        assert d["cls"] == cls, (mask, d)


def test_band_rule_counts_positions_exactly(o=O):
    """The closed-form band count used by the 25% rule equals a direct count."""
    for n in range(1, 41):
        for kl in range(0, min(n, 7)):
            for ku in range(0, min(n, 7)):
                assert o.is_banded(n, kl, ku) == (4 * _band_positions(n, kl, ku) <= n * n), (n, kl, ku)
    # smallest n at which common widths count as banded (equality is banded)
    first = {}
    for kl, ku in [(1, 1), (2, 2), (4, 4), (1, 4), (0, 0)]:
        first[(kl, ku)] = next(n for n in range(1, 200) if n > max(kl, ku) and o.is_banded(n, kl, ku))
    assert first == {(1, 1): 12, (2, 2): 19, (4, 4): 34, (1, 4): 22, (0, 0): 4}


def test_band_scan_planted_bands_and_transpose(o=O):
    rng = np.random.default_rng(11)
    for t in range(60):
        n = int(rng.integers(5, 120))
        kl = int(rng.integers(0, n))
        ku = int(rng.integers(0, n))
        i, j = np.indices((n, n))
        a = np.where(((i - j) <= kl) & ((j - i) <= ku), rng.standard_normal((n, n)), 0.0)
        a[kl, 0] = 1.0  # make sure the extreme diagonals are occupied
        a[0, ku] = 1.0
        a = F(a)
        assert o.band_scan(a) == (kl, ku)
        assert o.band_scan(F(a.T)) == (ku, kl)
        d, dt = o.detect(a), o.detect(F(a.T))
        swap = {oracle.TRI_UPPER: oracle.TRI_LOWER, oracle.TRI_LOWER: oracle.TRI_UPPER}
        if d["cls"] in swap and kl != ku:
            assert dt["cls"] == swap[d["cls"]]
    # -0.0 counts as zero (IEEE compare)
    a = F(np.eye(6))
    a[5, 0] = -0.0
    a[0, 5] = -0.0
    assert o.band_scan(a) == (0, 0)


def test_likely_sympd_conditions(o=O):
    tol = 100 * EPS
    # positive diagonal (Fig. 4 line 8: <= 0 fails)
    a = F(np.diag([1.0, 2.0, 3.0]) + 0.1 * (np.ones((3, 3)) - np.eye(3)))
    assert o.likely_sympd(a)
    b = a.copy(order="F"); b[1, 1] = 0.0
    assert not o.likely_sympd(b)
    b = a.copy(order="F"); b[2, 2] = -1.0
    assert not o.likely_sympd(b)
    # symmetry, relative branch (large entries): tol*max ~ 2.2e-11
    a = F([[3000.0, 1000.0], [1000.0, 3000.0]])
    b = a.copy(order="F"); b[1, 0] = 1000.0 + 1e-12
    assert o.likely_sympd(b)
    b[1, 0] = 1000.0 + 1e-10
    assert not o.likely_sympd(b)
    # symmetry, absolute branch (small entries): tol*max ~ 2.2e-17
    a = F([[1.0, 1e-3], [1e-3, 1.0]])
    b = a.copy(order="F"); b[1, 0] = 1e-3 + 1e-14
    assert o.likely_sympd(b)  # delta < tol (absolute) although delta > tol*max
    b[1, 0] = 1e-3 + 1e-13
    assert not o.likely_sympd(b)
    # line 15 tests only the lower element, with ">=": an upper element equal to
    # max_diag passes, a lower one fails (line 16 holds strictly in both cases)
    m = 1.0
    near = m * (1.0 - 1e-15)
    up = F([[m, m], [near, m]])  # A[0,1] = m (upper), A[1,0] slightly below
    lo = F([[m, near], [m, m]])  # A[1,0] = m (lower)
    assert abs(up[0, 1] - up[1, 0]) <= tol
    assert o.likely_sympd(up)
    assert not o.likely_sympd(lo)
    # line 16 with ">=": equality fails, slightly less passes
    a = F([[2.0, 1.5, 0.0], [1.5, 1.0, 0.0], [0.0, 0.0, 3.0]])
    assert not o.likely_sympd(a)  # 1.5 + 1.5 == 2 + 1
    a[0, 1] = a[1, 0] = np.nextafter(1.5, 0.0)
    assert o.likely_sympd(a)


def test_likely_sympd_permutation_invariant(o=O):
    rng = np.random.default_rng(3)
    for t in range(40):
        n = int(rng.integers(2, 40))
        a = W.fig3_sympd(n, rng)
        if t % 3 == 1:
            a[int(rng.integers(1, n)), 0] *= 1 + 1e-9  # asymmetric beyond tolerance
        if t % 3 == 2:
            a = F(a + np.diag(rng.uniform(-3, 0, n)))  # may break dominance or positivity
        p = rng.permutation(n)
        assert o.likely_sympd(a) == o.likely_sympd(F(a[np.ix_(p, p)]))


def test_fig3_generator_is_detected_sympd(o=O):
    for s in range(20):
        a = W.fig3_sympd(100, np.random.default_rng(s))
        assert o.detect(a)["cls"] == oracle.SYMPD
        x, r = o.solve(a, F(np.random.default_rng(s).random((100, 1))))
        assert r["route"] == 3 and r["fallback"] == 0 and r["berr"] < 1e-15


# ---------------------------------------------------------------- factorisations and solves

def _cramer(a, b):
    n = len(b)
    A = [[Fraction(float(a[i, j])) for j in range(n)] for i in range(n)]
    B = [Fraction(float(v)) for v in b]

    def det(M):
        if len(M) == 1:
            return M[0][0]
        return sum(((-1) ** c) * M[0][c] * det([row[:c] + row[c + 1:] for row in M[1:]]) for c in range(len(M)))

    D = det(A)
    out = []
    for k in range(n):
        Mk = [row[:k] + [B[i]] + row[k + 1:] for i, row in enumerate(A)]
        out.append(det(Mk) / D)
    return np.array([float(v) for v in out])


@pytest.mark.parametrize("kind", ["general", "spd", "upper", "lower", "diag"])
def test_cramer_small_systems(kind, o=O):
    rng = np.random.default_rng(5)
    for n in range(1, 5):
        for t in range(15):
            if kind == "general":
                a = rng.standard_normal((n, n)) + 2 * np.eye(n)
                if n > 1:
                    a[0, 1] = a[0, 1] or 0.5
                    a[1, 0] = a[1, 0] or 0.5
            elif kind == "spd":
                g = rng.standard_normal((n, n))
                a = g.T @ g
                a = 0.5 * (a + a.T) + n * np.eye(n)
            elif kind == "upper":
                a = np.triu(rng.standard_normal((n, n))) + 2 * np.eye(n)
            elif kind == "lower":
                a = np.tril(rng.standard_normal((n, n))) + 2 * np.eye(n)
            else:
                a = np.diag(rng.uniform(1, 3, n))
            a = F(a)
            b = rng.standard_normal(n)
            x, r = o.solve(a, F(b.reshape(n, 1)))
            xe = _cramer(a, b)
            kappa = np.linalg.cond(a, 1)
            assert r["status"] == 0 and r["fallback"] == 0
            assert np.max(np.abs(x[:, 0] - xe)) <= 50 * kappa * EPS * max(1.0, np.max(np.abs(xe))), (kind, n, r)


def test_routes_for_cramer_kinds(o=O):
    rng = np.random.default_rng(2)
    a = F(np.diag(rng.uniform(1, 3, 4)))
    assert o.detect(a)["cls"] == oracle.BANDED  # n=4 diagonal: 4 positions of 16 = 25%
    assert o.detect(F(np.diag([1.0, 2.0, 3.0])))["cls"] == oracle.TRI_UPPER  # 3 of 9 > 25%


def _run_known_x(a, o, nrhs=3, seed=0):
    rng = np.random.default_rng(seed)
    n = a.shape[0]
    x = F(rng.standard_normal((n, nrhs)))
    b = F(a @ x)
    xs, r = o.solve(a, b)
    return x, xs, r


@pytest.mark.parametrize("case", ["a_dense", "b_spd", "c_upper_scaled", "d_banded", "e_illcond"])
def test_known_x_true(case, o=O):
    a, _ = W.small_case(case)
    x, xs, r = _run_known_x(a, o)
    n = a.shape[0]
    assert r["status"] == 0 and r["fallback"] == 0
    assert r["berr"] <= 4 * n * EPS
    kappa = np.linalg.cond(a, 1)
    fe = np.max(np.abs(xs - x)) / np.max(np.abs(x))
    assert fe <= 10 * n * kappa * EPS


def test_getrf_matches_lapack(o=O):
    rng = np.random.default_rng(9)
    for n in [1, 2, 7, 33, 100]:
        a = F(rng.standard_normal((n, n)))
        lu, ipiv, info = o.getrf(a)
        lu2, piv2, info2 = lapack.dgetrf(a)
        assert info == info2 == 0
        assert np.array_equal(ipiv, piv2)
        assert np.allclose(lu, lu2, rtol=0, atol=1e-12 * np.max(np.abs(a)) * n)
        b = rng.standard_normal((n, 2))
        for trans in (0, 1):
            x = o.getrs(lu, ipiv, F(b), trans=bool(trans))
            x2, _ = lapack.dgetrs(lu2, piv2, b, trans=trans)
            assert np.allclose(x, x2, rtol=1e-10, atol=1e-12)


def test_getrf_zero_pivot_and_ties(o=O):
    a = F([[0.0, 1.0, 2.0], [0.0, 3.0, 4.0], [0.0, 5.0, 7.0]])  # zero first column
    _, _, info = o.getrf(a)
    assert info == 1
    _, _, info2 = lapack.dgetrf(a)
    assert info2 == 1
    # ties go to the lowest row index (the IxAMAX convention)
    a = F([[1.0, 2.0, 0.0], [-3.0, 1.0, 1.0], [3.0, 0.0, 2.0]])
    _, ipiv, _ = o.getrf(a)
    _, piv2, _ = lapack.dgetrf(a)
    assert ipiv[0] == 1 and np.array_equal(ipiv, piv2)


def test_potrf_matches_lapack_and_failure_column(o=O):
    rng = np.random.default_rng(4)
    a = W.spd(200, rng)
    l, info = o.potrf(a)
    c, info2 = lapack.dpotrf(a, lower=1)
    assert info == info2 == 0
    assert np.allclose(l, np.tril(c), rtol=0, atol=1e-12)
    s = W.sym_indefinite(512, np.random.default_rng(0))
    assert o.detect(s)["cls"] == oracle.SYMPD
    _, info = o.potrf(s)
    _, info2 = lapack.dpotrf(s, lower=1)
    assert info == info2 > 0


def test_trsv_matches_lapack(o=O):
    rng = np.random.default_rng(8)
    n = 57
    for upper in (True, False):
        t = F(np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)) if upper else \
            F(np.tril(rng.standard_normal((n, n))) + 4 * np.eye(n))
        b = rng.standard_normal(n)
        for trans in (0, 1):
            for unit in (0, 1):
                x = o.trsv(t, b, upper, trans=bool(trans), unit=bool(unit))
                x2, info = lapack.dtrtrs(t, b, lower=int(not upper), trans=trans, unitdiag=unit)
                assert np.allclose(x, x2, rtol=1e-11, atol=1e-11), (upper, trans, unit)


def test_band_lu_equals_dense_lu(o=O):
    """Banded LU with partial pivoting makes the same pivots and the same U as dense LU."""
    rng = np.random.default_rng(12)
    for t in range(20):
        n = int(rng.integers(8, 90))
        kl, ku = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        ab = F(rng.standard_normal((kl + ku + 1, n)))
        for r in range(kl + ku + 1):
            d = ku - r
            if d > 0:
                ab[r, :d] = 0
            elif d < 0:
                ab[r, n + d:] = 0
        a = W.band_to_dense(ab, kl, ku)
        abf, ipiv, info = o.gbtrf(ab, kl, ku)
        lu, ipiv2, info2 = o.getrf(a)
        assert info == info2
        assert np.array_equal(ipiv, ipiv2)
        U = np.triu(lu)
        kd = kl + ku
        for j in range(n):
            for i in range(max(0, j - kd), j + 1):
                assert abf[kl + ku + i - j, j] == U[i, j], (t, i, j)
        assert np.count_nonzero(np.triu(U, kd + 1)) == 0
        if info == 0:
            b = F(rng.standard_normal((n, 2)))
            for trans in (0, 1):
                x = o.gbtrs(abf, kl, ku, ipiv, b, trans=bool(trans))
                x2 = o.getrs(lu, ipiv2, b, trans=bool(trans))
                assert np.allclose(x, x2, rtol=1e-9, atol=1e-9)
            # LAPACK's band LU: same info and solution
            lub, pivb, x3, infob = lapack.dgbsv(kl, ku, np.vstack([np.zeros((kl, n)), ab]), np.array(b))
            assert infob == 0
            assert np.allclose(o.gbtrs(abf, kl, ku, ipiv, b), x3, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- condition estimate

def test_rcond_is_lower_bound_and_close(o=O):
    rng = np.random.default_rng(21)
    for t in range(30):
        n = int(rng.integers(2, 120))
        a = F(rng.standard_normal((n, n)) + (t % 4) * np.eye(n))
        exact = np.linalg.norm(np.linalg.inv(a), 1) * np.linalg.norm(a, 1)
        rc, ns = o.rcond_general(a)
        assert 2 <= ns <= 11
        assert rc >= (1 / exact) * (1 - 1e-8)  # estimate of ||inv(A)|| never exceeds the truth
        assert rc <= 10 / exact


def test_rcond_exact_on_diagonal(o=O):
    d = np.array([3.0, -0.5, 7.0, 2.0, 0.25, -9.0])
    a = F(np.diag(d))
    rc, _ = o.rcond_general(a)
    assert rc == pytest.approx(np.min(np.abs(d)) / np.max(np.abs(d)), rel=1e-15)
    rc, _ = o.rcond_tri(a, True)
    assert rc == pytest.approx(0.25 / 9.0, rel=1e-15)
    a1 = F([[4.0]])
    assert o.rcond_general(a1)[0] == 1.0


def test_rcond_against_lapack_estimators(o=O):
    rng = np.random.default_rng(31)
    close = 0
    total = 0
    for t in range(25):
        n = int(rng.integers(5, 150))
        a = F(rng.standard_normal((n, n)) + 3 * np.eye(n))
        lu2, piv2, _ = lapack.dgetrf(a)
        r2, _ = lapack.dgecon(lu2, np.linalg.norm(a, 1), norm="1")
        r1, _ = o.rcond_general(a)
        s = W.spd(n, rng)
        c, _ = lapack.dpotrf(s, lower=1)
        s2, _ = lapack.dpocon(c, np.linalg.norm(s, 1), uplo="L")
        s1, _ = o.rcond_chol(s)
        t_ = F(np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n))
        t2, _ = lapack.dtrcon(t_, norm="1", uplo="U")
        t1, _ = o.rcond_tri(t_, True)
        for x1, x2 in ((r1, r2), (s1, s2), (t1, t2)):
            total += 1
            close += abs(x1 - x2) <= 1e-8 * abs(x2)
            assert 0.2 * x2 <= x1 <= 5 * x2
    assert close >= 0.9 * total  # same estimator family: nearly always the same value


def test_band_rcond_matches_dense(o=O):
    rng = np.random.default_rng(41)
    for t in range(10):
        n = int(rng.integers(30, 200))
        kl, ku = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        ab = W.banded_storage(n, kl, ku, rng)
        a = W.band_to_dense(ab, kl, ku)
        rb, _ = o.rcond_band(ab, kl, ku)
        rd, _ = o.rcond_general(a)
        assert rb == pytest.approx(rd, rel=1e-8)


# ---------------------------------------------------------------- fallback rule

def test_prescribed_spectrum_triggers_fallback(o=O):
    n = 64
    for seed in range(8):
        g = np.random.default_rng(seed)
        for smin, fires in ((1e-14, False), (1e-18, True), (1e-20, True)):
            a = W.ill_conditioned(n, np.random.default_rng(seed), smin)
            x = F(g.standard_normal((n, 1)))
            xs, r = o.solve(a, F(a @ x))
            assert (r["fallback"] != 0) == fires, (seed, smin, r)
            assert r["route"] == (5 if fires else 4)
        s = np.concatenate([np.logspace(0, -6, n - 8), np.zeros(8)])
        a = W.prescribed_spectrum(n, s, np.random.default_rng(seed))
        xs, r = o.solve(a, F(a @ g.standard_normal((n, 1))))
        assert r["fallback"] in (1, 2) and r["route"] == 5 and r["rank"] == n - 8
        assert r["berr"] < 1e-13
        xs, r = o.solve(a, F(a @ g.standard_normal((n, 1))), no_approx=True)
        assert r["status"] == oracle.__dict__.get("ERR_SINGULAR", -3)


def test_rule_threshold_is_half_eps(o=O):
    """rcond < 0.5*eps with a strict '<'; a custom threshold moves the cut."""
    a = W.ill_conditioned(64, np.random.default_rng(1), 1e-14)
    _, r = o.solve(a, F(np.ones((64, 1))))
    rc = r["rcond"]
    assert r["fallback"] == 0 and rc > 0.5 * EPS
    _, r2 = o.solve(a, F(np.ones((64, 1))), rcond_threshold=rc)
    assert r2["fallback"] == 0  # equal to the threshold: not below
    _, r3 = o.solve(a, F(np.ones((64, 1))), rcond_threshold=np.nextafter(rc, 1.0))
    assert r3["fallback"] == 2 and r3["route"] == 5


def test_failures_and_errors(o=O):
    n = 12
    a = F(np.random.default_rng(0).standard_normal((n, n)) + 3 * np.eye(n))
    a[:, 4] = 0.0
    x, r = o.solve(a, F(np.ones((n, 1))))
    assert r["cls"] == oracle.GENERAL and r["info"] == 5 and r["fallback"] == 1 and r["route"] == 5
    t = F(np.triu(np.ones((n, n))))
    t[3, 3] = 0.0
    x, r = o.solve(t, F(np.ones((n, 1))))
    assert r["cls"] == oracle.TRI_UPPER and r["info"] == 4 and r["fallback"] == 1
    b = F(np.ones((n, 1)))
    bad = a.copy(order="F"); bad[2, 3] = np.nan
    assert o.solve(bad, b)[1]["status"] == -2
    bad[2, 3] = np.inf
    assert o.solve(bad, b)[1]["status"] == -2
    x, r = o.solve(F(np.eye(n)), b, force_general=True)
    assert r["cls"] == oracle.GENERAL and r["route"] == 4 and r["kl"] == -1


def test_sym_indefinite_reroutes_to_lu(o=O):
    a = W.sym_indefinite(400, np.random.default_rng(0))
    x = F(np.random.default_rng(1).standard_normal((400, 2)))
    xs, r = o.solve(a, F(a @ x))
    assert r["cls"] == oracle.SYMPD and r["chol_failed"] == 1 and r["route"] == 4
    assert r["fallback"] == 0 and r["berr"] < 1e-14


# ---------------------------------------------------------------- SVD fallback

def test_jacobi_2x2_closed_form(o=O):
    a = F([[3.0, 1.0], [2.0, 4.0]])
    u, s, v, sw = o.jacobi_svd(a)
    ex = np.linalg.svd(a, compute_uv=False)
    # closed form: sigma^2 are the eigenvalues of A^T A
    ata = a.T @ a
    tr, det = np.trace(ata), np.linalg.det(ata)
    lam = np.array([(tr + np.sqrt(tr * tr - 4 * det)) / 2, (tr - np.sqrt(tr * tr - 4 * det)) / 2])
    assert np.allclose(np.sort(s)[::-1], np.sqrt(lam), rtol=1e-14)
    assert np.allclose(np.sort(s)[::-1], ex, rtol=1e-14)
    assert np.allclose(u @ v.T, a, atol=1e-14)  # U holds sigma_i u_i: A V = U


def test_jacobi_prescribed_singular_values(o=O):
    for n, seed in ((16, 0), (40, 1), (64, 2)):
        s = np.sort(np.random.default_rng(seed).uniform(0.01, 2.0, n))[::-1]
        a = W.prescribed_spectrum(n, s, np.random.default_rng(seed + 10))
        u, sg, v, sw = o.jacobi_svd(a)
        assert np.allclose(np.sort(sg)[::-1], s, rtol=0, atol=4 * n * EPS * s[0])
        assert np.allclose(v.T @ v, np.eye(n), atol=1e-13)
        assert np.allclose(a @ v, u, atol=1e-13)


def test_svd_lstsq_min_norm_matches_lapack(o=O):
    """Exactly rank-deficient systems (zero rows/columns placed by permutations), so
    the numerical rank is unambiguous; x must be LAPACK's minimum-norm solution."""
    n, r = 48, 42
    for seed in range(5):
        g = np.random.default_rng(seed)
        c = W.prescribed_spectrum(r, np.logspace(0, -4, r), g)
        a = np.zeros((n, n))
        a[:r, :r] = c
        p, q = g.permutation(n), g.permutation(n)
        a = F(a[np.ix_(p, q)])
        b = F(g.standard_normal((n, 2)))
        x, rank, sg, sw = o.svd_lstsq(a, b)
        x2, res, rank2, sv = sla.lstsq(a, b, cond=EPS, lapack_driver="gelsd")
        assert rank == rank2 == r
        kappa_kept = 1e4  # sigma_max / smallest kept sigma
        assert np.max(np.abs(x - x2)) <= 10 * n * kappa_kept * EPS * np.max(np.abs(x2))
        # the minimum-norm solution has no component in the null space: the
        # unknowns that multiply the zero columns are exactly zero
        zero_cols = np.nonzero(~np.any(a != 0, axis=0))[0]
        assert len(zero_cols) == n - r and np.all(x[zero_cols, :] == 0.0)


# ---------------------------------------------------------------- backward error

def test_berr_definition(o=O):
    a = F([[2.0, 1.0], [1.0, 3.0]])
    x = F([[1.0], [1.0]])
    b = F([[3.0], [4.0]])
    w, per = o.berr(a, b, x)
    assert w == 0.0
    b2 = F([[3.5], [4.0]])  # residual 0.5; ||A||_inf = 4, ||x|| = 1, ||b|| = 4
    w, per = o.berr(a, b2, x)
    assert w == pytest.approx(0.5 / (4 * 1 + 4))


def _eta_exact(a, b, x):
    """Normwise backward error of x in exact rational arithmetic (the definition, no rounding but the last)."""
    n = a.shape[0]
    A = [[Fraction(float(a[i, j])) for j in range(n)] for i in range(n)]
    anorm = max(sum(abs(v) for v in row) for row in A)
    out = []
    for k in range(b.shape[1]):
        X = [Fraction(float(v)) for v in x[:, k]]
        r = [Fraction(float(b[i, k])) - sum(A[i][j] * X[j] for j in range(n)) for i in range(n)]
        rn = max(abs(v) for v in r)
        den = anorm * max(abs(v) for v in X) + max(abs(Fraction(float(v))) for v in b[:, k])
        out.append(float(rn / den) if den else (0.0 if rn == 0 else math.inf))
    return np.array(out)


@pytest.mark.parametrize("n", [3, 8, 25, 60])
def test_berr_exact_rational(n, o=O):
    """The residual of a backward-stable solution is as small as the rounding of a plain FP64
    evaluation of b - A x; the oracle's backward error must still be exact to a few ulps: it equals the
    exact rational value for a LAPACK solution (tiny residual), a perturbed one and a mixed scale."""
    rng = np.random.default_rng(40 + n)
    a = F(rng.standard_normal((n, n)) * np.exp(rng.uniform(-3, 3, (n, n))))
    b = F(rng.standard_normal((n, 3)))
    x = F(np.linalg.solve(a, b))
    x[:, 1] *= 1.0 + 1e-9 * rng.standard_normal(n)  # a genuine residual
    x[:, 2] = x[:, 2] * 1e6  # large scale
    b[:, 2] *= 1e6
    w, per = o.berr(a, b, x)
    ex = _eta_exact(a, b, x)
    assert np.all(ex[[0, 2]] < 1e-14) and ex[1] > 1e-12
    assert np.allclose(per, ex, rtol=1e-13, atol=0.0), (per, ex)
    assert w == per.max()


def test_berr_band_hand_and_against_dense(o=O):
    # hand-worked: A = [[4,1,0],[2,5,1],[0,3,6]] (kl = ku = 1), x = (1,1,1), b = (5,8.5,9): residual (0,0.5,0);
    # ||A||_inf = 9, ||x|| = 1, ||b|| = 9: eta = 0.5 / 18
    ab = F([[0.0, 1.0, 1.0], [4.0, 5.0, 6.0], [2.0, 3.0, 0.0]])
    x = F([[1.0], [1.0], [1.0]])
    b = F([[5.0], [8.5], [9.0]])
    xl = x.ctypes.data_as(oracle._P)
    w = o.lib.orc_berr_band(3, 1, 1, 1, ab.ctypes.data_as(oracle._P), 3, b.ctypes.data_as(oracle._P), 3, xl, 3)
    assert w == 0.5 / 18.0
    # a random band with a backward-stable solution: the band evaluation equals the dense one and the exact value
    rng = np.random.default_rng(3)
    n, kl, ku = 40, 3, 2
    ab = W.banded_storage(n, kl, ku, rng)
    a = W.band_to_dense(ab, kl, ku)
    b = F(rng.standard_normal((n, 2)))
    xs = F(np.linalg.solve(a, b))
    wb = o.lib.orc_berr_band(n, kl, ku, 2, ab.ctypes.data_as(oracle._P), ab.shape[0], b.ctypes.data_as(oracle._P), n,
                             xs.ctypes.data_as(oracle._P), n)
    wd, _ = o.berr(a, b, xs)
    ex = _eta_exact(a, b, xs).max()
    assert wb == pytest.approx(ex, rel=1e-13) and wd == pytest.approx(ex, rel=1e-13)


# ---------------------------------------------------------------- whole small configuration

def test_small_configuration_routes(o=O):
    exp = {"a_dense": (oracle.GENERAL, 4, 0), "b_spd": (oracle.SYMPD, 3, 0),
           "c_upper": (oracle.TRI_UPPER, 5, 2), "c_upper_scaled": (oracle.TRI_UPPER, 2, 0),
           "d_banded": (oracle.BANDED, 1, 0), "e_illcond": (oracle.GENERAL, 4, 0),
           "e_illcond_1e18": (oracle.GENERAL, 5, 2)}
    for name, (cls, route, fb) in exp.items():
        a, b = W.small_case(name)
        x, r = o.solve(a, b)
        assert (r["cls"], r["route"], r["fallback"]) == (cls, route, fb), (name, r)
        assert r["berr"] < 1e-13, name
    # triangular literal generator: the independent LAPACK estimate agrees that it is below 0.5 eps
    a, _ = W.small_case("c_upper")
    rc, _ = lapack.dtrcon(a, norm="1", uplo="U")
    assert rc < 0.5 * EPS


def test_band_layout_driver(o=O):
    rng = np.random.default_rng(17)
    n, kl, ku = 3000, 3, 2
    ab = W.banded_storage(n, kl, ku, rng)
    x = F(rng.standard_normal((n, 2)))
    b = W.band_matvec(ab, kl, ku, x)
    xs, r = o.solve_band(ab, kl, ku, b)
    assert r["cls"] == oracle.BANDED and (r["kl"], r["ku"]) == (kl, ku) and r["route"] == 1
    assert r["berr"] < 1e-15
    a = W.band_to_dense(ab, kl, ku)
    xd, rd = o.solve(a, b)
    assert np.allclose(xs, xd, rtol=1e-12, atol=1e-12)
    assert r["rcond"] == pytest.approx(rd["rcond"], rel=1e-10)
    # stored band wider than the true band: detection finds the true widths
    ab2 = np.zeros((kl + ku + 5, n), order="F")
    ab2[2:2 + kl + ku + 1, :] = ab  # ku_in = ku + 2, kl_in = kl + 2
    xs2, r2 = o.solve_band(ab2, kl + 2, ku + 2, b)
    assert (r2["kl"], r2["ku"]) == (kl, ku) and np.array_equal(xs2, xs)
    # fallback on a huge band system is infeasible
    ab3 = ab.copy(order="F")
    ab3[:, 10] = 0.0  # an all-zero column stays zero under elimination -> exact zero pivot
    _, r3 = o.solve_band(ab3, kl, ku, b, dense_limit=1000)
    assert r3["status"] == -6


# ---------------------------------------------------------------- Section V extensions
# Plain symmetric matrices by LDL^T with Bunch-Kaufman pivoting, tridiagonal matrices by
# tridiagonal LU with partial pivoting (the future work the paper names; off by default).

BK_ALPHA = (1.0 + np.sqrt(17.0)) / 8.0


def _d_matrix(d, e):
    n = d.shape[0]
    return np.diag(d) + np.diag(e[: n - 1], -1) + np.diag(e[: n - 1], 1)


def test_sytrf_bk_matches_lapack_ldl(o=O):
    """LAPACK's dsytrf (through scipy.linalg.ldl) takes the same Bunch-Kaufman decisions:
    the block diagonal D and the permuted unit lower factor agree."""
    rng = np.random.default_rng(41)
    for n in (1, 2, 3, 5, 17, 40, 90):
        for t in range(3):
            a = rng.standard_normal((n, n))
            if t == 1:
                a[np.diag_indices(n)] *= 1e-3  # small diagonal: many 2x2 pivots
            a = F(a + a.T)
            l, d, e, perm, info = o.sytrf_bk(a)
            assert info == 0
            lu2, d2, p2 = sla.ldl(a, lower=True)
            np.testing.assert_allclose(_d_matrix(d, e), d2, rtol=1e-10, atol=1e-12 * np.abs(d2).max())
            pt = np.eye(n)[perm].T
            np.testing.assert_allclose(pt @ l, lu2, rtol=1e-9, atol=1e-11)


def test_sytrf_bk_factorisation_identities(o=O):
    """P A P^T = L D L^T, unit lower L, D of 1x1 and 2x2 blocks, perm a permutation, the
    multipliers of 1x1 columns bounded by 1/(1-alpha), inertia of D = inertia of A."""
    rng = np.random.default_rng(42)
    for n in (4, 33, 120):
        a = rng.standard_normal((n, n))
        a[np.diag_indices(n)] *= 0.05
        a = F(a + a.T)
        l, d, e, perm, info = o.sytrf_bk(a)
        assert info == 0 and sorted(perm) == list(range(n))
        assert np.all(np.diag(l) == 1.0) and np.all(np.triu(l, 1) == 0.0)
        dm = _d_matrix(d, e)
        p = np.eye(n)[perm]
        np.testing.assert_allclose(p @ a @ p.T, l @ dm @ l.T, atol=1e-12 * n * np.abs(a).max())
        blocks = np.flatnonzero(e[: n - 1])
        assert np.all(np.diff(blocks) >= 2), "2x2 blocks do not overlap"
        assert np.all(l[blocks + 1, blocks] == 0.0), "no multiplier inside a 2x2 block"
        assert len(blocks) > 0, "this matrix needs 2x2 pivots"
        one = np.setdiff1d(np.arange(n), np.concatenate([blocks, blocks + 1]))
        if one.size:
            assert np.abs(l[:, one] - np.eye(n)[:, one]).max() <= 1.0 / (1.0 - BK_ALPHA) + 1e-12
        ev_a = np.linalg.eigvalsh(a)
        ev_d = np.linalg.eigvalsh(dm)
        assert (np.sum(ev_a > 0), np.sum(ev_a < 0)) == (np.sum(ev_d > 0), np.sum(ev_d < 0))


def test_sytrf_bk_pivot_rules_by_hand(o=O):
    """The three Bunch-Kaufman cases on 3x3 matrices worked out by hand."""
    # |a00| >= alpha*colmax: 1x1, no interchange
    a = F([[4.0, 1.0, 2.0], [1.0, 3.0, 0.5], [2.0, 0.5, 5.0]])
    l, d, e, perm, info = o.sytrf_bk(a)
    assert list(perm)[0] == 0 and e[0] == 0.0 and d[0] == 4.0
    # |a00| small, a_rr large against its row: 1x1 with interchange 0 <-> r (r = 2)
    a = F([[0.0, 1.0, 2.0], [1.0, 0.0, 0.5], [2.0, 0.5, 10.0]])
    l, d, e, perm, info = o.sytrf_bk(a)
    assert perm[0] == 2 and d[0] == 10.0 and e[0] == 0.0
    # |a00| small and a_rr small: 2x2 pivot on (0, r) with r moved to position 1
    a = F([[0.0, 1.0, 3.0], [1.0, 0.0, 0.5], [3.0, 0.5, 0.0]])
    l, d, e, perm, info = o.sytrf_bk(a)
    assert list(perm[:2]) == [0, 2] and e[0] == 3.0 and d[0] == 0.0 and d[1] == 0.0
    # |a00| * rowmax >= alpha * colmax^2: 1x1 with no interchange although |a00| < alpha*colmax
    a = F([[1.0, 2.0, 0.0], [2.0, 0.0, 8.0], [0.0, 8.0, 0.0]])
    l, d, e, perm, info = o.sytrf_bk(a)
    assert perm[0] == 0 and d[0] == 1.0 and e[0] == 0.0


def test_sytrf_bk_zero_column_info(o=O):
    a = F(np.diag([2.0, 0.0, 3.0, 0.0]))
    _, d, e, perm, info = o.sytrf_bk(a)
    assert info == 2 and d[1] == 0.0
    assert lapack.dsytrf(a, lower=1)[2] == 2


def test_sytrs_and_rcond_sym_against_lapack(o=O):
    rng = np.random.default_rng(43)
    close = total = 0
    for t in range(15):
        n = int(rng.integers(3, 120))
        a = rng.standard_normal((n, n))
        a = F(a + a.T + (0.0 if t % 2 else 0.5) * np.eye(n))
        l, d, e, perm, info = o.sytrf_bk(a)
        assert info == 0
        b = F(rng.standard_normal((n, 3)))
        x = o.sytrs_bk(l, d, e, perm, b)
        ref = np.linalg.solve(a, b)
        np.testing.assert_allclose(x, ref, rtol=0, atol=10 * n * np.linalg.cond(a) * EPS * np.abs(ref).max())
        lu2, ipiv2, info2 = lapack.dsytrf(a, lower=1)
        r2, _ = lapack.dsycon(lu2, ipiv2, np.linalg.norm(a, 1), lower=1)
        r1, _ = o.rcond_sym_bk(a)
        exact = 1.0 / (np.linalg.norm(a, 1) * np.linalg.norm(np.linalg.inv(a), 1))
        assert r1 >= exact * (1 - 1e-10) and r1 <= 3 * n * exact  # estimate of ||inv(A)||_1 is a lower bound
        total += 1
        close += abs(r1 - r2) <= 1e-8 * abs(r2)
    assert close >= 0.9 * total


def _tridiag(n, rng, dominant=False):
    dl, dm, du = rng.standard_normal(n - 1), rng.standard_normal(n), rng.standard_normal(n - 1)
    if dominant:
        dm = dm + 4.0 * np.sign(dm)
    return dl, dm, du


def test_gttrf_matches_lapack_bitwise(o=O):
    """dgttrf runs the same eliminations in the same order: identical factors and pivots."""
    rng = np.random.default_rng(44)
    for n in (3, 4, 7, 50, 301):  # (scipy's wrapper takes n >= 3)
        for dom in (False, True):
            dl, dm, du = _tridiag(n, rng, dom)
            got = o.gttrf(dl, dm, du)
            ref = lapack.dgttrf(dl.copy(), dm.copy(), du.copy())
            for k in range(4):
                assert np.array_equal(got[k], ref[k][: got[k].shape[0]]), (n, k)
            assert np.array_equal(got[4], ref[4] - 1) and got[5] == ref[5]


def test_gttrs_both_directions_and_rcond(o=O):
    rng = np.random.default_rng(45)
    close = total = 0
    for n in (2, 5, 64, 257):
        dl, dm, du = _tridiag(n, rng)
        a = np.diag(dm) + np.diag(dl, -1) + np.diag(du, 1)
        f = o.gttrf(dl, dm, du)
        assert f[5] == 0
        b = F(rng.standard_normal((n, 2)))
        for trans in (False, True):
            x = o.gttrs(*f[:5], b, trans=trans)
            ref = np.linalg.solve(a.T if trans else a, b)
            np.testing.assert_allclose(x, ref, rtol=0, atol=1e3 * np.linalg.cond(a) * EPS * np.abs(ref).max())
        ab = np.zeros((3, n))
        ab[0, 1:], ab[1], ab[2, :-1] = du, dm, dl
        r_band, _ = o.rcond_band(F(ab), 1, 1)
        r_gt, _ = o.rcond_gt(dl, dm, du)
        if n >= 3:  # (scipy's wrapper takes n >= 3)
            lf = lapack.dgttrf(dl.copy(), dm.copy(), du.copy())
            r2, _ = lapack.dgtcon(*lf[:5], np.linalg.norm(a, 1))
            total += 1
            close += abs(r_gt - r2) <= 1e-8 * abs(r2)
        # the banded route with kl = ku = 1 forms the same factors: the same estimate
        assert abs(r_gt - r_band) <= 1e-12 * r_band
    assert close >= 0.75 * total


def test_gttrf_zero_pivot_info(o=O):
    dl, dm, du = np.zeros(3), np.array([1.0, 0.0, 2.0, 3.0]), np.array([0.0, 0.0, 1.0])
    f = o.gttrf(dl, dm, du)
    assert f[5] == 2 and f[5] == lapack.dgttrf(dl.copy(), dm.copy(), du.copy())[5]


def test_extension_routes_in_the_driver(o=O):
    rng = np.random.default_rng(46)
    # plain symmetric (fails Fig. 4): class sym, LDL^T; the paper's driver keeps LU
    n = 150
    a = rng.standard_normal((n, n))
    a = F(a + a.T)
    b = F(rng.standard_normal((n, 2)))
    x0, r0 = o.solve(a, b)
    x1, r1 = o.solve(a, b, ext=oracle.EXT_SYM)
    assert r0["cls"] == oracle.GENERAL and r0["route"] == 4
    assert r1["cls"] == oracle.SYM and r1["route"] == 6 and r1["fallback"] == 0 and r1["berr"] < 1e-14
    np.testing.assert_allclose(x1, x0, rtol=0, atol=1e-8 * np.abs(x0).max())
    assert 0.2 * r0["rcond"] <= r1["rcond"] <= 5 * r0["rcond"]
    # a not exactly symmetric matrix stays general
    a2 = a.copy(order="F")
    a2[3, 7] += 1e-15
    _, r2 = o.solve(a2, b, ext=oracle.EXT_SYM)
    assert r2["cls"] == oracle.GENERAL and r2["route"] == 4
    # sympd by Fig. 4 but Cholesky fails: LDL^T instead of LU
    s = W.sym_indefinite(300, np.random.default_rng(0))
    bs = F(rng.standard_normal((300, 1)))
    _, rs = o.solve(s, bs, ext=oracle.EXT_SYM)
    assert rs["cls"] == oracle.SYMPD and rs["chol_failed"] == 1 and rs["route"] == 6 and rs["berr"] < 1e-14
    # singular symmetric: zero pivot -> solver failure -> SVD fallback
    z = F([[1.0, 0.0, 1.0], [0.0, 0.0, 0.0], [1.0, 0.0, 2.0]])
    _, rz = o.solve(z, F(np.ones((3, 1))), ext=oracle.EXT_SYM)
    assert rz["route"] == 5 and rz["fallback"] == 1 and rz["info"] == 2
    # tridiagonal: the tridiagonal route, same x as the band LU
    n = 2000
    dl, dm, du = _tridiag(n, rng)
    ab = np.zeros((3, n))
    ab[0, 1:], ab[1], ab[2, :-1] = du, dm, dl
    bt = F(rng.standard_normal((n, 3)))
    xb, rb = o.solve_band(F(ab), 1, 1, bt)
    xt, rt = o.solve_band(F(ab), 1, 1, bt, ext=oracle.EXT_TRIDIAG)
    assert rb["route"] == 1 and rt["route"] == 7 and rt["cls"] == oracle.BANDED and rt["fallback"] == 0
    np.testing.assert_allclose(xt, xb, rtol=1e-12, atol=1e-12 * np.abs(xb).max())
    assert abs(rt["rcond"] - rb["rcond"]) <= 1e-12 * rb["rcond"]
    dense = np.diag(dm) + np.diag(dl, -1) + np.diag(du, 1)
    xd, rd = o.solve(F(dense), bt, ext=oracle.EXT_TRIDIAG)
    assert rd["route"] == 7 and np.array_equal(xd, xt)
