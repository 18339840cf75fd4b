"""TEST INFRASTRUCTURE ONLY: ctypes binding of the plain FP64 CPU oracle.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package. It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libada_oracle.so")
SRC_PATH = os.path.join(_HERE, "ada_oracle.c")

GENERAL, BANDED, TRI_UPPER, TRI_LOWER, SYMPD, SYM = 0, 1, 2, 3, 4, 5
CLASS_NAMES = {GENERAL: "general", BANDED: "banded", TRI_UPPER: "tri_upper", TRI_LOWER: "tri_lower", SYMPD: "sympd",
               SYM: "sym"}
ROUTE_NAMES = {0: "none", 1: "band_lu", 2: "tri", 3: "chol", 4: "lu", 5: "svd", 6: "ldlt", 7: "tridiag"}
# Section V extensions (future work of the paper), off by default
EXT_SYM, EXT_TRIDIAG = 1, 2
EPS = np.finfo(np.float64).eps


def build(src: str = SRC_PATH, out: str = LIB_PATH, extra: tuple = ()) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", out, src, "-lm", *extra]
    subprocess.run(cmd, check=True)
    return out


class _Detect(ctypes.Structure):
    _fields_ = [("kl", ctypes.c_int32), ("ku", ctypes.c_int32), ("banded", ctypes.c_int32),
                ("likely_sympd", ctypes.c_int32), ("cls", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cls", ctypes.c_int32), ("kl", ctypes.c_int32),
                ("ku", ctypes.c_int32), ("route", ctypes.c_int32), ("chol_failed", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("info", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("rcond", ctypes.c_double), ("berr", ctypes.c_double)]


_P = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)


def _dp(a):
    return a.ctypes.data_as(_P)


def _ip(a):
    return a.ctypes.data_as(_PI)


class Oracle:
    """Wraps one loaded copy of the oracle library (tests may load mutated copies)."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            build(out=path)
        self.lib = ctypes.CDLL(path)
        L = self.lib
        i, d = ctypes.c_int, ctypes.c_double
        L.orc_band_scan.argtypes = [i, _P, i, _PI, _PI]
        L.orc_is_banded.argtypes = [ctypes.c_int64] * 3
        L.orc_is_banded.restype = i
        L.orc_likely_sympd.argtypes = [i, _P, i]
        L.orc_likely_sympd.restype = i
        L.orc_detect.argtypes = [i, _P, i, ctypes.POINTER(_Detect)]
        L.orc_getrf.argtypes = [i, _P, i, _PI]
        L.orc_getrf.restype = i
        L.orc_getrs.argtypes = [i, i, i, _P, i, _PI, _P, i]
        L.orc_potrf_lower.argtypes = [i, _P, i]
        L.orc_potrf_lower.restype = i
        L.orc_potrs_lower.argtypes = [i, i, _P, i, _P, i]
        L.orc_trsv.argtypes = [i, i, i, i, _P, i, _P]
        L.orc_gbtrf.argtypes = [i, i, i, _P, i, _PI]
        L.orc_gbtrf.restype = i
        L.orc_gbtrs.argtypes = [i, i, i, i, i, _P, i, _PI, _P, i]
        for nm in ("orc_norm1_general", "orc_norm1_sym_lower"):
            getattr(L, nm).argtypes = [i, _P, i]
            getattr(L, nm).restype = d
        L.orc_norm1_tri.argtypes = [i, i, _P, i]
        L.orc_norm1_tri.restype = d
        L.orc_norm1_band.argtypes = [i, i, i, _P, i, i]
        L.orc_norm1_band.restype = d
        L.orc_rcond_general.argtypes = [i, _P, i, _PI, d, _PI]
        L.orc_rcond_general.restype = d
        L.orc_rcond_chol.argtypes = [i, _P, i, d, _PI]
        L.orc_rcond_chol.restype = d
        L.orc_rcond_tri.argtypes = [i, i, _P, i, d, _PI]
        L.orc_rcond_tri.restype = d
        L.orc_rcond_band.argtypes = [i, i, i, _P, i, _PI, d, _PI]
        L.orc_rcond_band.restype = d
        L.orc_jacobi_svd.argtypes = [i, _P, i, _P, i, _P, i]
        L.orc_jacobi_svd.restype = i
        L.orc_svd_lstsq.argtypes = [i, i, _P, i, _P, i, _P, i, _P, _PI]
        L.orc_svd_lstsq.restype = i
        L.orc_berr.argtypes = [i, i, _P, i, _P, i, _P, i, _P]
        L.orc_berr.restype = d
        L.orc_berr_band.argtypes = [i, i, i, i, _P, i, _P, i, _P, i]
        L.orc_berr_band.restype = d
        L.orc_solve.argtypes = [i, i, _P, i, _P, i, _P, i, i, d, i, ctypes.POINTER(_Result)]
        L.orc_solve_band.argtypes = [i, i, i, i, _P, i, _P, i, _P, i, i, d, ctypes.c_int64, ctypes.POINTER(_Result)]
        L.orc_solve_ext.argtypes = [i, i, _P, i, _P, i, _P, i, i, d, i, i, ctypes.POINTER(_Result)]
        L.orc_solve_band_ext.argtypes = [i, i, i, i, _P, i, _P, i, _P, i, i, d, ctypes.c_int64, i,
                                         ctypes.POINTER(_Result)]
        L.orc_sytrf_bk.argtypes = [i, _P, i, _P, _P, _PI]
        L.orc_sytrf_bk.restype = i
        L.orc_sytrs_bk.argtypes = [i, i, _P, i, _P, _P, _PI, _P, i]
        L.orc_rcond_sym_bk.argtypes = [i, _P, i, _P, _P, _PI, d, _PI]
        L.orc_rcond_sym_bk.restype = d
        L.orc_gttrf.argtypes = [i, _P, _P, _P, _P, _PI]
        L.orc_gttrf.restype = i
        L.orc_gttrs.argtypes = [i, i, i, _P, _P, _P, _P, _PI, _P, i]
        L.orc_rcond_gt.argtypes = [i, _P, _P, _P, _P, _PI, d, _PI]
        L.orc_rcond_gt.restype = d
        L.orc_num_threads.restype = i

    # ---- helpers ----
    @staticmethod
    def _mat(a):
        a = np.asfortranarray(a, dtype=np.float64)
        return a

    def num_threads(self) -> int:
        return int(self.lib.orc_num_threads())

    def set_threads(self, k: int) -> None:
        """Threads of the oracle's parallel loops from now on (OpenMP's runtime setting)."""
        self.lib.omp_set_num_threads(ctypes.c_int(int(k)))

    def band_scan(self, a):
        a = self._mat(a)
        kl, ku = ctypes.c_int(), ctypes.c_int()
        self.lib.orc_band_scan(a.shape[0], _dp(a), a.shape[0], ctypes.byref(kl), ctypes.byref(ku))
        return kl.value, ku.value

    def is_banded(self, n, kl, ku) -> bool:
        return bool(self.lib.orc_is_banded(n, kl, ku))

    def likely_sympd(self, a) -> bool:
        a = self._mat(a)
        return bool(self.lib.orc_likely_sympd(a.shape[0], _dp(a), a.shape[0]))

    def detect(self, a) -> dict:
        a = self._mat(a)
        d = _Detect()
        self.lib.orc_detect(a.shape[0], _dp(a), a.shape[0], ctypes.byref(d))
        return {"kl": d.kl, "ku": d.ku, "banded": bool(d.banded), "likely_sympd": bool(d.likely_sympd), "cls": d.cls}

    def getrf(self, a):
        lu = self._mat(a).copy(order="F")
        n = lu.shape[0]
        ipiv = np.zeros(n, dtype=np.intc)
        info = self.lib.orc_getrf(n, _dp(lu), n, _ip(ipiv))
        return lu, ipiv, info

    def getrs(self, lu, ipiv, b, trans=False):
        x = self._mat(b).copy(order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        n = lu.shape[0]
        self.lib.orc_getrs(int(trans), n, x2.shape[1], _dp(lu), n, _ip(ipiv), _dp(x2), n)
        return x2.reshape(x.shape, order="F")

    def potrf(self, a):
        l = self._mat(a).copy(order="F")
        n = l.shape[0]
        info = self.lib.orc_potrf_lower(n, _dp(l), n)
        return np.asfortranarray(np.tril(l)), info

    def potrs(self, l, b):
        x = self._mat(b).copy(order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        l = self._mat(l)
        n = l.shape[0]
        self.lib.orc_potrs_lower(n, x2.shape[1], _dp(l), n, _dp(x2), n)
        return x2.reshape(x.shape, order="F")

    def trsv(self, t, b, upper, trans=False, unit=False):
        t = self._mat(t)
        x = np.array(b, dtype=np.float64, copy=True)
        self.lib.orc_trsv(int(upper), int(trans), int(unit), t.shape[0], _dp(t), t.shape[0], _dp(x))
        return x

    def gbtrf(self, ab_in, kl, ku):
        """ab_in: LAPACK band storage (kl+ku+1) x n; returns the factored (2kl+ku+1) x n array, ipiv, info."""
        ab_in = self._mat(ab_in)
        n = ab_in.shape[1]
        ab = np.zeros((2 * kl + ku + 1, n), order="F")
        ab[kl:, :] = ab_in
        ipiv = np.zeros(n, dtype=np.intc)
        info = self.lib.orc_gbtrf(n, kl, ku, _dp(ab), ab.shape[0], _ip(ipiv))
        return ab, ipiv, info

    def gbtrs(self, ab, kl, ku, ipiv, b, trans=False):
        x = self._mat(b).copy(order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        n = ab.shape[1]
        self.lib.orc_gbtrs(int(trans), n, kl, ku, x2.shape[1], _dp(ab), ab.shape[0], _ip(ipiv), _dp(x2), n)
        return x2.reshape(x.shape, order="F")

    def norm1_general(self, a):
        a = self._mat(a)
        return self.lib.orc_norm1_general(a.shape[0], _dp(a), a.shape[0])

    def norm1_sym_lower(self, a):
        a = self._mat(a)
        return self.lib.orc_norm1_sym_lower(a.shape[0], _dp(a), a.shape[0])

    def norm1_tri(self, a, upper):
        a = self._mat(a)
        return self.lib.orc_norm1_tri(int(upper), a.shape[0], _dp(a), a.shape[0])

    def rcond_general(self, a):
        lu, ipiv, info = self.getrf(a)
        ns = ctypes.c_int()
        r = self.lib.orc_rcond_general(lu.shape[0], _dp(lu), lu.shape[0], _ip(ipiv), self.norm1_general(a), ctypes.byref(ns))
        return r, ns.value

    def rcond_chol(self, a):
        l, info = self.potrf(a)
        assert info == 0
        l = self._mat(l)
        ns = ctypes.c_int()
        r = self.lib.orc_rcond_chol(l.shape[0], _dp(l), l.shape[0], self.norm1_sym_lower(a), ctypes.byref(ns))
        return r, ns.value

    def rcond_tri(self, a, upper):
        a = self._mat(a)
        ns = ctypes.c_int()
        r = self.lib.orc_rcond_tri(int(upper), a.shape[0], _dp(a), a.shape[0], self.norm1_tri(a, upper), ctypes.byref(ns))
        return r, ns.value

    def rcond_band(self, ab_in, kl, ku):
        ab_in = self._mat(ab_in)
        n = ab_in.shape[1]
        anorm = self.lib.orc_norm1_band(n, kl, ku, _dp(ab_in), ab_in.shape[0], ku)
        ab, ipiv, info = self.gbtrf(ab_in, kl, ku)
        ns = ctypes.c_int()
        r = self.lib.orc_rcond_band(n, kl, ku, _dp(ab), ab.shape[0], _ip(ipiv), anorm, ctypes.byref(ns))
        return r, ns.value

    def jacobi_svd(self, a, max_sweeps=30):
        u = self._mat(a).copy(order="F")
        n = u.shape[0]
        v = np.zeros((n, n), order="F")
        s = np.zeros(n)
        sweeps = self.lib.orc_jacobi_svd(n, _dp(u), n, _dp(v), n, _dp(s), max_sweeps)
        return u, s, v, sweeps

    def svd_lstsq(self, a, b):
        a = self._mat(a)
        b = self._mat(b)
        b2 = b.reshape(b.shape[0], -1, order="F")
        n = a.shape[0]
        x = np.zeros_like(b2, order="F")
        s = np.zeros(n)
        sw = ctypes.c_int()
        rank = self.lib.orc_svd_lstsq(n, b2.shape[1], _dp(a), n, _dp(b2), n, _dp(x), n, _dp(s), ctypes.byref(sw))
        return x.reshape(b.shape, order="F"), rank, s, sw.value

    def berr(self, a, b, x):
        a, b, x = self._mat(a), self._mat(b), self._mat(x)
        b2 = b.reshape(b.shape[0], -1, order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        n = a.shape[0]
        per = np.zeros(b2.shape[1])
        w = self.lib.orc_berr(n, b2.shape[1], _dp(a), n, _dp(b2), n, _dp(x2), n, _dp(per))
        return w, per

    def berr_band(self, ab, kl, ku, b, x):
        """Backward error of x for the band-storage matrix (kl+ku+1) x n (accurate residual)."""
        ab, b, x = self._mat(ab), self._mat(b), self._mat(x)
        b2 = b.reshape(b.shape[0], -1, order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        n = ab.shape[1]
        return self.lib.orc_berr_band(n, kl, ku, b2.shape[1], _dp(ab), ab.shape[0], _dp(b2), n, _dp(x2), n)

    def sytrf_bk(self, a):
        """Bunch-Kaufman LDL^T of the lower triangle: returns L (unit lower, as a full matrix), d, e
        (the sub-diagonal of the 2x2 blocks), perm (P A P^T = L D L^T, row i of P A is row perm[i])
        and info."""
        f = self._mat(a).copy(order="F")
        n = f.shape[0]
        d, e = np.zeros(n), np.zeros(n)
        perm = np.zeros(n, dtype=np.intc)
        info = self.lib.orc_sytrf_bk(n, _dp(f), n, _dp(d), _dp(e), _ip(perm))
        return np.tril(f, -1) + np.eye(n), d, e, perm, info

    def sytrs_bk(self, l, d, e, perm, b):
        x = self._mat(b).copy(order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        l = self._mat(l)
        n = l.shape[0]
        self.lib.orc_sytrs_bk(n, x2.shape[1], _dp(l), n, _dp(d), _dp(e), _ip(perm), _dp(x2), n)
        return x2.reshape(x.shape, order="F")

    def rcond_sym_bk(self, a):
        l, d, e, perm, info = self.sytrf_bk(a)
        assert info == 0
        l = self._mat(l)
        ns = ctypes.c_int()
        r = self.lib.orc_rcond_sym_bk(l.shape[0], _dp(l), l.shape[0], _dp(d), _dp(e), _ip(perm),
                                      self.norm1_sym_lower(a), ctypes.byref(ns))
        return r, ns.value

    def gttrf(self, dl, dm, du):
        """Tridiagonal LU with partial pivoting: returns dl (multipliers), dm, du, du2, ipiv, info."""
        dl, dm, du = (np.array(v, dtype=np.float64, copy=True) for v in (dl, dm, du))
        n = dm.shape[0]
        dl2, du_2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        dl2[: n - 1] = dl
        du_2[: n - 1] = du
        du2 = np.zeros(max(n, 1))
        ipiv = np.zeros(n, dtype=np.intc)
        info = self.lib.orc_gttrf(n, _dp(dl2), _dp(dm), _dp(du_2), _dp(du2), _ip(ipiv))
        return dl2[: n - 1], dm, du_2[: n - 1], du2[: max(n - 2, 0)], ipiv, info

    def gttrs(self, dl, dm, du, du2, ipiv, b, trans=False):
        x = self._mat(b).copy(order="F")
        x2 = x.reshape(x.shape[0], -1, order="F")
        n = dm.shape[0]
        pad = lambda v: np.concatenate([np.asarray(v, dtype=np.float64), np.zeros(2)])
        self.lib.orc_gttrs(int(trans), n, x2.shape[1], _dp(pad(dl)), _dp(np.asarray(dm, dtype=np.float64)),
                           _dp(pad(du)), _dp(pad(du2)), _ip(np.asarray(ipiv, dtype=np.intc)), _dp(x2), n)
        return x2.reshape(x.shape, order="F")

    def rcond_gt(self, dl, dm, du):
        """Condition estimate from the tridiagonal LU of the matrix with diagonals dl, dm, du."""
        dm = np.asarray(dm, dtype=np.float64)
        n = dm.shape[0]
        anorm = np.abs(dm).copy()
        anorm[1:] += np.abs(np.asarray(du, dtype=np.float64))
        anorm[:-1] += np.abs(np.asarray(dl, dtype=np.float64))
        f = self.gttrf(dl, dm, du)
        assert f[5] == 0
        pad = lambda v: np.concatenate([np.asarray(v, dtype=np.float64), np.zeros(2)])
        fl, fd, fu, fu2 = pad(f[0]), np.ascontiguousarray(f[1]), pad(f[2]), pad(f[3])
        ns = ctypes.c_int()
        r = self.lib.orc_rcond_gt(n, _dp(fl), _dp(fd), _dp(fu), _dp(fu2), _ip(f[4]), float(anorm.max()),
                                  ctypes.byref(ns))
        return r, ns.value

    def solve(self, a, b, no_approx=False, rcond_threshold=-1.0, force_general=False, ext=0):
        a = self._mat(a)
        b = self._mat(b)
        b2 = b.reshape(b.shape[0], -1, order="F")
        n = a.shape[0]
        x = np.zeros_like(b2, order="F")
        r = _Result()
        self.lib.orc_solve_ext(n, b2.shape[1], _dp(a), a.shape[0], _dp(b2), b2.shape[0], _dp(x), n,
                               int(no_approx), float(rcond_threshold), int(force_general), int(ext), ctypes.byref(r))
        return x.reshape(b.shape, order="F"), _res_dict(r)

    def solve_band(self, ab, kl, ku, b, no_approx=False, rcond_threshold=-1.0, dense_limit=1 << 26, ext=0):
        ab = self._mat(ab)
        b = self._mat(b)
        b2 = b.reshape(b.shape[0], -1, order="F")
        n = ab.shape[1]
        x = np.zeros_like(b2, order="F")
        r = _Result()
        self.lib.orc_solve_band_ext(n, kl, ku, b2.shape[1], _dp(ab), ab.shape[0], _dp(b2), b2.shape[0], _dp(x), n,
                                    int(no_approx), float(rcond_threshold), int(dense_limit), int(ext),
                                    ctypes.byref(r))
        return x.reshape(b.shape, order="F"), _res_dict(r)


def _res_dict(r: _Result) -> dict:
    return {k: getattr(r, k) for k, _ in _Result._fields_}


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
