"""Shared checks of the GPU parity tests against the oracle.

* backward error: the library reports eta = max_k ||b_k - A x_k||_inf /
  (||A||_inf ||x_k||_inf + ||b_k||_inf) for the x it returns; the oracle
  evaluates the same quantity on that same x with exact products and
  compensated sums, so the two must agree to a relative 1e-6 (both residuals
  are accurate to a few units in their last place; the norms of A differ by
  the order of their plain sums, at most 2 n eps relative);
* route decisions near the threshold: the estimate is only good to a factor
  of about 3 and the GPU's differs from the oracle's by summation order, so a
  system whose oracle rcond lies within a factor 4 of the threshold may take
  either side of it. Such systems are reported, and their route, fallback and
  x are not asserted (the class and band widths still are).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

EPS = float(np.finfo(np.float64).eps)
THRESHOLD = 0.5 * EPS  # rcond below this falls back to the SVD (strict "<")
GUARD = 4.0
BERR_RTOL = 1e-6

O = oracle.get()
near_threshold_cases: list = []


def near_threshold(rcond: float, thr: float = THRESHOLD) -> bool:
    """True when the oracle's rcond is within a factor GUARD of the threshold."""
    if not (rcond > 0.0) or not (thr > 0.0) or math.isinf(rcond):
        return False
    return abs(math.log10(rcond / thr)) < math.log10(GUARD)


def oracle_berr(a, b, x, band=None) -> float:
    """The oracle's backward error of x (dense matrix, or band storage with band=(kl, ku))."""
    x = np.asarray(x, dtype=np.float64).reshape(np.asarray(b).shape)
    if band is not None:
        return float(O.berr_band(a, band[0], band[1], b, x))
    w, _ = O.berr(a, b, x)
    return float(w)


def check_berr(reported: float, a, b, x, band=None) -> float:
    """The library's backward error equals the oracle's evaluation of the same x; returns it."""
    ob = oracle_berr(a, b, x, band)
    if math.isnan(ob):
        assert math.isnan(reported), (reported, ob)
        return ob
    assert abs(reported - ob) <= BERR_RTOL * ob + 1e-300, f"backward error {reported!r} vs oracle {ob!r}"
    return ob


def note_near_threshold(tag: str, rr: dict, r) -> None:
    msg = f"near the rcond threshold (not asserted): {tag} oracle rcond={rr['rcond']:.3e} route={rr['route']}" \
          f" | GPU rcond={r.rcond:.3e} route={r.route}"
    near_threshold_cases.append(msg)
    print(msg, flush=True)
