"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles matrices; it holds none of
the solver's arithmetic. Both the GPU library's tests/benchmark and the CPU
oracle consume exactly the arrays produced here (Fortran order, float64).

The paper's experiments (Section III) use random banded (5 diagonals), lower
triangular, symmetric positive definite and dense systems; Fig. 3 shows the
sympd generator R^T R + I with R = randu - 0.5. The recipes below follow those
descriptions at the sizes of the benchmark configurations.
"""
from __future__ import annotations

import math

import numpy as np


def rng_for(cfg: int, k: int) -> np.random.Generator:
    """Seed convention: default_rng(100*cfg + k)."""
    return np.random.default_rng(100 * int(cfg) + int(k))


def _f(a: np.ndarray) -> np.ndarray:
    return np.asfortranarray(a, dtype=np.float64)


def dense_general(n: int, rng: np.random.Generator) -> np.ndarray:
    """N(0,1) entries plus 16*I."""
    a = rng.standard_normal((n, n))
    a[np.diag_indices(n)] += 16.0
    return _f(a)


def spd(n: int, rng: np.random.Generator) -> np.ndarray:
    """G^T G / n + I with G N(0,1); symmetrised so both triangles are bitwise equal."""
    g = rng.standard_normal((n, n))
    m = g.T @ g / n
    m = 0.5 * (m + m.T)
    m[np.diag_indices(n)] += 1.0
    return _f(m)


def fig3_sympd(n: int, rng: np.random.Generator) -> np.ndarray:
    """Fig. 3 of the paper: R = randu(n,n) - 0.5; A = R^T R; A.diag() += 1."""
    r = rng.random((n, n)) - 0.5
    a = r.T @ r
    a = 0.5 * (a + a.T)
    a[np.diag_indices(n)] += 1.0
    return _f(a)


def triangular(n: int, rng: np.random.Generator, upper: bool = True, scaled: bool = False) -> np.ndarray:
    """N(0,1) strictly on one side of the diagonal, diagonal 1+|N(0,1)|.

    scaled=True divides the off-diagonal entries by sqrt(n); that keeps the
    condition number moderate at large n (the unscaled family has a condition
    number that grows exponentially with n).
    """
    a = rng.standard_normal((n, n))
    d = 1.0 + np.abs(rng.standard_normal(n))
    a = np.triu(a, 1) if upper else np.tril(a, -1)
    if scaled:
        a = a / np.sqrt(n)
    a[np.diag_indices(n)] = d
    return _f(a)


def banded_storage(n: int, kl: int, ku: int, rng: np.random.Generator) -> np.ndarray:
    """Band matrix in LAPACK band storage: AB[ku+i-j, j] = A[i, j], (kl+ku+1) x n.

    Off-diagonal band entries N(0,1); the diagonal is 5 + the sum of the absolute
    off-diagonal band entries of its row (strict diagonal dominance).
    """
    ab = rng.standard_normal((kl + ku + 1, n))
    for r in range(kl + ku + 1):
        d = ku - r  # column offset j - i of this storage row
        if d > 0:
            ab[r, :d] = 0.0  # entries (i, j) with i = j - d < 0
        elif d < 0:
            ab[r, n + d:] = 0.0  # entries with i = j - d >= n
    rowabs = np.zeros(n)
    for r in range(kl + ku + 1):
        d = ku - r
        if d == 0:
            continue
        if d > 0:
            rowabs[: n - d] += np.abs(ab[r, d:])
        else:
            rowabs[-d:] += np.abs(ab[r, : n + d])
    ab[ku, :] = 5.0 + rowabs
    return _f(ab)


def band_to_dense(ab: np.ndarray, kl: int, ku: int) -> np.ndarray:
    n = ab.shape[1]
    a = np.zeros((n, n), order="F")
    for r in range(kl + ku + 1):
        d = ku - r
        if d >= 0:
            j = np.arange(d, n)
        else:
            j = np.arange(0, n + d)
        a[j - d, j] = ab[r, j]
    return a


def band_matvec(ab: np.ndarray, kl: int, ku: int, x: np.ndarray) -> np.ndarray:
    """b = A x for band storage (used to build right-hand sides)."""
    n = ab.shape[1]
    x2 = x.reshape(n, -1)
    b = np.zeros_like(x2)
    for r in range(kl + ku + 1):
        d = ku - r
        if d >= 0:
            j = np.arange(d, n)
        else:
            j = np.arange(0, n + d)
        b[j - d, :] += ab[r, j][:, None] * x2[j, :]
    return _f(b.reshape(x.shape))


def banded_dense(n: int, kl: int, ku: int, rng: np.random.Generator) -> np.ndarray:
    return band_to_dense(banded_storage(n, kl, ku, rng), kl, ku)


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian with the sign fix."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    return _f(q)


def prescribed_spectrum(n: int, s: np.ndarray, rng: np.random.Generator, symmetric: bool = False) -> np.ndarray:
    """U diag(s) V^T with Haar U, V (V = U when symmetric)."""
    u = haar_orthogonal(n, rng)
    v = u if symmetric else haar_orthogonal(n, rng)
    a = (u * np.asarray(s, dtype=np.float64)[None, :]) @ v.T
    return _f(a)


def ill_conditioned(n: int, rng: np.random.Generator, smin: float = 1e-14) -> np.ndarray:
    """U diag(s) V^T with s log-spaced from 1 down to smin."""
    s = np.logspace(0.0, np.log10(smin), n)
    return prescribed_spectrum(n, s, rng)


def sym_indefinite(n: int, rng: np.random.Generator) -> np.ndarray:
    """I + (W + W^T)/sqrt(2) * 2/sqrt(n): symmetric, positive and dominant diagonal
    entries, so it passes the sympd heuristic, but indefinite (spectrum ~[-3, 5])."""
    w = rng.standard_normal((n, n))
    a = (w + w.T) / np.sqrt(2.0) * (2.0 / np.sqrt(n))
    a[np.diag_indices(n)] += 1.0
    return _f(a)


def x_true(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    return _f(rng.standard_normal((n, nrhs)))


def rhs_for(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    return _f(a @ x)


def spectrum_system_torch(n: int, kappa: float, spd: bool, nrhs: int, seed: int, device):
    """U diag(s) V^T (V = U for SPD) with Haar U, V (QR of a Gaussian, signs fixed), s log-spaced
    from 1 to 1/kappa, so the 2-norm condition number is kappa by construction; b = A x_true,
    x_true ~ N(0,1). Formed with torch on `device` (input generation only: at n = 16384 the host
    QR takes minutes). Returns column-major (A, B, x_true)."""
    import math

    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar():
        q, r = torch.linalg.qr(torch.randn(n, n, dtype=torch.float64, device=device, generator=g))
        return q * torch.sign(torch.diagonal(r))[None, :]

    u = haar()
    v = u if spd else haar()
    s = torch.logspace(0.0, -math.log10(kappa), n, dtype=torch.float64, device=device)
    a = (u * s[None, :]) @ v.T
    del u, v
    x = torch.randn(n, nrhs, dtype=torch.float64, device=device, generator=g)
    b = a @ x
    return a.T.contiguous().T, b.T.contiguous().T, x


# ---- the benchmark systems -------------------------------------------------

SMALL_CASES = ("a_dense", "b_spd", "c_upper", "c_upper_scaled", "d_banded", "e_illcond", "e_illcond_1e18")
LARGE_CASES = ("dense", "spd", "lower", "lower_scaled", "banded", "symindef")


def small_case(name: str, k: int = 0, nrhs: int = 1):
    """The five 1-RHS systems of the small configuration (plus two labelled variants).

    Returns (A, B) with A dense n x n."""
    g = rng_for(0, k)
    if name == "a_dense":
        a = dense_general(256, g)
    elif name == "b_spd":
        a = spd(256, g)
    elif name == "c_upper":
        a = triangular(256, g, upper=True)
    elif name == "c_upper_scaled":
        a = triangular(256, g, upper=True, scaled=True)
    elif name == "d_banded":
        a = banded_dense(1024, 2, 2, g)
    elif name == "e_illcond":
        a = ill_conditioned(64, g, 1e-14)
    elif name == "e_illcond_1e18":
        a = ill_conditioned(64, g, 1e-18)
    else:
        raise ValueError(name)
    x = x_true(a.shape[0], nrhs, g)
    return a, rhs_for(a, x)


def large_case(name: str, nrhs: int = 1, k: int = 0, n: int | None = None):
    """Systems of the large single-system configuration.

    Dense/SPD/lower-triangular n=8192, banded n=1,000,000 (kl=ku=5, band storage),
    symmetric-indefinite n=4096. Returns (A, B, layout) where layout is
    ("dense",) or ("band", kl, ku)."""
    g = rng_for(1, k)
    if name == "dense":
        a = dense_general(n or 8192, g)
    elif name == "spd":
        a = spd(n or 8192, g)
    elif name == "lower":
        a = triangular(n or 8192, g, upper=False)
    elif name == "lower_scaled":
        a = triangular(n or 8192, g, upper=False, scaled=True)
    elif name == "symindef":
        a = sym_indefinite(n or 4096, g)
    elif name == "banded":
        nn = n or 1_000_000
        ab = banded_storage(nn, 5, 5, g)
        x = x_true(nn, nrhs, g)
        return ab, band_matvec(ab, 5, 5, x), ("band", 5, 5)
    else:
        raise ValueError(name)
    x = x_true(a.shape[0], nrhs, g)
    return a, rhs_for(a, x), ("dense",)


BATCH_MIX = (("dense", 0.40), ("spd", 0.30), ("banded", 0.15), ("triangular", 0.10), ("spectrum", 0.05))


def batched_case(count: int, k: int = 0, n_lo: int = 8, n_hi: int = 256, nrhs_hi: int = 8):
    """Many independent small systems: n uniform in [n_lo, n_hi], nrhs uniform in [1, nrhs_hi],
    class mix 40% dense general, 30% SPD, 15% banded (kl, ku uniform in [1, 4]), 10% triangular
    (upper or lower, off-diagonals N(0,1)), 5% prescribed spectrum with condition 1e15.
    Returns a list of (kind, A, B)."""
    g = rng_for(3, k)
    kinds = [m[0] for m in BATCH_MIX]
    probs = np.array([m[1] for m in BATCH_MIX])
    out = []
    for _ in range(count):
        n = int(g.integers(n_lo, n_hi + 1))
        nrhs = int(g.integers(1, nrhs_hi + 1))
        kind = kinds[int(g.choice(len(kinds), p=probs))]
        if kind == "dense":
            a = dense_general(n, g)
        elif kind == "spd":
            a = spd(n, g)
        elif kind == "banded":
            a = banded_dense(n, int(g.integers(1, 5)), int(g.integers(1, 5)), g)
        elif kind == "triangular":
            a = triangular(n, g, upper=bool(g.integers(0, 2)))
        else:
            a = prescribed_spectrum(n, np.logspace(0, -15, n), g)
        out.append((kind, a, rhs_for(a, x_true(n, nrhs, g))))
    return out


def serving_system(k: int, n_lo: int = 16, n_hi: int = 4096, nrhs_hi: int = 8):
    """One request system of the serving configuration: n log-uniform in [n_lo, n_hi],
    nrhs uniform in [1, nrhs_hi], the batched class mix. Returns (kind, A, B)."""
    g = rng_for(4, k)
    n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
    nrhs = int(g.integers(1, nrhs_hi + 1))
    kinds = [m[0] for m in BATCH_MIX]
    probs = np.array([m[1] for m in BATCH_MIX])
    kind = kinds[int(g.choice(len(kinds), p=probs))]
    if kind == "dense":
        a = dense_general(n, g)
    elif kind == "spd":
        a = spd(n, g)
    elif kind == "banded":
        a = banded_dense(n, int(g.integers(1, 5)), int(g.integers(1, 5)), g)
    elif kind == "triangular":
        a = triangular(n, g, upper=bool(g.integers(0, 2)))
    else:
        a = prescribed_spectrum(n, np.logspace(0, -15, n), g)
    return kind, a, rhs_for(a, x_true(n, nrhs, g))


def poisson_arrivals(rate: float, duration: float, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate over [0, duration)."""
    g = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)
