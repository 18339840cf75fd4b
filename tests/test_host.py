"""Host-side logic without the GPU: the server's footprint rule, argument checks of the batched
and serving entry points, the precision option, and the seeded workload generators."""
import ctypes
import math
import os

import numpy as np
import pytest

from paper_2007_11208_amd import ada
from paper_2007_11208_amd import workloads as W


def _lib():
    if not os.path.exists(ada.LIB_PATH):
        pytest.skip("libada.so not built")
    return ada.lib()


def test_request_footprint():
    L = _lib()
    r = ada.Request()
    r.n, r.nrhs, r.lda, r.ldb, r.ldx = 200, 3, 200, 200, 200
    assert L.ada_request_footprint(ctypes.byref(r)) == 0  # small: the batch worker's fixed buffers
    r.n = r.lda = r.ldb = r.ldx = 1000
    big = L.ada_request_footprint(ctypes.byref(r))
    assert big == ada.workspace_size(1000, 3, ada.make_opts())
    r.keep_factor = 1
    kept = L.ada_request_footprint(ctypes.byref(r))
    assert kept >= ada.workspace_size(1000, 8, ada.make_opts()) + 1000 * 1000 * 8
    r.keep_factor, r.reuse = 0, 7
    assert L.ada_request_footprint(ctypes.byref(r)) == 0  # reuse: the kept factors' memory
    r.reuse, r.n, r.lda, r.ldb, r.ldx = 0, 100, 100, 100, 100
    r.opts = ada.make_opts(precision="bf16_ir")  # BF16 needs the single-system path
    assert L.ada_request_footprint(ctypes.byref(r)) > 0


def test_batched_and_server_reject_bad_arguments():
    L = _lib()
    assert L.ada_batched_workspace_size(0) == 0
    assert 0 < L.ada_batched_workspace_size(10) < L.ada_batched_workspace_size(10000)
    rc = L.ada_solve_batched(None, 1, None, None, None, None, None, 0, None, None, None)
    assert rc == ada.ERR_ARG
    h = ctypes.c_void_p()
    assert L.ada_server_create(None, None, 0, 1, ctypes.byref(h)) == ada.ERR_ARG
    t = ctypes.c_uint64()
    assert L.ada_submit(None, None, ctypes.byref(t)) == ada.ERR_ARG
    assert L.ada_poll(None, 1, None, None, 0) == ada.ERR_ARG
    assert L.ada_factor_release(None, 1) == ada.ERR_ARG


def test_precision_option():
    _lib()
    assert ada.make_opts().precision == ada.PREC_FP64
    assert ada.make_opts(precision="fp32_ir").precision == ada.PREC_FP32_IR
    assert ada.make_opts(precision="bf16_ir").precision == ada.PREC_BF16_IR
    with pytest.raises(ValueError):
        ada.make_opts(precision="fp16")


def test_serving_generator_sizes_and_mix():
    ns, kinds = [], []
    for k in range(400):
        kind, a, b = W.serving_system(k, n_hi=512)
        n = a.shape[0]
        assert 16 <= n <= 512 and b.shape[0] == n and 1 <= b.shape[1] <= 8
        ns.append(n)
        kinds.append(kind)
    # log-uniform: the median sits near the geometric mean of the range
    assert abs(math.log(np.median(ns)) - 0.5 * (math.log(16) + math.log(512))) < 0.35
    frac = {k: kinds.count(k) / len(kinds) for k, _ in W.BATCH_MIX}
    for k, p in W.BATCH_MIX:
        assert abs(frac[k] - p) < 0.08, (k, frac[k], p)
    # seeded: the same k gives the same system
    _, a1, b1 = W.serving_system(5, n_hi=512)
    _, a2, b2 = W.serving_system(5, n_hi=512)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_poisson_arrivals():
    t = W.poisson_arrivals(2000.0, 2.0, seed=1)
    assert np.all(np.diff(t) > 0) and t[0] > 0 and t[-1] < 2.0
    assert abs(len(t) - 4000) < 4 * math.sqrt(4000)  # Poisson count within four standard deviations
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 2000.0) < 0.1 / 2000.0


def test_extension_option_and_footprint():
    """The Section V extensions are bits of the options; a small request that asks for them takes a
    solve worker (the batched kernel runs the paper's routes only), so it has a footprint."""
    L = _lib()
    assert ada.make_opts().extensions == 0
    assert ada.make_opts(extensions=("sym",)).extensions == ada.EXT_SYM
    assert ada.make_opts(extensions=("sym",)).extensions == ada.EXT_SYM
    with pytest.raises(ValueError):
        ada.make_opts(extensions=("ldlt",))
    assert ctypes.sizeof(ada.Opts) == ada.make_opts().struct_size
    r = ada.Request()
    r.n, r.nrhs, r.lda, r.ldb, r.ldx = 100, 1, 100, 100, 100
    assert L.ada_request_footprint(ctypes.byref(r)) == 0
    r.opts = ada.make_opts(extensions=("sym",))
    assert L.ada_request_footprint(ctypes.byref(r)) == ada.workspace_size(100, 1, r.opts)
    assert ada.ROUTE_NAMES[ada.ROUTE_LDLT] == "ldlt" and ada.CLASS_NAMES[ada.CLASS_SYM] == "sym"


def test_band_workspace_keeps_the_maps():
    """The band-solve scratch holds the factor's chunk maps and output responses for the four sweep
    kinds (4 n (kl+ku) doubles for the responses alone), independent of the right-hand sides."""
    o = ada.make_opts(layout=ada.LAYOUT_BAND, kl_in=5, ku_in=5)
    w1 = ada.workspace_size(1_000_000, 1, o)
    assert w1 > 4 * 1_000_000 * 10 * 8
    w8 = ada.workspace_size(1_000_000, 8, o)
    assert w8 > w1
