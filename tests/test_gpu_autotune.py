"""GPU tests of the band-solve autotuner (ada_autotune_band): it picks one of the candidate LDS
staging pieces for an order and band widths, keeps it in the context, and the solves that use it
give bit-identical results to the built-in choice (the piece changes how rows are staged, not the
arithmetic)."""
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


def band_system(n, kl, ku, nrhs, seed):
    rng = np.random.default_rng(seed)
    ab = rng.standard_normal((kl + ku + 1, n))
    # well conditioned for every width; interchanges still happen where a sub-diagonal entry is larger
    ab[ku] += (3.0 + 0.5 * (kl + ku)) * np.sign(ab[ku])
    for r in range(ku):
        ab[r, : ku - r] = 0.0
    for r in range(ku + 1, kl + ku + 1):
        ab[r, n - (r - ku):] = 0.0
    b = rng.standard_normal((n, nrhs))
    return np.asfortranarray(ab), np.asfortranarray(b)


@pytest.mark.parametrize("kl,ku,nrhs", [(5, 5, 1), (2, 3, 3), (1, 1, 1), (12, 9, 2)])
def test_autotuned_band_solve_is_bit_identical(ada, kl, ku, nrhs):
    print(f"case kl={kl} ku={ku} nrhs={nrhs}", flush=True)
    ab, b = band_system(30000, kl, ku, nrhs, seed=kl * 100 + ku)
    A = torch.from_numpy(ab).to("cuda:0")
    B = torch.from_numpy(b).to("cuda:0")
    plain = ada.Context(0)
    tuned = ada.Context(0)
    piece, ms = tuned.autotune_band(30000, kl, ku, nrhs)
    print(f"  piece {piece}, {ms:.3f} ms per solve", flush=True)
    assert piece in (8, 16, 32, 64) and ms > 0.0
    x0, r0 = ada.solve(A, B, layout="band", kl_in=kl, ku_in=ku, ctx=plain)
    x1, r1 = ada.solve(A, B, layout="band", kl_in=kl, ku_in=ku, ctx=tuned)
    torch.cuda.synchronize()
    assert r0.route == r1.route == "band_lu"
    assert torch.equal(x0, x1)
    assert r0.rcond == r1.rcond and r0.berr == r1.berr
    assert check_berr(r1.berr, ab, b, x1.cpu().numpy(), band=(kl, ku)) <= 1e-14


def test_autotune_rejects_bad_arguments(ada):
    ctx = ada.Context(0)
    for args in ((30000, 0, 0, 1), (30000, 20, 12, 1), (30000, 2, 2, 0), (30000, 2, 2, 65), (30000, -1, 3, 1),
                 (100, 2, 2, 1)):
        with pytest.raises(ada.AdaError):
            ctx.autotune_band(*args)
