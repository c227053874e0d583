"""Status paths through the C ABI on the GPU, and block widths above the
tiled entry path (b = 33 and 64).

  MLG_ERR_ISOLATED   a node whose degree is zero (direct: every weight
                     underflows) or below what the NFFT degree pass can tell
                     from zero (its measured error margin); a genuinely small
                     degree that the pass does resolve is accepted and matches
                     the oracle row by row within the FP64 gate (1e-6)
  MLG_WARN_NOT_CONVERGED   the eigensolver with max_restarts = 0 and an
                     unreachable tolerance: info filled, the best Ritz pairs
                     returned (ascending, orthonormal)
  MLG_ERR_ARG        a non-finite point coordinate (direct and NFFT layers)
  MLG_ERR_RANGE      an NFFT bandwidth that is not a power of two (N = 48)
"""
import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2007_05239_amd.mlg as m
    return m


def case_id(msg):
    print(msg, flush=True)


def cluster_with(point, n=2000, seed=901):
    """n points uniform in the unit ball of R^3 plus one extra point."""
    P = gen.uniform_ball(n, 3, 1.0, seed)
    return np.ascontiguousarray(np.vstack([P, np.asarray(point, dtype=np.float64)[None, :]]))


def expect_status(mlg, code, fn):
    with pytest.raises(mlg.MlgError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


@pytest.mark.parametrize("prec", [64, 32])
def test_isolated_direct(mlg, prec):
    pts = cluster_with([100.0, 100.0, 100.0])
    case_id("isolated direct FP%d n=%d" % (prec, pts.shape[0]))
    expect_status(mlg, mlg.MLG_ERR_ISOLATED,
                  lambda: mlg.Graph([pts], [0.3], mlg.kparams("direct", precision=prec)))


def test_isolated_nfft_unresolvable_degree(mlg):
    # nearest distance 3, sigma 0.3: weights about e^-100, far below the
    # FP64 NFFT degree pass's error
    pts = cluster_with([4.0, 0.0, 0.0])
    case_id("isolated NFFT n=%d" % pts.shape[0])
    expect_status(mlg, mlg.MLG_ERR_ISOLATED,
                  lambda: mlg.Graph([pts], [0.3], mlg.kparams("nfft", precision=32, N=0)))


def test_small_degree_resolved_nfft(mlg):
    # nearest distance about 0.8: degree ~1e-4 of the typical one, well
    # above the degree pass's error; accepted, and every degree row matches
    # the oracle within the FP64 gate, row by row
    pts = cluster_with([1.8, 0.0, 0.0])
    case_id("small degree NFFT n=%d" % pts.shape[0])
    g = mlg.Graph([pts], [0.3], mlg.kparams("nfft", precision=32, N=0))
    deg = g.degrees(0)
    ref = oracle.degrees(pts, 0.3)
    assert ref[-1] < 1e-3 * np.median(ref)
    assert (np.abs(deg - ref) / ref).max() <= 1e-6
    g.close()


def test_not_converged_returns_best_pairs(mlg):
    n, k = 600, 8
    pts, _ = gen.gaussian_mixture(n, 3, 4, 0.08, 911)
    g = mlg.Graph([pts], [0.2], mlg.kparams("direct", precision=64))
    case_id("lanczos max_restarts=0 n=%d k=%d" % (n, k))
    lam, V, info = g.lanczos_eigs(0, k, block=2, tol=1e-15, max_restarts=0, seed=3)
    assert not info["converged"]
    assert info["restarts"] == 0 and info["iters"] >= 1 and info["matvecs"] >= 2
    assert 0 <= info["nconv"] < k and info["max_resid"] > 1e-15
    assert np.all(np.isfinite(lam)) and np.all(np.diff(lam) >= 0)
    assert lam[0] > -1e-10 and lam[-1] < 2.0
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    # each pair's residual is what info reports at most
    LV = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, V)
    res = np.linalg.norm(LV - V * lam[None, :], axis=0)
    assert res.max() <= info["max_resid"] * 1.01 + 1e-10
    # the best pairs still bracket the true spectrum: no Ritz value below
    # the smallest eigenvalue, and lambda_0 (= 0) is approximated
    lo, _ = oracle.eigs_dense([oracle.Layer(pts, 0.2)], k)
    assert np.all(lam >= lo - 1e-10)
    g.close()


@pytest.mark.parametrize("method", ["direct", "nfft"])
def test_non_finite_point(mlg, method):
    pts, _ = gen.gaussian_mixture(500, 3, 3, 0.1, 921)
    for bad in (np.nan, np.inf):
        P = pts.copy()
        P[123, 1] = bad
        case_id("non-finite point %s %r" % (method, bad))
        expect_status(mlg, mlg.MLG_ERR_ARG,
                      lambda: mlg.Graph([P], [0.3], mlg.kparams(method, precision=32)))


def test_bandwidth_not_power_of_two(mlg):
    pts, _ = gen.gaussian_mixture(500, 3, 3, 0.1, 931)
    case_id("NFFT N=48")
    expect_status(mlg, mlg.MLG_ERR_RANGE,
                  lambda: mlg.Graph([pts], [0.3], mlg.kparams("nfft", precision=32, N=48)))


@pytest.mark.parametrize("b", [33, 64])
@pytest.mark.parametrize("method,prec,gate", [("nfft", 32, 1e-4), ("direct", 64, 1e-12)])
def test_wide_blocks_against_oracle(mlg, b, method, prec, gate):
    """Blocks wider than the entry kernel's LDS tile (32 vectors): strides 64."""
    n = 3000
    p3, _ = gen.gaussian_mixture(n, 3, 4, 0.05, 941)
    p2 = gen.uniform_ball(n, 2, 1.0, 942)
    sig = [0.15, 0.4]
    kp = mlg.kparams(method, precision=prec, N=0, window=6)
    g = mlg.Graph([p3, p2], sig, [kp, kp])
    X = gen.test_vectors(n, b, 943)
    case_id("wide block %s FP%d b=%d" % (method, prec, b))
    Y = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X)
    ref = oracle.lsym_matvec([oracle.Layer(p3, sig[0]), oracle.Layer(p2, sig[1])], X)
    err = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= gate, err
    Yw = g.laplacian_matvec(0, mlg.MLG_OP_W, X)
    refw = oracle.kernel_rows(p3, sig[0], X)
    errw = np.linalg.norm(Yw - refw, axis=0) / np.linalg.norm(refw, axis=0)
    assert errw.max() <= gate, errw
    # the first 16 columns as a block of 16 (the tiled entry path)
    Y16 = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X[:, :16])
    d16 = np.linalg.norm(Y16 - Y[:, :16], axis=0) / np.linalg.norm(Y16, axis=0)
    assert d16.max() <= gate, d16
    g.close()
