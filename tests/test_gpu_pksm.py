"""GPU parity of the p < 0 power mean (Sec. 2 shifted power mean; Sec. 3
polynomial Krylov method) through the C ABI.

Gates.  The Krylov power stops when its coefficient vector changes by <= tol
relative to ||x|| delta^p, delta^p = ||(L_sym + delta I)^p||; errors are
measured in the same norm, per column, max over the block:
  direct FP64 layers:   <= 1e-10 at tol 1e-12 against the exact definition
                        (dense eigendecompositions) and against the oracle's
                        own Krylov approximation;
  NFFT layers:          a matvec error e of the layer operator moves the power
                        by about |p| / delta * e, so the gate is the matvec gate
                        times max(1, |p| / delta): FP64 parameters 1e-6, FP32
                        1e-4;
  eigenvalues of L_{p,delta} on direct FP64 layers: 1e-8 absolute.
"""
import math

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


def two_layers(n, seed):
    p3, _ = gen.gaussian_mixture(n, 3, 4, 0.05, seed)
    p2 = gen.uniform_ball(n, 2, 1.0, seed + 1)
    return [p3, p2], [0.12, 0.3]


def power_err(Y, ref, X, p):
    """max over columns of ||Y - ref|| / (||x|| delta^p)."""
    delta = oracle.shift_delta(p)
    Y = np.asarray(Y).reshape(ref.shape)
    den = np.linalg.norm(X, axis=0) * delta ** p
    den = np.where(den > 0, den, 1.0)
    return float((np.linalg.norm(Y - ref, axis=0) / den).max())


@pytest.fixture(scope="module")
def direct_case(mlg):
    n = 777   # several 128-row tiles and a ragged tail
    pts, sig = two_layers(n, 501)
    g = mlg.Graph(pts, sig, [mlg.kparams("direct", 64)] * 2)
    layers = [oracle.Layer(p, s) for p, s in zip(pts, sig)]
    yield dict(n=n, g=g, layers=layers)
    g.close()


@pytest.mark.parametrize("p", [-10.0, -1.0, -0.5])
@pytest.mark.parametrize("layer", [-1, 1])
def test_power_matvec_direct_fp64(mlg, direct_case, p, layer):
    c = direct_case
    X = gen.test_vectors(c["n"], 3, 502)
    case_id("power matvec direct fp64 n=%d p=%g layer=%d b=3" % (c["n"], p, layer))
    Y, info = c["g"].power_mean_matvec(layer, p, X, tol=1e-12)
    assert info["converged"] and 4 <= info["steps"] <= 128
    sel = c["layers"] if layer < 0 else [c["layers"][layer]]
    ref = oracle.power_mean_power_matvec(sel, p, X)
    assert power_err(Y, ref, X, p) <= 1e-10
    # the oracle's own Krylov approximation, layer by layer
    acc = 0
    for L in sel:
        Ls = oracle.lsym_dense(L)
        acc = acc + np.stack([oracle.pksm_apply(Ls, p, X[:, j], tol=1e-12)[0]
                              for j in range(X.shape[1])], axis=1)
    assert power_err(Y, acc / len(sel), X, p) <= 1e-10


def test_power_matvec_special_columns(mlg, direct_case):
    """A zero column stays zero; the null vector D^1/2 1 of L_sym^(0) is
    scaled by delta^p exactly (up to rounding); columns are independent."""
    c = direct_case
    n, p = c["n"], -10.0
    delta = oracle.shift_delta(p)
    L0 = c["layers"][0]
    x_null = np.sqrt(L0.deg) / np.linalg.norm(np.sqrt(L0.deg))
    x_rand = gen.test_vectors(n, 1, 503)[:, 0]
    X = np.stack([np.zeros(n), x_null, x_rand], axis=1)
    case_id("power matvec special columns n=%d" % n)
    Y, info = c["g"].power_mean_matvec(0, p, X, tol=1e-12)
    assert info["converged"]
    assert not np.asarray(Y)[:, 0].any()
    np.testing.assert_allclose(Y[:, 1], delta ** p * x_null, rtol=0, atol=1e-12 * delta ** p)
    Y1, _ = c["g"].power_mean_matvec(0, p, x_rand[:, None], tol=1e-12)
    ref = oracle.power_mean_power_matvec([L0], p, x_rand[:, None])
    assert power_err(Y1, ref, x_rand[:, None], p) <= 1e-10
    assert power_err(Y[:, 2:], ref, x_rand[:, None], p) <= 1e-10


def test_power_matvec_repeat_bit_identical_and_step_limit(mlg, direct_case):
    c = direct_case
    X = gen.test_vectors(c["n"], 4, 504)
    case_id("power matvec repeat + step limit n=%d" % c["n"])
    Y1, i1 = c["g"].power_mean_matvec(-1, -2.0, X, tol=1e-12)
    Y2, i2 = c["g"].power_mean_matvec(-1, -2.0, X, tol=1e-12)
    assert np.array_equal(Y1, Y2) and i1 == i2
    Y3, i3 = c["g"].power_mean_matvec(-1, -0.1, X, tol=1e-15, max_steps=4)
    assert i3["steps"] == 4 and not i3["converged"] and np.isfinite(Y3).all()


def test_power_matvec_basis_growth(mlg, direct_case):
    """More than 16 Krylov steps (tolerance out of reach, limit 40): the
    basis grows past its first 16 slots with the written slots kept; the
    result is the exact power."""
    c = direct_case
    X = gen.test_vectors(c["n"], 3, 507)
    case_id("power matvec basis growth n=%d up to 40 steps" % c["n"])
    Y, info = c["g"].power_mean_matvec(-1, -0.1, X, tol=1e-15, max_steps=40)
    assert 16 < info["steps"] <= 40 and np.isfinite(Y).all()
    ref = oracle.power_mean_power_matvec(c["layers"], -0.1, X)
    assert power_err(Y, ref, X, -0.1) <= 1e-10


def test_power_matvec_arguments(mlg, direct_case):
    g = direct_case["g"]
    X = np.ones((direct_case["n"], 1))
    with pytest.raises(mlg.MlgError) as e:
        g.power_mean_matvec(-1, 0.0, X)
    assert e.value.code == mlg.MLG_ERR_ARG
    with pytest.raises(mlg.MlgError) as e:
        g.power_mean_matvec(-1, 1.0, X)
    assert e.value.code == mlg.MLG_ERR_ARG
    with pytest.raises(mlg.MlgError) as e:
        g.power_mean_matvec(-1, -1.0, X, max_steps=3)
    assert e.value.code == mlg.MLG_ERR_ARG
    with pytest.raises(mlg.MlgError) as e:
        g.lanczos_eigs(-1, 4, p=2.0)
    assert e.value.code == mlg.MLG_ERR_NOT_IMPL


def test_power_matvec_more_layers_than_lanes(mlg):
    """Four layers on three lanes: layers 0-2 run side by side, layer 3 after
    them on the first lane; the terms are added in layer order."""
    n, p = 500, -2.0
    pts = [gen.gaussian_mixture(n, 3, 3, 0.06, 520)[0], gen.uniform_ball(n, 2, 1.0, 521),
           gen.gaussian_mixture(n, 2, 4, 0.05, 522)[0], gen.uniform_ball(n, 1, 1.0, 523)]
    sig = [0.15, 0.3, 0.1, 0.2]
    g = mlg.Graph(pts, sig, [mlg.kparams("direct", 64)] * 4)
    layers = [oracle.Layer(q, s) for q, s in zip(pts, sig)]
    X = gen.test_vectors(n, 3, 524)
    case_id("power matvec 4 layers / 3 lanes n=%d p=%g" % (n, p))
    Y, info = g.power_mean_matvec(-1, p, X, tol=1e-12)
    Y2, _ = g.power_mean_matvec(-1, p, X, tol=1e-12)
    g.close()
    assert info["converged"] and np.array_equal(Y, Y2)
    assert power_err(Y, oracle.power_mean_power_matvec(layers, p, X), X, p) <= 1e-10


@pytest.mark.parametrize("prec,window,gate,b", [(64, 12, 1e-6, 4), (32, 6, 1e-4, 4),
                                                (32, 6, 1e-4, 12), (32, 6, 1e-4, 16)])
def test_power_matvec_nfft(mlg, prec, window, gate, b):
    """b = 12 and 16 take the fused next-vector/summation-input kernel with
    the FP32 slice written four columns at a time (16) or padded past b
    (12)."""
    n, p = 2500, -10.0
    pts, sig = two_layers(n, 511)
    kp = [mlg.kparams("nfft", prec, N=64, window=window)] * 2
    g = mlg.Graph(pts, sig, kp)
    layers = [oracle.Layer(q, s) for q, s in zip(pts, sig)]
    X = gen.test_vectors(n, b, 512)
    case_id("power matvec nfft fp%d n=%d p=%g b=%d" % (prec, n, p, b))
    Y, info = g.power_mean_matvec(-1, p, X, tol=1e-12)
    g.close()
    assert info["converged"]
    err = power_err(Y, oracle.power_mean_power_matvec(layers, p, X), X, p)
    case_id("  error %.3e (gate %.1e)" % (err, gate * abs(p) / oracle.shift_delta(p)))
    assert err <= gate * max(1.0, abs(p) / oracle.shift_delta(p))


@pytest.mark.parametrize("p", [-10.0, -1.0])
def test_lanczos_negative_p_direct(mlg, direct_case, p):
    """k smallest eigenpairs of L_{p,delta} (two layers) against the dense
    eigendecomposition of its p-th power."""
    c = direct_case
    k = 6
    case_id("lanczos L_{p,delta} direct fp64 n=%d p=%g k=%d" % (c["n"], p, k))
    lam, V, info = c["g"].lanczos_eigs(-1, k, block=4, tol=1e-10, seed=505, p=p)
    assert info["converged"] and info["inner_unconverged"] == 0, info
    lo, Vo = oracle.power_mean_eigs(c["layers"], p, k)
    delta = oracle.shift_delta(p)
    assert np.all(np.diff(lam) >= 0) and lam[0] >= delta - 1e-12
    np.testing.assert_allclose(lam, lo, rtol=0, atol=1e-8)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    # eigenvectors: each GPU vector lies in the oracle's eigenspace
    Q = oracle.power_mean_power_dense(c["layers"], p)
    mu = lam ** p
    res = np.linalg.norm(Q @ V - V * mu[None, :], axis=0) / delta ** p
    assert res.max() <= 1e-8, res


def test_lanczos_negative_p_single_layer(mlg, direct_case):
    """layer t >= 0: the eigenpairs of L_sym^(t) + delta I."""
    c = direct_case
    p, k = -10.0, 5
    case_id("lanczos L_sym + delta I direct fp64 n=%d k=%d" % (c["n"], k))
    lam, V, info = c["g"].lanczos_eigs(0, k, block=4, tol=1e-10, seed=506, p=p)
    assert info["converged"], info
    l1, _, _ = c["g"].lanczos_eigs(0, k, block=4, tol=1e-10, seed=506)
    np.testing.assert_allclose(lam, l1 + math.log(11.0), rtol=0, atol=1e-8)
    # residuals with the layer's own L_sym (the cluster eigenvalues are close,
    # so the vectors are compared through their eigen-equation)
    LV = c["g"].laplacian_matvec(0, mlg.MLG_OP_LSYM, V) + math.log(11.0) * V
    assert np.linalg.norm(LV - V * lam[None, :], axis=0).max() <= 1e-8
