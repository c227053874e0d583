"""GPU tests of the NFFT parameter selection (mlg_autotune_layer): the chosen
window and bandwidth meet the error budget on the full product against the
oracle (the tuner itself measures a row sample, so the full-product gate is
twice the budget), an unreachable budget is reported as MLG_ERR_RANGE with
the most accurate candidate, and host and device inputs measure the same
candidates with the same errors.
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


def rel_err(Y, ref):
    Y = np.asarray(Y).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return float((np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())


@pytest.fixture(scope="module")
def ball():
    n = 6000
    return gen.uniform_ball(n, 3, 0.25, 1002), 0.05


@pytest.mark.parametrize("prec,tol", [(32, 1e-4), (64, 1e-9)])
def test_autotune_meets_budget(mlg, ball, prec, tol):
    pts, sig = ball
    case_id("autotune fp%d tol %.0e n=%d" % (prec, tol, pts.shape[0]))
    kp, info = mlg.autotune_layer(pts, sig, precision=prec, b=8, tol=tol, nrows=256, seed=5)
    case_id("  chose N=%d w=%d bin=%d err %.2e %.3f ms (%d tried, %d within)" % (
        info["N"], info["window"], info["bin"], info["err"], info["ms"], info["tried"], info["passed"]))
    assert info["err"] <= tol and info["ms"] > 0 and 1 <= info["passed"] <= info["tried"]
    assert kp.N == info["N"] and kp.window == info["window"] and kp.bin == info["bin"]
    assert kp.precision == prec and info["bin"] in (1, 2, 4)
    X = gen.test_vectors(pts.shape[0], 4, 1003)
    Y = mlg.kernel_matvec(pts, sig, X, kp)
    assert rel_err(Y, oracle.kernel_matvec(pts, sig, X)) <= 2 * tol


@pytest.mark.parametrize("d,sig", [(1, 0.2), (2, 0.3)])
def test_autotune_low_dimensions(mlg, d, sig):
    pts = gen.uniform_ball(4000, d, 1.0, 1010 + d)
    case_id("autotune fp32 d=%d" % d)
    kp, info = mlg.autotune_layer(pts, sig, precision=32, b=4, tol=1e-4, nrows=256, seed=9)
    case_id("  chose N=%d w=%d bin=%d err %.2e" % (info["N"], info["window"], info["bin"], info["err"]))
    assert info["err"] <= 1e-4
    X = gen.test_vectors(pts.shape[0], 4, 1012)
    Y = mlg.kernel_matvec(pts, sig, X, kp)
    assert rel_err(Y, oracle.kernel_matvec(pts, sig, X)) <= 2e-4


def test_autotune_unreachable_budget(mlg, ball):
    pts, sig = ball
    case_id("autotune fp32 unreachable tol")
    with pytest.raises(mlg.MlgError) as e:
        mlg.autotune_layer(pts, sig, precision=32, b=4, tol=1e-10, nrows=64, seed=6)
    assert e.value.code == mlg.MLG_ERR_RANGE
    info = e.value.info
    assert info["tried"] >= 1 and info["passed"] == 0 and info["err"] > 1e-10 and info["ms"] < 0


def test_autotune_device_input_same_candidates(mlg, ball):
    import torch
    pts, sig = ball
    case_id("autotune host vs device input")
    kh, ih = mlg.autotune_layer(pts, sig, precision=32, b=4, tol=1e-4, nrows=128, seed=7)
    kd, idv = mlg.autotune_layer(torch.from_numpy(pts).cuda(), sig, precision=32, b=4, tol=1e-4,
                                 nrows=128, seed=7)
    # which candidates are tried and which meet the budget depends only on the
    # (deterministic) errors; the pick among those within the budget is by
    # measured time
    assert (ih["tried"], ih["passed"]) == (idv["tried"], idv["passed"])
    if (kh.N, kh.window, kh.bin) == (kd.N, kd.window, kd.bin):
        assert ih["err"] == idv["err"]
