"""GPU parity at the full workload sizes, on sampled outputs.

At these sizes the oracle cannot form the whole product, so each check takes
rows the oracle evaluates one by one (an O(n) pass per row), or properties
that hold at any size (residuals, orthonormality, spectrum bounds,
bit-identical repeats).  Gates as in the small-size parity tests: relative
error per vector, max over the block, 1e-6 for FP64-parameter NFFT and 1e-4
for FP32 NFFT; Allen--Cahn scores and labels bit-exact on the same
eigenpairs.

Workloads (seeded, synthetic; see workloads/gen.py):
  ball      n = 1e5 uniform 3-D ball, sigma 0.05, N = 64, FP64 window 14 / FP32 6
  image     1000 x 1000 image, 3 layers (RGB, pixel xy, 3x3-mean RGB)
  cube      512 x 512 pixels x 104 bands, 52 two-band layers, N in {32,64,128}
  large     n = 1e7 per layer, 3 layers d = 3, sigma 0.02, N = 128
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


def rows_rel_err(Y_rows, ref_rows):
    """Relative error of the sampled rows, per vector, max over vectors."""
    Y_rows = np.asarray(Y_rows).reshape(ref_rows.shape[0], -1)
    ref_rows = ref_rows.reshape(ref_rows.shape[0], -1)
    return float((np.linalg.norm(Y_rows - ref_rows, axis=0)
                  / np.linalg.norm(ref_rows, axis=0)).max())


def sample_rows(n, count, seed):
    return np.sort(gen.rng(seed).choice(n, size=count, replace=False))


def device_block(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


# ---------------------------------------------------------------------------
# ball: n = 1e5
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def ball():
    return gen.config2()


@pytest.mark.parametrize("prec,window,gate", [(64, 14, 1e-6), (32, 6, 1e-4)])
def test_ball_weight_rows(mlg, ball, prec, window, gate):
    pts, sig, n = ball["layers"][0], ball["sigma"][0], ball["n"]
    rows = sample_rows(n, 256, ball["base_seed"] + 400)
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", prec, N=64, window=window), degrees=False)
    for b in (1, 8, 32):
        X = gen.test_vectors(n, b, ball["base_seed"] + 300 + b)
        case_id("ball n=%d FP%d N=64 w=%d b=%d" % (n, prec, window, b))
        Y = g.laplacian_matvec(0, mlg.MLG_OP_W, X)
        ref = oracle.kernel_rows(pts, sig, X, rows)
        assert rows_rel_err(np.asarray(Y)[rows], ref) <= gate
    g.close()


def test_ball_lanczos_fp64_residuals(mlg, ball):
    """20 smallest eigenpairs of L_sym on the FP64 path: every residual
    ||L phi - lambda phi|| bounds the distance of lambda to the spectrum
    (symmetric operator), and sampled rows of L phi from the oracle confirm
    the operator the residuals were taken with."""
    pts, sig, n = ball["layers"][0], ball["sigma"][0], ball["n"]
    k = ball["k"]
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", 64, N=64, window=14))
    case_id("ball lanczos FP64 n=%d k=%d" % (n, k))
    lam, V, info = g.lanczos_eigs(0, k, block=4, tol=1e-9, seed=ball["base_seed"] + 200)
    assert info["converged"], info
    assert np.all(np.diff(lam) >= 0) and lam[0] > -1e-10 and lam[-1] < 2.0
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    LV = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, V)
    res = np.linalg.norm(LV - V * lam[None, :], axis=0)
    assert res.max() <= 1e-8, res
    # the operator itself against the oracle, on sampled rows of L V
    L = oracle.Layer(pts, sig)
    rows = sample_rows(n, 128, ball["base_seed"] + 401)
    ref = oracle.lsym_matvec([L], V, rows)
    assert np.abs(LV[rows] - ref).max() <= 1e-9 * np.abs(V).max()
    # the smallest eigenvalue of L_sym is 0 with eigenvector D^1/2 1
    phi0 = np.sqrt(L.deg) / np.linalg.norm(np.sqrt(L.deg))
    assert abs(lam[0]) <= 1e-9
    assert abs(abs(phi0 @ V[:, 0]) - 1.0) <= 1e-8
    # the 20 eigenvalues against the oracle's (stored: ARPACK on the FP64
    # direct sum, tests/golden/make_golden.py), the FP64-path gate
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "ball_n100000_eigs.json")))
    assert gold["n"] == n and gold["sigma"] == sig and gold["k"] == k
    err = np.abs(lam - np.asarray(gold["eigenvalues"])).max()
    case_id("  eigenvalue error vs oracle %.2e" % err)
    assert err <= 1e-8
    g.close()


# ---------------------------------------------------------------------------
# image: 1000 x 1000, three layers, FP32 NFFT as timed by the benchmark
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def image():
    return gen.config3()


def bench_params(mlg, T):
    return [mlg.kparams("nfft", 32, N=0, window=6, eps_B=1.0 / 16, p_reg=5) for _ in range(T)]


@pytest.fixture(scope="module")
def image_graph(mlg, image):
    c = image
    layers = [device_block(L) for L in c["layers"]]
    g = mlg.Graph(layers, c["sigma"], bench_params(mlg, len(layers)))
    yield g
    g.close()


def test_image_weight_and_degree_rows(mlg, image, image_graph):
    c, g = image, image_graph
    n, T, b = c["n"], len(c["layers"]), 16
    rows = sample_rows(n, 128, c["base_seed"] + 400)
    X = gen.test_vectors(n, b, c["base_seed"] + 300)
    for t in range(T):
        case_id("image layer %d W x n=%d b=%d" % (t, n, b))
        Y = g.laplacian_matvec(t, mlg.MLG_OP_W, X)
        ref = oracle.kernel_rows(c["layers"][t], c["sigma"][t], X, rows)
        assert rows_rel_err(np.asarray(Y)[rows], ref) <= 1e-4
        # degrees gated row by row (D^-1/2 amplifies the error of small degrees)
        dref = oracle.kernel_rows(c["layers"][t], c["sigma"][t], np.ones(n), rows)
        assert (np.abs(g.degrees(t)[rows] - dref) / dref).max() <= 1e-6


def test_image_L1_rows_against_stored_oracle(mlg, image, image_graph):
    """4096 rows of L_1 X (b = 16, the benchmark's block) of the image graph
    against stored oracle rows: tests/golden/image1000_L1_rows4096_b16.npz,
    written by tests/golden/make_golden.py from the CPU oracle alone, with
    every layer's degrees summed over all 10^6 nodes.  Also the stored
    D^-1/2 of those rows against the graph's degrees, row by row."""
    import os
    c, g = image, image_graph
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "image1000_L1_rows4096_b16.npz")
    z = np.load(path, allow_pickle=False)
    rows, ref = z["rows"], z["L1X"]
    n, T = c["n"], len(c["layers"])
    assert np.allclose(z["sigma"], c["sigma"], rtol=0, atol=0)
    X = device_block(gen.test_vectors(n, 16, c["base_seed"] + 300))
    case_id("image L_1 x against 4096 stored oracle rows n=%d b=16" % n)
    Y = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X).cpu().numpy()
    assert rows_rel_err(Y[rows], ref) <= 1e-4
    for t in range(T):
        dinv = 1.0 / np.sqrt(g.degrees(t)[rows])
        assert (np.abs(dinv - z["dinv_sqrt_rows"][:, t]) / z["dinv_sqrt_rows"][:, t]).max() <= 1e-6


def test_image_L1_repeat_bit_identical(mlg, image, image_graph):
    c, g = image, image_graph
    X = device_block(gen.test_vectors(c["n"], 16, c["base_seed"] + 301))
    case_id("image L_1 repeats n=%d b=16" % c["n"])
    Y1 = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X).cpu().numpy()
    Y2 = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X).cpu().numpy()
    assert np.array_equal(Y1, Y2)
    # L_1 = I - (1/T) sum_t N_t, each N_t from its own single-layer product
    T = len(c["layers"])
    acc = 0
    for t in range(T):
        acc = acc + g.laplacian_matvec(t, mlg.MLG_OP_NADJ, X).cpu().numpy()
    Xh = X.cpu().numpy()
    np.testing.assert_allclose(Y1, Xh - acc / T, atol=1e-12 * np.abs(Xh).max())
    # the captured product runs the layers as parallel branches; the same
    # product without the graph, layers one after another, is bit-identical
    _, Yseq = g.profile_stages(-1, mlg.MLG_OP_LSYM, X, reps=1, return_y=True)
    assert np.array_equal(Y1, Yseq.cpu().numpy())


def test_image_lanczos_and_allen_cahn(mlg, image, image_graph):
    """20 eigenpairs of L_1 (FP64 Lanczos on the FP32 operator), then the
    Allen--Cahn classifier on them, bit-exact against the oracle run on the
    same eigenpairs (a fixed number of iterations at this size)."""
    c, g = image, image_graph
    n, k = c["n"], c["k"]
    case_id("image lanczos L_1 n=%d k=%d" % (n, k))
    lam, V, info = g.lanczos_eigs(-1, k, block=4, tol=1e-5, seed=c["base_seed"] + 200)
    assert info["converged"], info
    assert np.all(np.diff(lam) >= 0) and lam[0] > -1e-4 and lam[-1] < 2.0
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    LV = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, V)
    assert np.linalg.norm(LV - V * lam[None, :], axis=0).max() <= 1e-5
    lab = gen.label_set(n, c["classes"], c["label_fraction"], c["base_seed"] + 100)
    case_id("image allen-cahn n=%d k=%d m=%d 12 iterations" % (n, k, c["m"]))
    U, pred, it = mlg.allen_cahn_ssl(lam, V, lab, c["m"], tol=0.0, max_iter=12)
    Uo, po, ito, _ = oracle.allen_cahn(lam, V, lab, c["m"], tol=0.0, max_iter=12)
    assert it == ito == 12
    assert np.array_equal(U, Uo) and np.array_equal(pred, po)


def test_image_power_inverse_rows(mlg, image, image_graph):
    """p = -1 on one layer: Y = (L_sym + delta I)^-1 X, so (L_sym + delta I) Y
    = X, checked with the layer operator the Krylov power used (that
    operator's sampled rows and degrees are checked against the oracle in
    test_image_weight_and_degree_rows; the oracle cannot form all 10^6
    degrees, which every row of L_sym Y needs)."""
    c, g = image, image_graph
    n, p = c["n"], -1.0
    delta = math.log(2.0)
    X = gen.test_vectors(n, 4, c["base_seed"] + 302)
    Xd = device_block(X)
    case_id("image (L_sym^(0) + delta I)^-1 x n=%d b=4" % n)
    Y, info = g.power_mean_matvec(0, p, Xd, tol=1e-9)
    assert info["converged"], info
    R = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, Y) + delta * Y - Xd
    R = R.cpu().numpy()
    assert (np.linalg.norm(R, axis=0) / np.linalg.norm(X, axis=0)).max() <= 1e-6


def test_image_lanczos_negative_p(mlg, image, image_graph):
    """20 smallest eigenpairs of L_{-10,delta} (three layers) through the
    Krylov power: residuals of the p-th power, order and bounds."""
    c, g = image, image_graph
    n, k, p = c["n"], c["k"], -10.0
    delta = math.log(11.0)
    case_id("image lanczos L_{-10,delta} n=%d k=%d block=16" % (n, k))
    lam, V, info = g.lanczos_eigs(-1, k, block=16, tol=1e-5, seed=c["base_seed"] + 201, p=p)
    case_id("  %s" % info)
    assert info["converged"] and info["inner_unconverged"] == 0, info
    assert np.all(np.diff(lam) >= 0) and lam[0] >= delta - 1e-9 and lam[-1] <= 2.0 + delta
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    QV, _ = g.power_mean_matvec(-1, p, device_block(V[:, :16]), tol=1e-9)
    QV = QV.cpu().numpy()
    res = np.linalg.norm(QV - V[:, :16] * lam[None, :16] ** p, axis=0) / delta ** p
    assert res.max() <= 2e-5, res


# ---------------------------------------------------------------------------
# cube: 52 two-band layers with uneven sigma and grid size
# ---------------------------------------------------------------------------
def test_cube_52_layers(mlg):
    c = gen.config4()
    n, T, b = c["n"], len(c["layers"]), 16
    # bins chosen by the plan, as in the benchmark's cube product
    kp = [mlg.kparams("nfft", 32, N=c["N"][t], window=6, bin=0) for t in range(T)]
    g = mlg.Graph([device_block(L) for L in c["layers"]], c["sigma"], kp)
    bins = [g.layer_info(t)["bin"] for t in range(T)]
    case_id("cube bins chosen: %s" % {k: bins.count(k) for k in sorted(set(bins))})
    assert set(bins) <= {1, 2, 4}
    X = gen.test_vectors(n, b, c["base_seed"] + 300)
    Xd = device_block(X)
    rows = sample_rows(n, 256, c["base_seed"] + 400)
    worst = 0.0
    for t in range(T):
        Y = g.laplacian_matvec(t, mlg.MLG_OP_W, Xd).cpu().numpy()
        ref = oracle.kernel_rows(c["layers"][t], c["sigma"][t], X, rows)
        worst = max(worst, rows_rel_err(Y[rows], ref))
    case_id("cube 52 layers n=%d b=%d worst sampled W error %.3e" % (n, b, worst))
    assert worst <= 1e-4
    # the batched mean over all layers equals the mean of the per-layer products
    Y1 = g.laplacian_matvec(-1, mlg.MLG_OP_NADJ, Xd).cpu().numpy()
    acc = 0
    for t in range(T):
        acc = acc + g.laplacian_matvec(t, mlg.MLG_OP_NADJ, Xd).cpu().numpy()
    np.testing.assert_allclose(Y1, acc / T, atol=1e-12 * np.abs(Y1).max())
    g.close()


# ---------------------------------------------------------------------------
# large: n = 1e7 points per layer
# ---------------------------------------------------------------------------
def test_large_fp32_and_fp64_rows(mlg):
    c = gen.config5()
    n, T = c["n"], len(c["layers"])
    layers = [device_block(L) for L in c["layers"]]
    rows = sample_rows(n, 256, c["base_seed"] + 400)
    b = 16
    X = gen.test_vectors(n, b, c["base_seed"] + 300)
    Xd = device_block(X)
    # bins of 1 and of 2 grid cells per side (patches of 6^3 and 7^3 cells
    # on the matrix-core kernels; the large-scale product runs with 2)
    graphs = {bn: mlg.Graph(layers, c["sigma"],
                            [mlg.kparams("nfft", 32, N=c["N"], window=6, bin=bn) for _ in range(T)],
                            degrees=False) for bn in (1, 2)}
    for t in range(T):
        ref = oracle.kernel_rows(c["layers"][t], c["sigma"][t], X, rows)
        for bn, g in graphs.items():
            case_id("large layer %d FP32 W x n=%d b=%d bin=%d" % (t, n, b, bn))
            Y = g.laplacian_matvec(t, mlg.MLG_OP_W, Xd).cpu().numpy()
            assert rows_rel_err(Y[rows], ref) <= 1e-4
    for g in graphs.values():
        g.close()
    kp64 = [mlg.kparams("nfft", 64, N=c["N"], window=12) for _ in range(T)]
    g = mlg.Graph(layers[:1], c["sigma"][:1], kp64[:1], degrees=False)
    case_id("large layer 0 FP64 W x n=%d b=1" % n)
    Y = g.laplacian_matvec(0, mlg.MLG_OP_W, Xd[:, :1].contiguous()).cpu().numpy()
    ref = oracle.kernel_rows(c["layers"][0], c["sigma"][0], X[:, :1], rows)
    assert rows_rel_err(Y[rows], ref) <= 1e-6
    g.close()


def test_large_lanczos_30_eigenpairs(mlg):
    """30 smallest eigenpairs of L_1 at n = 10^7 (three FP32 NFFT layers with
    bins of 2 cells, as the large-scale benchmark runs them; FP64 degrees,
    block Lanczos with FP64 CGS2 full reorthogonalisation): every residual
    ||L_1 phi - lambda phi|| within tol (it bounds the eigenvalue error of
    the symmetric operator), orthonormal vectors,
    eigenvalues ascending in [0, 2), and sampled rows of the operator the
    residuals were taken with against the oracle's W rows."""
    import torch
    c = gen.config5()
    n, T, k = c["n"], len(c["layers"]), c["k"]
    layers = [device_block(L) for L in c["layers"]]
    kp = [mlg.kparams("nfft", 32, N=c["N"], window=6, bin=2) for _ in range(T)]
    case_id("large graph with degrees n=%d T=%d bin=2" % (n, T))
    g = mlg.Graph(layers, c["sigma"], kp)
    tol = 1e-5
    case_id("large lanczos L_1 n=%d k=%d block=16 tol=%g" % (n, k, tol))
    lam, V, info = g.lanczos_eigs(-1, k, block=16, tol=tol, seed=c["base_seed"] + 200,
                                  device=True)
    case_id("  %s" % info)
    assert info["converged"] and info["nconv"] == k, info
    lam = lam.cpu().numpy()
    assert np.all(np.diff(lam) >= 0) and lam[0] > -1e-4 and lam[-1] < 2.0
    G = (V.t() @ V).cpu().numpy()
    np.testing.assert_allclose(G, np.eye(k), atol=1e-10)
    LV = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, V)
    res = torch.linalg.norm(LV - V * torch.from_numpy(lam).to(V.device)[None, :], dim=0)
    assert float(res.max()) <= tol * (1 + 1e-3), res
    # the W rows behind that operator, against the oracle (sampled rows)
    rows = sample_rows(n, 128, c["base_seed"] + 402)
    Vh = V[:, :4].cpu().numpy()
    for t in range(T):
        Y = g.laplacian_matvec(t, mlg.MLG_OP_W, V[:, :4].contiguous()).cpu().numpy()
        ref = oracle.kernel_rows(c["layers"][t], c["sigma"][t], Vh, rows)
        assert rows_rel_err(Y[rows], ref) <= 1e-4
    g.close()
