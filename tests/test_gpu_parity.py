"""GPU parity: the HIP library through its C ABI against the CPU oracle on the
same seeded inputs.

Gates (relative error per vector, max over the block; eigenvalues absolute):
  direct FP64 1e-12, direct FP32 1e-5, NFFT with FP64 parameters 1e-6,
  NFFT FP32 1e-4, eigenvalues (FP64 path) 1e-8, Allen--Cahn scores and
  labels bit-exact on the same eigenpairs.
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


def rel_err(Y, ref):
    Y = np.asarray(Y).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return float((np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())


def case_id(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# direct summation (config 1 shape: n = 2000, 5-component GMM in R^3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("b", [1, 3, 16])
def test_direct_fp64_weight_matvec(mlg, b):
    c = gen.config1()
    pts = c["layers"][0]
    X = gen.test_vectors(c["n"], b, c["base_seed"] + 300)
    case_id("direct fp64 W x n=%d b=%d" % (c["n"], b))
    Y = mlg.kernel_matvec(pts, 0.1, X, mlg.kparams("direct", 64))
    ref = oracle.kernel_matvec(pts, 0.1, X)
    assert rel_err(Y, ref) <= 1e-12


@pytest.mark.parametrize("b", [1, 16])
def test_direct_fp32_weight_matvec(mlg, b):
    c = gen.config1()
    pts = c["layers"][0]
    X = gen.test_vectors(c["n"], b, c["base_seed"] + 301)
    case_id("direct fp32 W x n=%d b=%d" % (c["n"], b))
    Y = mlg.kernel_matvec(pts, 0.1, X, mlg.kparams("direct", 32))
    assert rel_err(Y, oracle.kernel_matvec(pts, 0.1, X)) <= 1e-5


def test_direct_lsym_and_degrees(mlg):
    c = gen.config1()
    pts = c["layers"][0]
    L = oracle.Layer(pts, 0.1)
    g = mlg.Graph([pts], [0.1], mlg.kparams("direct", 64))
    np.testing.assert_allclose(g.degrees(0), L.deg, rtol=1e-13)
    X = gen.test_vectors(c["n"], 5, c["base_seed"] + 302)
    case_id("direct fp64 L_sym x n=%d b=5" % c["n"])
    Y = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    assert rel_err(Y, oracle.lsym_matvec([L], X)) <= 1e-12
    # invariant: L_sym D^1/2 1 = 0
    v = np.sqrt(L.deg)
    r = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, v)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(v)


def test_direct_ragged_small_n(mlg):
    for n in [2, 3, 65, 257]:
        pts = gen.uniform_ball(n, 2, 1.0, 90 + n)
        X = gen.test_vectors(n, 2, 91 + n)
        case_id("direct fp64 ragged n=%d" % n)
        Y = mlg.kernel_matvec(pts, 0.8, X, mlg.kparams("direct", 64))
        np.testing.assert_allclose(Y, oracle.kernel_matvec(pts, 0.8, X), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# NFFT fast summation (config 2 shape: uniform 3-D ball, sigma = 0.05)
# ---------------------------------------------------------------------------
def ball_case(n=6000):
    pts = gen.uniform_ball(n, 3, 0.25, 1002)
    return pts, 0.05


@pytest.mark.parametrize("b", [1, 8])
def test_nfft_fp64_weight_matvec(mlg, b):
    pts, sig = ball_case()
    X = gen.test_vectors(pts.shape[0], b, 1302)
    case_id("nfft fp64 W x n=%d b=%d N=64 w=12" % (pts.shape[0], b))
    Y = mlg.kernel_matvec(pts, sig, X, mlg.kparams("nfft", 64, N=64, window=12))
    assert rel_err(Y, oracle.kernel_matvec(pts, sig, X)) <= 1e-6


@pytest.mark.parametrize("b", [1, 8, 32])
def test_nfft_fp32_weight_matvec(mlg, b):
    pts, sig = ball_case()
    X = gen.test_vectors(pts.shape[0], b, 1303)
    case_id("nfft fp32 W x n=%d b=%d N=64 w=6" % (pts.shape[0], b))
    Y = mlg.kernel_matvec(pts, sig, X, mlg.kparams("nfft", 32, N=64, window=6))
    assert rel_err(Y, oracle.kernel_matvec(pts, sig, X)) <= 1e-4


@pytest.mark.parametrize("b", [1, 5, 32])
def test_nfft_fp32_side64_grid_blocks(mlg, b):
    """FP32 d = 3 layer on a 64^3 grid (N = 32), the size whose x and y FFT
    passes run per plane, at 1, 4 and 16 complex vector pairs."""
    n = 3001
    pts, _ = gen.gaussian_mixture(n, 3, 5, 0.05, 81)
    sig = 0.4
    X = gen.test_vectors(n, b, 82)
    case_id("nfft fp32 W x d=3 n=%d b=%d N=32 w=6" % (n, b))
    Y = mlg.kernel_matvec(pts, sig, X, mlg.kparams("nfft", 32, N=32, window=6))
    assert rel_err(Y, oracle.kernel_matvec(pts, sig, X)) <= 1e-4


@pytest.mark.parametrize("bin_", [2, 4])
@pytest.mark.parametrize("prec,window,gate", [(32, 6, 1e-4), (64, 12, 1e-6)])
@pytest.mark.parametrize("d", [2, 3])
def test_nfft_bins(mlg, bin_, prec, window, gate, d):
    """Bins of 2 and 4 grid cells per side (the vector-ALU summation kernels
    in d = 3; degrees with a window whose patch fits one task)."""
    n = 3001
    pts, _ = gen.gaussian_mixture(n, d, 4, 0.08, 30 + d)
    sig = 0.3
    L = oracle.Layer(pts, sig)
    case_id("nfft fp%d L_sym d=%d bin=%d w=%d n=%d b=4" % (prec, d, bin_, window, n))
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", prec, N=64, window=window, bin=bin_))
    assert g.layer_info(0)["bin"] == bin_
    np.testing.assert_allclose(g.degrees(0), L.deg, rtol=1e-8)
    X = gen.test_vectors(n, 4, 35 + d)
    Y = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    g.close()
    assert rel_err(Y, oracle.lsym_matvec([L], X)) <= gate


@pytest.mark.parametrize("d,N,n,sig,expect", [(2, 128, 6000, 0.3, 4), (3, 64, 6000, 0.3, 2),
                                               (2, 16, 60000, 1.0, 1)])
def test_nfft_fp32_automatic_bin(mlg, d, N, n, sig, expect):
    """bin = 0: the plan doubles the bin edge while occupied bins hold fewer
    than 256 points on average, within the matrix-core patch limits (d = 3
    stops at 2: patch edge 7).  Sparse layers end at 4 (d = 2) and 2 (d = 3),
    a dense one stays at 1.  The product matches the oracle at the FP32 gate,
    is bit-identical to the explicit bin's plan and differs from bin 1 by
    FP32 rounding only."""
    pts = gen.uniform_ball(n, d, 1.0, 1301 + d)
    X = gen.test_vectors(n, 16, 1305 + d)
    L = oracle.Layer(pts, sig)
    case_id("nfft fp32 L_sym automatic bin d=%d N=%d n=%d b=16" % (d, N, n))
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", 32, N=N, window=6, bin=0))
    assert g.layer_info(0)["bin"] == expect
    Y = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    g.close()
    assert rel_err(Y, oracle.lsym_matvec([L], X)) <= 1e-4
    case_id("  explicit bin=%d and bin=1 plans" % expect)
    ge = mlg.Graph([pts], [sig], mlg.kparams("nfft", 32, N=N, window=6, bin=expect))
    Ye = ge.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    ge.close()
    assert np.array_equal(Y, Ye)
    g1 = mlg.Graph([pts], [sig], mlg.kparams("nfft", 32, N=N, window=6, bin=1))
    Y1 = g1.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    g1.close()
    assert rel_err(Y, Y1) <= 2e-6


def test_nfft_fp64_automatic_bin_is_one(mlg):
    """bin = 0 with precision 64 plans bins of one cell."""
    pts = gen.uniform_ball(3000, 2, 1.0, 1311)
    g = mlg.Graph([pts], [0.3], mlg.kparams("nfft", 64, N=128, window=12, bin=0))
    assert g.layer_info(0)["bin"] == 1
    g.close()


@pytest.mark.parametrize("b", [16, 32])
def test_nfft_fp32_bin2_matrix_core(mlg, b):
    """d = 3, bin 2, window 6: patches of 7^3 cells on the matrix-core
    kernels (three full tiles of (cx, cy) rows plus the one remaining cell).
    A dense core puts thousands of points in one bin (split tasks and their
    reductions).  Against the oracle at the FP32 gate, and against the
    vector-ALU kernels on the same plan (the first 8 vectors as a block of
    8), which differ only in FP32 rounding."""
    g = gen.rng(1201)
    n = 12007
    core = 0.004 * g.standard_normal((4000, 3))
    rest = gen.gaussian_mixture(n - 4000, 3, 4, 0.05, 1202)[0]
    pts = np.ascontiguousarray(np.vstack([core, rest]))
    X = gen.test_vectors(n, b, 1203)
    kp = mlg.kparams("nfft", 32, N=64, window=6, bin=2)
    case_id("nfft fp32 W x d=3 bin=2 w=6 (patch 7) n=%d b=%d" % (n, b))
    Y = mlg.kernel_matvec(pts, 0.3, X, kp)
    assert rel_err(Y, oracle.kernel_matvec(pts, 0.3, X)) <= 1e-4
    case_id("  same plan, block of 8 (vector-ALU kernels)")
    Y8 = mlg.kernel_matvec(pts, 0.3, X[:, :8], kp)
    assert rel_err(Y[:, :8], Y8) <= 2e-6


def test_nfft_fp32_bin2_lsym_and_batches(mlg):
    """L_sym through bin-2 (patch 7) matrix-core layers: one layer (scaled
    summation input) and four layers of d = 3, which run as one batch."""
    n = 5000
    pts = [gen.gaussian_mixture(n, 3, 3, 0.08, 1211 + t)[0] for t in range(4)]
    sig = [0.3, 0.25, 0.35, 0.28]
    kp = [mlg.kparams("nfft", 32, N=64, window=6, bin=2) for _ in range(4)]
    layers = [oracle.Layer(q, s) for q, s in zip(pts, sig)]
    X = gen.test_vectors(n, 16, 1215)
    case_id("nfft fp32 L_sym d=3 bin=2 one layer n=%d b=16" % n)
    g1 = mlg.Graph(pts[:1], sig[:1], kp[:1])
    assert g1.layer_info(0)["bin"] == 2
    Y1 = g1.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    g1.close()
    assert rel_err(Y1, oracle.lsym_matvec(layers[:1], X)) <= 1e-4
    import torch
    g = mlg.Graph(pts, sig, kp)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda")
    case_id("nfft fp32 L_sym d=3 bin=2 four layers (batched) n=%d b=16" % n)
    Y = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, Xd).cpu().numpy()
    assert rel_err(Y, oracle.lsym_matvec(layers, X)) <= 1e-4
    _, Yseq = g.profile_stages(-1, mlg.MLG_OP_LSYM, Xd, reps=1, return_y=True)
    assert np.array_equal(Y, Yseq.cpu().numpy())
    g.close()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_nfft_fp64_lsym_dims(mlg, d):
    pts, _ = gen.gaussian_mixture(3001, d, 4, 0.08, 40 + d)
    sig = 0.3       # scaled width ~0.06: Gaussian tail at N = 64 below 1e-12
    L = oracle.Layer(pts, sig)
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", 64, N=64, window=12))
    np.testing.assert_allclose(g.degrees(0), L.deg, rtol=1e-8)
    X = gen.test_vectors(3001, 4, 50 + d)
    case_id("nfft fp64 L_sym x d=%d n=3001 b=4" % d)
    Y = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    assert rel_err(Y, oracle.lsym_matvec([L], X)) <= 1e-6


@pytest.mark.parametrize("d,N,prec,window,gate", [(3, 128, 32, 6, 1e-4), (3, 128, 64, 12, 1e-6),
                                                    (2, 256, 32, 6, 1e-4), (2, 256, 64, 12, 1e-6),
                                                    (1, 256, 64, 12, 1e-6)])
def test_nfft_large_bandwidth_elementwise(mlg, d, N, prec, window, gate):
    """Bandwidths of 128 and 256 (grids of 256^3 and 512^2 cells), with a
    kernel narrow enough to need them: every row of W X and of L_sym X
    against the oracle."""
    n = 4000
    pts = gen.uniform_ball(n, d, 1.0, 70 + d)
    sig = 0.14 if N == 128 else 0.07
    X = gen.test_vectors(n, 4, 75 + d)
    case_id("nfft fp%d d=%d N=%d w=%d n=%d b=4" % (prec, d, N, window, n))
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", prec, N=N, window=window))
    assert g.layer_info(0)["N"] == N
    L = oracle.Layer(pts, sig)
    Yw = g.laplacian_matvec(0, mlg.MLG_OP_W, X)
    assert rel_err(Yw, oracle.kernel_matvec(pts, sig, X)) <= gate
    Y = g.laplacian_matvec(0, mlg.MLG_OP_LSYM, X)
    assert rel_err(Y, oracle.lsym_matvec([L], X)) <= gate
    g.close()


@pytest.mark.parametrize("d,N,prec,window,gate", [(3, 128, 32, 6, 1e-4), (3, 64, 64, 12, 1e-6),
                                                    (2, 256, 32, 6, 1e-4), (2, 128, 64, 12, 1e-6)])
def test_nfft_fused_gather_fft_b16(mlg, d, N, prec, window, gate):
    """Blocks of 16 vectors on grids of side 128..512 sum the cell table
    inside the first FFT pass: against the oracle, and against the separate
    gather (a block of 32 vectors, first 16 columns: every stage treats each
    vector the same way and the gathered sums are formed in the same order;
    the two x-transform kernels may contract multiply-adds differently, so
    the comparison is at rounding level: 1e-6 in FP32, 1e-13 in FP64)."""
    n = 4000
    pts = gen.uniform_ball(n, d, 1.0, 80 + d)
    sig = 0.14 if 2 * N == 256 else (0.07 if N == 256 else 0.28)
    X = gen.test_vectors(n, 32, 85 + d)
    case_id("nfft fused gather fp%d d=%d N=%d w=%d n=%d b=16" % (prec, d, N, window, n))
    g = mlg.Graph([pts], [sig], mlg.kparams("nfft", prec, N=N, window=window))
    Y16 = g.laplacian_matvec(0, mlg.MLG_OP_W, np.ascontiguousarray(X[:, :16]))
    assert rel_err(Y16, oracle.kernel_matvec(pts, sig, X[:, :16])) <= gate
    case_id("  same plan, block of 32 (separate gather)")
    Y32 = g.laplacian_matvec(0, mlg.MLG_OP_W, X)
    g.close()
    assert rel_err(Y16, Y32[:, :16]) <= (1e-6 if prec == 32 else 1e-13)


@pytest.mark.parametrize("b", [1, 5, 16])
def test_nfft_fp32_multilayer_mean(mlg, b):
    n = 4099
    p3, _ = gen.gaussian_mixture(n, 3, 5, 0.05, 61)
    p2 = gen.uniform_ball(n, 2, 10.0, 62)
    p1 = gen.uniform_ball(n, 1, 3.0, 63)
    sig = [0.4, 4.0, 0.8]   # scaled widths resolved by N = 32, 32, 64
    layers = [oracle.Layer(p, s) for p, s in zip([p3, p2, p1], sig)]
    kp = [mlg.kparams("nfft", 32, N=32, window=6), mlg.kparams("nfft", 32, N=32, window=6),
          mlg.kparams("nfft", 32, N=64, window=6)]
    g = mlg.Graph([p3, p2, p1], sig, kp)
    X = gen.test_vectors(n, b, 64)
    case_id("nfft fp32 L_1 x T=3 n=%d b=%d" % (n, b))
    Y = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X)
    assert rel_err(Y, oracle.lsym_matvec(layers, X)) <= 1e-4
    Y2 = g.laplacian_matvec(-1, mlg.MLG_OP_NADJ, X)
    assert rel_err(Y2, oracle.nadj_matvec(layers, X)) <= 1e-4 * (
        np.linalg.norm(X) / np.linalg.norm(oracle.nadj_matvec(layers, X)))
    # bit-identical repeats (no atomics anywhere)
    Y3 = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X)
    assert np.array_equal(Y, Y3)


def test_mixed_direct_and_nfft_layers(mlg):
    n = 1500
    p3, _ = gen.gaussian_mixture(n, 3, 3, 0.06, 71)
    p2 = gen.uniform_ball(n, 2, 1.0, 72)
    sig = [0.12, 0.5]
    layers = [oracle.Layer(p3, sig[0]), oracle.Layer(p2, sig[1])]
    g = mlg.Graph([p3, p2], sig, [mlg.kparams("direct", 64), mlg.kparams("nfft", 64, N=32, window=12)])
    X = gen.test_vectors(n, 2, 73)
    case_id("mixed direct+nfft fp64 L_1 x n=%d" % n)
    assert rel_err(g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, X), oracle.lsym_matvec(layers, X)) <= 1e-6


# ---------------------------------------------------------------------------
# Lanczos (config 1) and Allen--Cahn
# ---------------------------------------------------------------------------
def subspace_sine(A, B):
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def compare_eigvecs(lam_ref, V_ref, V, gap=1e-6, tol=1e-6):
    k = len(lam_ref)
    i = 0
    while i < k:
        j = i + 1
        while j < k and lam_ref[j] - lam_ref[j - 1] < gap:
            j += 1
        if j == k and j - i > 1:
            break  # a cluster cut by k: only its intersection is defined
        assert subspace_sine(V_ref[:, i:j], V[:, i:j]) <= tol, (i, j)
        i = j


def test_lanczos_direct_config1(mlg):
    c = gen.config1()
    pts = c["layers"][0]
    L = oracle.Layer(pts, 0.1)
    lam_ref, V_ref = oracle.eigs_dense([L], c["k"])
    g = mlg.Graph([pts], [0.1], mlg.kparams("direct", 64))
    case_id("lanczos direct fp64 n=2000 k=10 block=4")
    lam, V, info = g.lanczos_eigs(0, c["k"], block=4, tol=1e-10, seed=c["base_seed"] + 200)
    assert info["converged"], info
    np.testing.assert_allclose(lam, lam_ref, atol=1e-8)
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-12)
    compare_eigvecs(lam_ref, V_ref, V)


@pytest.mark.parametrize("n,k,block", [(30, 5, 4), (46, 8, 6)])
def test_lanczos_basis_capped_by_n(mlg, n, k, block):
    """Graphs so small that the basis rule max(4k, k + 6 block) is cut back
    to n - block columns: eigenpairs against the dense oracle."""
    pts, _ = gen.gaussian_mixture(n, 3, 3, 0.1, 1401 + n)
    L = oracle.Layer(pts, 0.3)
    lam_ref, V_ref = oracle.eigs_dense([L], k)
    g = mlg.Graph([pts], [0.3], mlg.kparams("direct", 64))
    case_id("lanczos direct fp64 n=%d k=%d block=%d (basis capped by n)" % (n, k, block))
    lam, V, info = g.lanczos_eigs(0, k, block=block, tol=1e-10, seed=1405 + n)
    g.close()
    assert info["converged"], info
    np.testing.assert_allclose(lam, lam_ref, atol=1e-8)
    compare_eigvecs(lam_ref, V_ref, V)


def test_lanczos_nfft_fp64_multilayer(mlg):
    n = 2500
    p3, _ = gen.gaussian_mixture(n, 3, 4, 0.05, 81)
    p2 = gen.uniform_ball(n, 2, 1.0, 82)
    sig = [0.3, 0.35]
    layers = [oracle.Layer(p3, sig[0]), oracle.Layer(p2, sig[1])]
    lam_ref, V_ref = oracle.eigs_dense(layers, 8)
    kp = mlg.kparams("nfft", 64, N=64, window=12)
    g = mlg.Graph([p3, p2], sig, [kp, kp])
    case_id("lanczos nfft fp64 L_1 n=%d k=8" % n)
    lam, V, info = g.lanczos_eigs(-1, 8, block=4, tol=1e-9, seed=7)
    assert info["converged"], info
    np.testing.assert_allclose(lam, lam_ref, atol=1e-8)


def test_allen_cahn_bit_exact(mlg):
    c = gen.config1()
    pts = c["layers"][0]
    L = oracle.Layer(pts, 0.1)
    lam, V = oracle.eigs_dense([L], c["k"])
    lab = gen.label_set(c["n"], c["classes"], c["label_fraction"], c["base_seed"] + 100)
    Uo, po, ito, margin = oracle.allen_cahn(lam, V, lab, c["m"], tol=0.0, max_iter=300)
    case_id("allen-cahn n=2000 k=10 m=5 300 iterations")
    U, pred, it = mlg.allen_cahn_ssl(lam, V, lab, c["m"], tol=0.0, max_iter=300)
    assert it == ito == 300
    assert np.array_equal(U, Uo)
    assert np.array_equal(pred, po)
    # with the tolerance: same stopping iteration
    Uo2, po2, ito2, _ = oracle.allen_cahn(lam, V, lab, c["m"], tol=1e-6, max_iter=300)
    U2, p2, it2 = mlg.allen_cahn_ssl(lam, V, lab, c["m"], tol=1e-6, max_iter=300)
    assert it2 == ito2 and np.array_equal(U2, Uo2) and np.array_equal(p2, po2)


@pytest.mark.parametrize("n,k,m", [(40_001, 120, 10), (20_003, 30, 16), (9_001, 12, 17),
                                   (5_003, 300, 4), (3_001, 7, 2), (3_001, 250, 16),
                                   (250, 5, 3)])
def test_allen_cahn_bit_exact_shapes(mlg, n, k, m):
    """The fused step (m <= 16, its LDS within 64 KiB; k > 256 too) and the
    general kernels (m > 16, or k = 250 with m = 16), ragged last chunk of
    256 rows, a single chunk: scores and labels bit-exact against the oracle
    after 20 iterations.  Any orthonormal basis serves as the eigenvector
    block of the scheme."""
    g = gen.rng(1000 + n)
    Phi, _ = np.linalg.qr(g.standard_normal((n, k)))
    lam = np.sort(g.uniform(0.0, 1.5, k))
    lab = gen.label_set(n, g.integers(0, m, n).astype(np.int32), 0.01, 2000 + n)
    case_id("allen-cahn shapes n=%d k=%d m=%d 20 iterations" % (n, k, m))
    U, pred, it = mlg.allen_cahn_ssl(lam, Phi, lab, m, tol=0.0, max_iter=20)
    Uo, po, ito, _ = oracle.allen_cahn(lam, Phi, lab, m, tol=0.0, max_iter=20)
    assert it == ito == 20
    assert np.array_equal(U, Uo) and np.array_equal(pred, po)


def test_allen_cahn_on_gpu_eigenpairs_end_to_end(mlg):
    c = gen.config1()
    pts = c["layers"][0]
    g = mlg.Graph([pts], [0.1], mlg.kparams("direct", 64))
    lam, V, info = g.lanczos_eigs(0, c["k"], block=4, tol=1e-10, seed=c["base_seed"] + 200)
    lab = gen.label_set(c["n"], c["classes"], c["label_fraction"], c["base_seed"] + 100)
    Uo, po, ito, _ = oracle.allen_cahn(lam, V, lab, c["m"], tol=0.0, max_iter=300)
    case_id("allen-cahn on GPU eigenpairs n=2000")
    U, pred, it = mlg.allen_cahn_ssl(lam, V, lab, c["m"], tol=0.0, max_iter=300)
    assert np.array_equal(pred, po) and np.array_equal(U, Uo)
    assert (pred == c["classes"]).mean() > 0.95


def test_nfft_fp32_heavy_bin_two_level_reduction(mlg):
    """A bin holding > 32 tasks of points exercises both reduction levels."""
    g = gen.rng(97)
    n = 24007
    core = 0.0005 * g.standard_normal((18000, 3))       # one very dense cell
    rest = gen.uniform_ball(n - 18000, 3, 1.0, 98)
    pts = np.ascontiguousarray(np.vstack([core, rest]))
    X = gen.test_vectors(n, 16, 99)
    case_id("nfft fp32 heavy bin n=%d b=16" % n)
    Y = mlg.kernel_matvec(pts, 0.3, X, mlg.kparams("nfft", 32, N=64, window=6))
    assert rel_err(Y, oracle.kernel_matvec(pts, 0.3, X)) <= 1e-4
    Y64 = mlg.kernel_matvec(pts, 0.3, X[:, :2], mlg.kparams("nfft", 64, N=64, window=12))
    assert rel_err(Y64, oracle.kernel_matvec(pts, 0.3, X[:, :2])) <= 1e-6


# ---------------------------------------------------------------------------
# the whole product (entry, layer summations, exit) as one captured graph
# whose entry and exit nodes are re-pointed when X or Y change
# ---------------------------------------------------------------------------
def test_whole_product_graph_replays(mlg):
    """Products on alternating X and Y buffers enqueued back to back with
    MLG_ASYNC (each call re-points the graph's entry and exit nodes while
    earlier launches are still queued), then eager work, three times over;
    and the same sequence waiting for each product: every result equal bit
    for bit to the product computed without the graph (layers one after
    another)."""
    import torch
    n, b = 5000, 16
    p3a = gen.gaussian_mixture(n, 3, 3, 0.08, 1231)[0]
    p2 = gen.uniform_ball(n, 2, 1.0, 1232)
    p3b = gen.gaussian_mixture(n, 3, 4, 0.06, 1233)[0]
    pts, sig = [p3a, p2, p3b], [0.3, 0.35, 0.25]
    g = mlg.Graph(pts, sig, [mlg.kparams("nfft", 32, N=32, window=6) for _ in pts])
    Xs = [torch.from_numpy(np.ascontiguousarray(gen.test_vectors(n, b, 1240 + i))).to("cuda")
          for i in range(3)]
    refs = [g.profile_stages(-1, mlg.MLG_OP_LSYM, X, reps=1, return_y=True)[1].cpu().numpy()
            for X in Xs]
    Xc = [X.t().contiguous() for X in Xs]
    plan = [(0, 0), (1, 1), (2, 2), (0, 3), (2, 0)]   # (input, output buffer)
    for rnd in range(4):
        Yc = [torch.full((b, n), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4)]
        torch.cuda.synchronize()
        wait = rnd == 3
        case_id("whole-product graph, round %d: %d products, wait=%s" % (rnd, len(plan), wait))
        for xi, yi in plan:
            g.laplacian_matvec_into(-1, mlg.MLG_OP_LSYM, Xc[xi], Yc[yi], sync=False, wait=wait)
        g.synchronize()
        torch.cuda.synchronize()
        # buffer 0 was written twice (inputs 0, then 2): it holds the last
        assert np.array_equal(Yc[0].t().cpu().numpy(), refs[2])
        assert np.array_equal(Yc[1].t().cpu().numpy(), refs[1])
        assert np.array_equal(Yc[2].t().cpu().numpy(), refs[2])
        assert np.array_equal(Yc[3].t().cpu().numpy(), refs[0])
        # eager work between the rounds: a one-layer product and a torch op
        g.laplacian_matvec(0, mlg.MLG_OP_W, Xs[1][:, :4].contiguous())
        Xs[1].mul_(1.0)
        torch.cuda.synchronize()
    g.close()


# ---------------------------------------------------------------------------
# batched layers: more FP32 matrix-core layers of one dimension and patch
# edge than branches run as one launch per stage (uneven N grouped for the
# FFT)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("b", [16, 32])
def test_batched_layers_against_oracle_and_per_layer_path(mlg, b):
    n = 5000
    p2 = [gen.uniform_ball(n, 2, 1.0, 961 + t) for t in range(4)]
    p3 = [gen.gaussian_mixture(n, 3, 3, 0.08, 971 + t)[0] for t in range(4)]
    pts = p2[:2] + p3[:2] + p2[2:] + p3[2:]
    sig = [0.35, 0.5, 0.2, 0.22, 0.45, 0.3, 0.25, 0.18]
    Ns = [32, 64, 32, 64, 128, 32, 32, 32]
    kp = [mlg.kparams("nfft", 32, N=N, window=6) for N in Ns]
    g = mlg.Graph(pts, sig, kp)
    import torch
    X = gen.test_vectors(n, b, 981)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda")
    case_id("batched layers n=%d T=8 (d=2 x4, d=3 x4) b=%d" % (n, b))
    Y = g.laplacian_matvec(-1, mlg.MLG_OP_LSYM, Xd).cpu().numpy()
    ref = oracle.lsym_matvec([oracle.Layer(q, s) for q, s in zip(pts, sig)], X)
    assert rel_err(Y, ref) <= 1e-4
    # the stage-profiled product walks the layers one by one without batches:
    # the same bits
    _, Yseq = g.profile_stages(-1, mlg.MLG_OP_LSYM, Xd, reps=1, return_y=True)
    assert np.array_equal(Y, Yseq.cpu().numpy())
    # and the layer mean equals the mean of the one-layer products
    acc = 0
    for t in range(len(pts)):
        acc = acc + g.laplacian_matvec(t, mlg.MLG_OP_NADJ, Xd).cpu().numpy()
    Y1 = g.laplacian_matvec(-1, mlg.MLG_OP_NADJ, Xd).cpu().numpy()
    np.testing.assert_allclose(Y1, acc / len(pts), atol=1e-12 * np.abs(Y1).max())
    g.close()
