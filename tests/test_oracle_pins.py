"""Pins of the CPU oracle against things other than itself: brute force,
closed forms, invariants of the graph Laplacian, and independent
re-derivations (finite differences, a different simplex-projection algorithm,
the dense implicit step of the scheme).  None of these call the GPU library.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads import gen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


# ---------------------------------------------------------------------------
# weight matrix (Sec. 2, Sec. 4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [1, 2, 3])
def test_kernel_matvec_brute_force(d):
    g = gen.rng(7 + d)
    n = 13
    pts = g.uniform(-1, 1, size=(n, d))
    sigma = 0.7
    x = g.standard_normal(n)
    y = oracle.kernel_matvec(pts, sigma, x)
    for i in range(n):
        terms = []
        for j in range(n):
            if j == i:
                continue
            r2 = math.fsum((pts[i, k] - pts[j, k]) ** 2 for k in range(d))
            terms.append(math.exp(-r2 / sigma ** 2) * x[j])
        ref = math.fsum(terms)
        assert abs(y[i] - ref) <= 1e-15 * math.fsum(abs(t) for t in terms) + 1e-300


def test_weight_matrix_is_bitwise_symmetric_and_zero_diagonal():
    pts, _ = gen.gaussian_mixture(40, 3, 3, 0.2, 5)
    W = oracle.kernel_matvec(pts, 0.3, np.eye(40))
    assert np.all(np.diag(W) == 0.0)
    assert np.array_equal(W, W.T)


def test_sampled_rows_equal_full_rows():
    pts, _ = gen.gaussian_mixture(300, 2, 3, 0.1, 6)
    X = gen.test_vectors(300, 3, 11)
    full = oracle.kernel_matvec(pts, 0.2, X)
    rows = np.array([0, 17, 299, 150, 17])
    part = oracle.kernel_rows(pts, 0.2, X, rows)
    assert np.array_equal(part, full[rows])


def test_kernel_matvec_matches_dense_numpy():
    pts, _ = gen.gaussian_mixture(200, 3, 4, 0.1, 9)
    X = gen.test_vectors(200, 4, 12)
    W = oracle.dense_weight(pts, 0.15)
    np.testing.assert_allclose(oracle.kernel_matvec(pts, 0.15, X), W @ X, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Laplacians and their spectra (Sec. 2, Sec. 3)
# ---------------------------------------------------------------------------
def test_two_nodes_spectrum():
    L = oracle.Layer(np.array([[0.0], [0.3]]), 0.5)
    lam, _ = oracle.eigs_dense([L], 2)
    np.testing.assert_allclose(lam, [0.0, 2.0], atol=1e-14)


def test_equilateral_triangle_spectrum():
    p = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3) / 2]])
    L = oracle.Layer(p, 1.3)
    lam, _ = oracle.eigs_dense([L], 3)
    np.testing.assert_allclose(lam, [0.0, 1.5, 1.5], atol=1e-13)


def circle_closed_form(n, R, sigma):
    """W is circulant for equally spaced points on a circle; its normalised
    adjacency has eigenvalues sum_j w_j cos(2 pi k j / n) / sum_j w_j."""
    j = np.arange(1, n)
    w = np.exp(-(2 * R * np.sin(np.pi * j / n)) ** 2 / sigma ** 2)
    k = np.arange(n)
    mu = (w[None, :] * np.cos(2 * np.pi * np.outer(k, j) / n)).sum(1) / w.sum()
    return np.sort(1.0 - mu)


def test_circle_graph_dense_closed_form():
    n, R, s = 64, 1.0, 0.6
    L = oracle.Layer(gen.circle_points(n, R), s)
    lam, _ = oracle.eigs_dense([L], n)
    np.testing.assert_allclose(lam, circle_closed_form(n, R, s), atol=1e-13)


@pytest.mark.slow
def test_circle_graph_iterative_closed_form():
    n, R, s = 1500, 1.0, 0.05
    L = oracle.Layer(gen.circle_points(n, R, d=3, phase=0.25), s)
    lam, V = oracle.eigs_iterative([L], 8, tol=1e-13)
    np.testing.assert_allclose(lam, circle_closed_form(n, R, s)[:8], atol=1e-10)


def test_lsym_annihilates_sqrt_degree_vector():
    pts, _ = gen.gaussian_mixture(250, 3, 3, 0.1, 21)
    L = oracle.Layer(pts, 0.2)
    v = np.sqrt(L.deg)
    r = oracle.lsym_matvec([L], v)
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(v)


def test_spectrum_range_and_trace():
    pts, _ = gen.gaussian_mixture(150, 2, 3, 0.1, 22)
    L = oracle.Layer(pts, 0.15)
    A = oracle.dense_nadj([L])
    Ls = np.eye(150) - A
    assert abs(np.trace(Ls) - 150) < 1e-10
    ev = np.linalg.eigvalsh(Ls)
    assert ev.min() > -1e-12 and ev.max() < 2 + 1e-12


def test_layer_mean_matches_dense_and_identical_layers():
    pts1, _ = gen.gaussian_mixture(120, 3, 3, 0.1, 31)
    pts2 = gen.uniform_ball(120, 2, 1.0, 32)
    La, Lb = oracle.Layer(pts1, 0.2), oracle.Layer(pts2, 0.5)
    X = gen.test_vectors(120, 2, 33)
    np.testing.assert_allclose(oracle.nadj_matvec([La, Lb], X), oracle.dense_nadj([La, Lb]) @ X,
                               rtol=1e-12, atol=1e-13)
    # T identical layers give the operator of one layer
    np.testing.assert_allclose(oracle.nadj_matvec([La, La, La], X), oracle.nadj_matvec([La], X),
                               rtol=1e-14, atol=1e-15)


def test_power_mean_single_layer_is_that_layer():
    pts, _ = gen.gaussian_mixture(60, 2, 2, 0.2, 41)
    L = oracle.Layer(pts, 0.3)
    Ls = np.eye(60) - oracle.dense_nadj([L])
    np.testing.assert_allclose(oracle.power_mean_dense([L], 1.0), Ls, atol=1e-12)
    delta = math.log(1 + 2.0)
    np.testing.assert_allclose(oracle.power_mean_dense([L], -2.0), Ls + delta * np.eye(60), atol=1e-10)


def two_small_layers(n=90, seed=61):
    pts1, _ = gen.gaussian_mixture(n, 2, 3, 0.15, seed)
    pts2 = gen.uniform_ball(n, 3, 1.0, seed + 1)
    return oracle.Layer(pts1, 0.3), oracle.Layer(pts2, 0.6)


def test_power_mean_power_negative_integer_p_is_inverse():
    """p = -1 and p = -2: the matrix power is the inverse (LAPACK solve, no
    eigendecomposition), Sec. 2 shifted power mean with delta = log(1+|p|)."""
    La, Lb = two_small_layers()
    X = gen.test_vectors(90, 3, 62)
    I = np.eye(90)
    for p in (-1.0, -2.0):
        delta = math.log(1 + abs(p))
        ref = 0
        for L in (La, Lb):
            A = oracle.lsym_dense(L) + delta * I
            Y = np.linalg.solve(A, X)
            if p == -2.0:
                Y = np.linalg.solve(A, Y)
            ref = ref + Y
        ref = ref / 2
        np.testing.assert_allclose(oracle.power_mean_power_matvec([La, Lb], p, X), ref,
                                   rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_power_mean_power_fractional_p_matches_sqrtm():
    """p = -1/2: (A)^(-1/2) = sqrtm(A)^-1 with scipy's Schur-based sqrtm."""
    import scipy.linalg
    La, _ = two_small_layers()
    p = -0.5
    A = oracle.lsym_dense(La) + math.log(1.5) * np.eye(90)
    ref = np.linalg.inv(np.real(scipy.linalg.sqrtm(A)))
    np.testing.assert_allclose(oracle.power_mean_power_dense([La], p), ref, atol=1e-11)


def test_power_mean_eigs_against_inverse_operator():
    """Two layers, p = -1: eigenpairs of L_{-1,delta} are mu^-1 of the mean of
    inverses (formed with solve), order reversed (Sec. 3)."""
    La, Lb = two_small_layers()
    delta = math.log(2.0)
    I = np.eye(90)
    Q = 0.5 * (np.linalg.solve(oracle.lsym_dense(La) + delta * I, I)
               + np.linalg.solve(oracle.lsym_dense(Lb) + delta * I, I))
    Q = 0.5 * (Q + Q.T)
    mu = np.sort(np.linalg.eigvalsh(Q))[::-1][:6]
    lam, V = oracle.power_mean_eigs([La, Lb], -1.0, 6)
    np.testing.assert_allclose(lam, 1.0 / mu, rtol=1e-11)
    assert np.all(np.diff(lam) >= 0) and lam[0] >= delta - 1e-12
    # eigenvectors of L_{-1,delta} itself
    Lp = oracle.power_mean_dense([La, Lb], -1.0)
    np.testing.assert_allclose(Lp @ V, V * lam[None, :], atol=1e-10)
    # one layer: L_sym + delta I, same vectors as the p = 1 eigensolver
    lam1, V1 = oracle.power_mean_eigs([La], -10.0, 5)
    l0, V0 = oracle.eigs_dense([La], 5)
    np.testing.assert_allclose(lam1, l0 + math.log(11.0), atol=1e-9)
    np.testing.assert_allclose(np.abs(V1.T @ V0), np.eye(5), atol=1e-6)


@pytest.mark.parametrize("p", [-10.0, -1.0, -0.3])
def test_pksm_converges_to_matrix_power(p):
    """The Lanczos approximation reaches (L_sym + delta I)^p x within the
    stopping tolerance (relative to ||x|| ||f(L)||, ||f(L)|| <= delta^p)."""
    La, _ = two_small_layers(160, 71)
    Ls = oracle.lsym_dense(La)
    x = gen.test_vectors(160, 1, 72)[:, 0]
    ref = oracle.power_mean_power_matvec([La], p, x)
    y, steps, conv = oracle.pksm_apply(Ls, p, x, tol=1e-12)
    delta = oracle.shift_delta(p)
    assert conv and steps < 80
    assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(x) * delta ** p
    # operator given as a function
    y2, steps2, _ = oracle.pksm_apply(lambda v: Ls @ v, p, x, tol=1e-12)
    assert steps2 == steps and np.array_equal(y, y2)


def test_pksm_special_inputs():
    La, _ = two_small_layers(120, 81)
    Ls = oracle.lsym_dense(La)
    p = -10.0
    delta = oracle.shift_delta(p)
    # zero vector
    y, steps, conv = oracle.pksm_apply(Ls, p, np.zeros(120))
    assert conv and steps == 0 and not y.any()
    # the null vector D^1/2 1 of L_sym: f(L) x = delta^p x
    x = np.sqrt(La.deg)
    y, steps, conv = oracle.pksm_apply(Ls, p, x)
    np.testing.assert_allclose(y, delta ** p * x, rtol=1e-12)
    # an exact invariant subspace of dimension 2: beta_2 = 0, v_3 = 0
    lam, V = np.linalg.eigh(Ls)
    x = V[:, 5] + 2 * V[:, 40]
    y, steps, conv = oracle.pksm_apply(Ls, p, x)
    ref = (lam[5] + delta) ** p * V[:, 5] + 2 * (lam[40] + delta) ** p * V[:, 40]
    assert conv
    np.testing.assert_allclose(y, ref, atol=1e-12 * np.abs(ref).max())
    # the step limit: no convergence at 4 steps with a tight tolerance
    x = gen.test_vectors(120, 1, 82)[:, 0]
    y, steps, conv = oracle.pksm_apply(Ls, -0.1, x, tol=1e-15, max_steps=4)
    assert steps == 4 and not conv


@pytest.mark.parametrize("d", [1, 2, 3])
def test_laplacian_kernel_brute_force(d):
    """Laplacian RBF exp(-||y||/sigma) (Sec. 4) against math.fsum."""
    g = gen.rng(17 + d)
    n = 11
    pts = g.uniform(-1, 1, size=(n, d))
    sigma = 0.6
    x = g.standard_normal(n)
    y = oracle.kernel_matvec(pts, sigma, x, kernel="laplacian")
    for i in range(n):
        terms = [math.exp(-math.sqrt(sum((pts[i, k] - pts[j, k]) ** 2 for k in range(d))) / sigma)
                 * x[j] for j in range(n) if j != i]
        assert abs(y[i] - math.fsum(terms)) <= 1e-15 * max(1.0, abs(math.fsum(terms)))


def test_laplacian_kernel_degrees_geometric_series():
    """Nodes 0, 1, ..., n-1 on a line: deg_i = sum_{j != i} q^|i-j|,
    q = exp(-1/sigma), a sum of two geometric series."""
    n, sigma = 40, 3.0
    pts = np.arange(n, dtype=np.float64)[:, None]
    q = math.exp(-1.0 / sigma)
    ref = np.array([q * (1 - q ** i) / (1 - q) + q * (1 - q ** (n - 1 - i)) / (1 - q)
                    for i in range(n)])
    np.testing.assert_allclose(oracle.degrees(pts, sigma, "laplacian"), ref, rtol=1e-14)
    L = oracle.Layer(pts, sigma, "laplacian")
    Ls = np.eye(n) - oracle.dense_nadj([L])
    # L_sym D^1/2 1 = 0 for any kernel
    assert np.abs(Ls @ np.sqrt(L.deg)).max() <= 1e-13


def test_median_pairwise_distance_by_hand():
    pts = np.array([[0.0, 0.0], [3.0, 4.0], [0.0, 1.0], [6.0, 8.0]])
    # pairs of rows 0, 1, 2: distances 5, 1, sqrt(9 + 9) -> median sqrt(18) (odd count)
    assert oracle.median_pairwise_distance(pts, [0, 1, 2]) == math.sqrt(18.0)
    # rows 0, 1, 3: 5, 10, 5 -> 5; all four rows: 5, 1, 10, sqrt(18), 5, sqrt(36 + 49) -> even
    assert oracle.median_pairwise_distance(pts, [0, 1, 3]) == 5.0
    d = sorted([5.0, 1.0, 10.0, math.sqrt(18.0), 5.0, math.sqrt(85.0)])
    assert oracle.median_pairwise_distance(pts, [0, 1, 2, 3]) == 0.5 * (d[2] + d[3])
    # a column subset
    assert oracle.median_pairwise_distance(pts, [0, 1, 3], cols=[1]) == 4.0


def test_eigs_well_separated_clusters_count():
    pts, _ = gen.gaussian_mixture(200, 2, 4, 0.01, 51, mean_low=0, mean_high=10)
    L = oracle.Layer(pts, 0.05)
    lam, _ = oracle.eigs_dense([L], 6)
    assert np.all(np.abs(lam[:4]) < 1e-10) and lam[4] > 0.1


def test_eigs_iterative_matches_dense():
    c = gen.config1(400)
    L = oracle.Layer(c["layers"][0], 0.1)
    l1, V1 = oracle.eigs_dense([L], 6)
    l2, V2 = oracle.eigs_iterative([L], 6, tol=1e-14)
    np.testing.assert_allclose(l1, l2, atol=1e-10)


def test_isolated_node_detected():
    p = np.array([[0.0, 0.0], [0.01, 0.0], [100.0, 100.0]])
    with pytest.raises(ValueError):
        oracle.Layer(p, 0.1)


# ---------------------------------------------------------------------------
# Allen--Cahn pieces (Sec. 5, Sec. 6, Appendix B)
# ---------------------------------------------------------------------------
def psi(u):
    m = len(u)
    out = 1.0
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1
        out *= 0.25 * np.abs(u - e).sum() ** 2
    return out


@pytest.mark.parametrize("m", [2, 3, 5, 8])
def test_potential_grad_vs_finite_differences(m):
    g = gen.rng(60 + m)
    for _ in range(5):
        u = g.uniform(0.05, 0.95, size=m)
        T = oracle.potential_grad(u)
        h = 1e-6
        fd = np.array([(psi(u + h * np.eye(m)[j]) - psi(u - h * np.eye(m)[j])) / (2 * h)
                       for j in range(m)])
        np.testing.assert_allclose(T, fd, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("m", [2, 4, 7])
def test_potential_grad_vanishes_at_corners(m):
    for q in range(m):
        assert np.all(oracle.potential_grad(np.eye(m)[q]) == 0.0)


def bisection_projection(y):
    """Simplex projection by bisection on the threshold tau with
    sum max(y - tau, 0) = 1 (a different algorithm from Chen & Ye's)."""
    lo, hi = y.min() - 1.0, y.max()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.maximum(y - mid, 0).sum() > 1.0:
            lo = mid
        else:
            hi = mid
    return np.maximum(y - 0.5 * (lo + hi), 0)


@pytest.mark.parametrize("m", [2, 3, 5, 10])
def test_simplex_projection(m):
    g = gen.rng(70 + m)
    for _ in range(50):
        y = g.standard_normal(m) * g.choice([0.1, 1, 10])
        x = oracle.simplex_project(y)
        assert np.all(x >= 0) and abs(x.sum() - 1) < 1e-14
        np.testing.assert_allclose(x, bisection_projection(y), atol=1e-13)
        np.testing.assert_allclose(oracle.simplex_project(x), x, atol=1e-15)
    s = g.dirichlet(np.ones(m))
    np.testing.assert_allclose(oracle.simplex_project(s), s, atol=1e-15)


def dense_scheme(Ls, labels, m, eps, omega0, c, dt, iters):
    """Implicit step of Sec. 5 with a dense solve of B = (1+c dt) I + eps dt L,
    then projection: the scheme before the eigenbasis is introduced."""
    n = Ls.shape[0]
    F = np.zeros((n, m))
    om = np.zeros(n)
    U = np.full((n, m), 1.0 / m)
    for i, l in enumerate(labels):
        if l >= 0:
            F[i, l] = 1
            om[i] = omega0
            U[i] = F[i]
    B = (1 + c * dt) * np.eye(n) + eps * dt * Ls
    for _ in range(iters):
        A = np.abs(U[:, None, :] - np.eye(m)[None, :, :]).sum(-1)      # a_iq
        S = 0.25 * A ** 2
        T = np.zeros((n, m))
        for q in range(m):
            prod = np.prod(np.delete(S, q, axis=1), axis=1)
            sgn = np.ones(m)
            sgn[q] = -1
            T += 0.5 * (A[:, q] * prod)[:, None] * sgn[None, :]
        R = (1 + c * dt) * U - dt / (2 * eps) * T - dt * om[:, None] * (U - F)
        Ut = np.linalg.solve(B, R)
        U = np.array([bisection_projection(r) for r in Ut])
    return U


def test_allen_cahn_full_basis_equals_dense_scheme():
    c = gen.config1(120)
    L = oracle.Layer(c["layers"][0], 0.1)
    lam, V = oracle.eigs_dense([L], 120)
    lab = gen.label_set(120, c["classes"], 0.1, 5)
    P = GOLD["allen_cahn_small_multilayer"]
    eps, om0, dt = P["eps"], P["omega0"], P["dt"]
    cc = om0 + P["c_minus_omega0_times_eps"] / eps
    U, pred, it, _ = oracle.allen_cahn(lam, V, lab, 5, eps=eps, omega0=om0, c=cc, dt=dt,
                                       tol=0.0, max_iter=6)
    assert it == 6
    Ls = np.eye(120) - oracle.dense_nadj([L])
    Ud = dense_scheme(Ls, lab, 5, eps, om0, cc, dt, 6)
    np.testing.assert_allclose(U, Ud, atol=1e-9)


def test_allen_cahn_all_labelled_reproduces_labels():
    c = gen.config1(300)
    L = oracle.Layer(c["layers"][0], 0.1)
    lam, V = oracle.eigs_dense([L], 40)
    U, pred, it, _ = oracle.allen_cahn(lam, V, c["classes"], 5, omega0=1e4, c=1e4 + 3 / 5e-3,
                                       tol=0.0, max_iter=50)
    assert np.array_equal(pred, c["classes"])


def test_allen_cahn_iteration_count_semantics():
    c = gen.config1(200)
    L = oracle.Layer(c["layers"][0], 0.1)
    lam, V = oracle.eigs_dense([L], 8)
    lab = gen.label_set(200, c["classes"], 0.05, 3)
    _, _, it, _ = oracle.allen_cahn(lam, V, lab, 5, tol=0.0, max_iter=17)
    assert it == 17
    _, _, it, _ = oracle.allen_cahn(lam, V, lab, 5, tol=1e300, max_iter=17)
    assert it == 1            # the loop body always runs once (do ... while)
    U, _, _, _ = oracle.allen_cahn(lam, V, lab, 5, tol=0.0, max_iter=5)
    assert np.all(U >= 0) and np.allclose(U.sum(1), 1.0, atol=1e-14)


def test_allen_cahn_is_deterministic():
    c = gen.config1(200)
    L = oracle.Layer(c["layers"][0], 0.1)
    lam, V = oracle.eigs_dense([L], 8)
    lab = gen.label_set(200, c["classes"], 0.05, 3)
    a = oracle.allen_cahn(lam, V, lab, 5, tol=0.0, max_iter=20)
    b = oracle.allen_cahn(lam, V, lab, 5, tol=0.0, max_iter=20)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_stored_image_rows_match_their_recipe():
    """The stored oracle rows of the image graph (written by
    tests/golden/make_golden.py from the oracle) belong to the seeded sample
    and kernel widths the recipe gives: sorted distinct rows from the row
    seed, 16 vectors, the three layers' sigma, finite values, and positive
    D^-1/2."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    z = np.load(os.path.join(here, "image1000_L1_rows4096_b16.npz"), allow_pickle=False)
    base = gen.SEED_BASE + 3
    n = 1000 * 1000
    assert np.array_equal(z["rows"], mg.image_sample(n, base))
    assert z["L1X"].shape == (mg.IMAGE_ROWS, mg.IMAGE_B) and np.isfinite(z["L1X"]).all()
    assert np.all(z["dinv_sqrt_rows"] > 0)
    # sigma of each layer by the workload rule (1000 seeded samples)
    img, _ = gen.synthetic_image(1000, 1000, base)
    assert z["sigma"][0] == gen.median_pairwise_distance(np.ascontiguousarray(img.reshape(n, 3)), 1000,
                                                         base + 10)


# ---------------------------------------------------------------------------
# Why the Laplacian RBF kernel stays on the direct path: the truncated Fourier
# series of Algorithm 1 (Sec. 4) converges algebraically for its cusp
# ---------------------------------------------------------------------------
def _truncation_error(kind, s, N, n=600, seed=5):
    """Relative error of W x when K is replaced by its truncated Fourier
    series K_RF (bandwidth N, coefficients from N^3 samples of the
    regularised kernel: two-point Taylor on (1/2 - eps_B, 1/2), eps_B = 1/16,
    5 matched derivatives).  Points sit on the 2N lattice inside the scaled
    ball (radius 1/4 - eps_B/2), so every pair difference is a lattice vector
    and K_RF there is read off one inverse FFT exactly."""
    import math
    epsB, p = 1.0 / 16, 5
    r0 = 0.5 - epsB
    if kind == "gauss":
        K = lambda r: np.exp(-r * r / (s * s))
        u = r0 / s
        H = [1.0, 2 * u]
        for j in range(1, p):
            H.append(2 * u * H[j] - 2 * j * H[j - 1])
        der = [(-1 / s) ** j * H[j] * math.exp(-u * u) for j in range(p)]
        kend = math.exp(-0.25 / (s * s))
    else:
        K = lambda r: np.exp(-r / s)
        der = [(-1 / s) ** j * math.exp(-r0 / s) for j in range(p)]
        kend = math.exp(-0.5 / s)
    A = np.zeros((2 * p, 2 * p))
    rhs = np.zeros(2 * p)
    for j in range(p):
        A[j, j] = math.factorial(j)
        rhs[j] = epsB ** j * der[j]
        for i in range(j, 2 * p):
            A[p + j, i] = math.factorial(i) / math.factorial(i - j)
        rhs[p + j] = kend if j == 0 else 0.0
    coef = np.linalg.solve(A, rhs)

    def KR(r):
        t = (r - r0) / epsB
        out = np.where((r > r0) & (r < 0.5), np.polyval(coef[::-1], t), K(r))
        return np.where(r >= 0.5, kend, out)

    k = np.fft.fftfreq(N, d=1.0 / N) / N
    g3 = np.meshgrid(k, k, k, indexing="ij")
    bh = np.fft.fftn(KR(np.sqrt(g3[0] ** 2 + g3[1] ** 2 + g3[2] ** 2))).real / N ** 3
    M = 2 * N
    big = np.zeros((M, M, M))
    idx = np.fft.fftfreq(N, d=1.0 / N).astype(int) % M
    big[np.ix_(idx, idx, idx)] = bh
    for ax in range(3):                 # the frequency -N/2 counts half at +-N/2
        a = np.moveaxis(big, ax, 0)
        half = 0.5 * a[M - N // 2].copy()
        a[M - N // 2] = half
        a[N // 2] = half
    krf = np.fft.ifftn(big).real * M ** 3
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    m = np.round(v * ((0.25 - epsB / 2) * rng.random(n) ** (1 / 3))[:, None] * M).astype(int)
    x = rng.standard_normal(n)
    dm = (m[:, None, :] - m[None, :, :]) % M
    r = np.sqrt((((m[:, None, :] - m[None, :, :]) / M) ** 2).sum(-1))
    off = ~np.eye(n, dtype=bool)
    W = K(r) * off
    Wt = krf[dm[..., 0], dm[..., 1], dm[..., 2]] * off
    return np.linalg.norm((Wt - W) @ x) / np.linalg.norm(W @ x)


def test_laplacian_kernel_series_decays_algebraically():
    g64 = _truncation_error("gauss", 0.1, 64)
    l32 = _truncation_error("lap", 0.1, 32)
    l64 = _truncation_error("lap", 0.1, 64)
    assert g64 < 1e-10                       # the Gaussian: spectral accuracy
    assert l64 > 1e-4                        # the Laplacian RBF misses even the FP32 gate
    assert 2.0 < l32 / l64 < 12.0            # and gains only a small factor per doubling of N


def test_stored_ball_eigenvalues_recipe():
    """The stored oracle eigenvalues of the 10^5-point ball belong to the
    workload recipe (n, sigma, k), are ascending in [0, 2) and start at the
    zero eigenvalue of L_sym (eigenvector D^1/2 1)."""
    import json
    import os
    z = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "ball_n100000_eigs.json")))
    c = gen.config2()
    assert z["n"] == c["n"] and z["sigma"] == c["sigma"][0] and z["k"] == c["k"]
    lam = np.asarray(z["eigenvalues"])
    assert lam.shape == (c["k"],) and np.all(np.diff(lam) >= 0)
    assert abs(lam[0]) < 1e-12 and lam[-1] < 2.0
