"""Pins of the oracle's Fourier approximation (Sec. 4: K_R, b_l, f_RF) to
what the mathematics fixes, independent of the oracle's own code paths:

* the regularised kernel meets K to order p at r0 = 1/2 - eps_B and reaches
  K(1/2) to order p at 1/2 (halving h divides the gap by about 2^p);
* b_l of a narrow Gaussian equals the Poisson-summed closed form
  sum_m (sqrt(pi) sigma)^d exp(-pi^2 sigma^2 |l + m N|^2);
* at lattice nodes (y on the grid 1/N) the trigonometric sum reproduces the
  sampled regularised kernel at the wrapped pair differences exactly;
* with the band covering the kernel, the trigonometric sum equals the
  direct C sum of the main oracle;
* with a band that truncates the kernel it does not (the error the fast
  summation's window error is separated from).
"""
import numpy as np
import pytest

import oracle
from oracle import fourier
from workloads import gen


@pytest.mark.parametrize("p", [3, 5])
def test_regularized_kernel_contact_orders(p):
    sigma, eps_B = 0.2, 1.0 / 16
    r0 = 0.5 - eps_B
    K = lambda r: np.exp(-np.asarray(r) ** 2 / sigma ** 2)
    for h in (1e-2, 5e-3):
        assert fourier.regularized_gaussian(np.array([r0 - h]), sigma, eps_B, p)[0] == K(r0 - h)
    gaps0 = [abs(fourier.regularized_gaussian(np.array([r0 + h]), sigma, eps_B, p)[0] - K(r0 + h))
             for h in (8e-3, 4e-3)]
    kend = K(0.5)
    gaps1 = [abs(fourier.regularized_gaussian(np.array([0.5 - h]), sigma, eps_B, p)[0] - kend)
             for h in (8e-3, 4e-3)]
    for g in (gaps0, gaps1):
        ratio = g[0] / g[1]
        assert 2 ** p * 0.75 <= ratio <= 2 ** p * 1.3, (p, g, ratio)
    # constant beyond 1/2
    far = fourier.regularized_gaussian(np.array([0.5, 0.6, 0.8]), sigma, eps_B, p)
    assert np.all(far == kend)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_fourier_coefficients_closed_form(d):
    sigma, N = 0.05, 32 if d == 3 else 64
    b = fourier.fourier_coefficients(sigma, d, N, 1.0 / 16, 5)
    l1 = np.fft.fftfreq(N, 1.0 / N)
    grids = np.meshgrid(*([l1] * d), indexing="ij")
    ref = np.zeros_like(b)
    for shift in np.ndindex(*([5] * d)):
        m = np.array(shift) - 2
        r2 = sum((g + mi * N) ** 2 for g, mi in zip(grids, m))
        ref += (np.sqrt(np.pi) * sigma) ** d * np.exp(-np.pi ** 2 * sigma ** 2 * r2)
    assert np.abs(b - ref).max() <= 1e-13 * ref.max()
    assert ref.max() == pytest.approx((np.sqrt(np.pi) * sigma) ** d)


@pytest.mark.parametrize("d,N", [(1, 16), (2, 16), (3, 8)])
def test_fourier_sum_interpolates_on_the_lattice(d, N):
    rng = np.random.default_rng(7 + d)
    n, sigma, eps_B, p = 60, 0.15, 1.0 / 16, 5
    k = rng.integers(-N // 2, N // 2, size=(n, d))
    y = k / N
    X = rng.standard_normal((n, 3))
    got = fourier.fourier_sum_scaled(y, sigma, X, N, eps_B, p)
    diff = y[:, None, :] - y[None, :, :]
    diff = diff - np.round(diff)          # wrap to the torus [-1/2, 1/2)
    r = np.sqrt((diff ** 2).sum(-1))
    KR = fourier.regularized_gaussian(r, sigma, eps_B, p)
    np.fill_diagonal(KR, 0.0)
    ref = KR @ X
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d,N,sigma,gate", [(1, 64, 0.3, 1e-11), (2, 64, 0.3, 1e-11),
                                             (3, 32, 0.43, 1e-8)])
def test_fourier_sum_equals_direct_sum_when_band_covers_kernel(d, N, sigma, gate):
    """The two error sources of K_RF are the dropped Gaussian tail,
    exp(-(pi sigma_s N / 2)^2), and the regularisation's kink of order p,
    scaled by K(r0); both are small at these (N, sigma)."""
    n = 300
    pts = gen.uniform_ball(n, d, 1.0, 51 + d)
    X = gen.test_vectors(n, 2, 52 + d)
    _, s = fourier.torus_scale(pts, 1.0 / 16)
    ss = s * sigma
    assert np.exp(-(np.pi * ss * N / 2) ** 2) < gate / 10
    assert np.exp(-(0.4375 / ss) ** 2) < gate / 10
    got = fourier.fourier_sum(pts, sigma, X, N)
    ref = oracle.kernel_matvec(pts, sigma, X)
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= gate, err


def test_fourier_sum_truncates_at_small_band():
    n, d, sigma = 300, 2, 0.2
    pts = gen.uniform_ball(n, d, 1.0, 61)
    X = gen.test_vectors(n, 1, 62)
    ref = oracle.kernel_matvec(pts, sigma, X)
    errs = []
    for N in (8, 16, 32):
        got = fourier.fourier_sum(pts, sigma, X, N)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[0] > 0.1 and errs[0] > errs[1] > 10 * errs[2], errs
