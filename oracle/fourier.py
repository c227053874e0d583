"""ORACLE -- test infrastructure only (same rules as the package: only
``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
may import it; it shares no code with the GPU library).

The Fourier approximation of the kernel sum that Algorithm 1 evaluates fast
(Sec. 4, eqs. for K_RF and f_RF), written as its plain definition: the
trigonometric sum over the frequency set, evaluated with explicit
non-equispaced Fourier matrices (an NDFT, O(n N^d)) instead of windows,
oversampled grids and FFTs.  The fast summation's window error is the only
difference between the two, so comparing them isolates it from the kernel's
truncation error.  FP64 throughout.

* ``torus_scale`` -- the rescale that puts every node in the ball of radius
  1/4 - eps_B/2 about the bounding-box centre, so that every pair difference
  lies where the regularised kernel equals K (Sec. 4, the node domain of
  Algorithm 1); sigma scales with the points.
* ``regularized_gaussian`` -- K_R: the Gaussian up to r0 = 1/2 - eps_B, on
  (r0, 1/2) the degree-(2p-1) polynomial that takes K's derivatives 0..p-1
  at r0 and the value K(1/2) with derivatives 1..p-1 zero at 1/2, and
  K(1/2) beyond (Sec. 4 names a regularised kernel and defers its form; this
  two-point Taylor form is the reading the library takes too).  The
  interpolating polynomial comes from scipy's Bernstein-basis Hermite
  construction, the Gaussian's derivatives from the recurrence
  P_{j+1} = P_j' - (2 r / sigma^2) P_j of K^(j) = P_j K.
* ``fourier_coefficients`` -- b_l = N^-d sum_{k in I_N} K_R(k/N)
  exp(-2 pi i l k / N), l in I_N (Sec. 4, footnote to Algorithm 1), by
  numpy's FFT.
* ``fourier_sum`` -- W_RF v = Re sum_l c_l b_l A_l (A_l^* v) - K(0) v with
  A_l = exp(2 pi i l y_j) (Sec. 4, eq. for f_RF and W = W~ - K(0) I).  The
  frequency set is {-N/2, ..., N/2}^d with the Nyquist term of each
  coordinate split evenly between -N/2 and +N/2 (c_l = 1/2 per coordinate
  at |l_t| = N/2) and b periodic in l with period N: this makes K_RF real
  and even, exactly symmetric in i and j, and equal to the sum over I_N at
  every lattice point (where exp(i pi N k/N) = exp(-i pi N k/N)).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import Polynomial
from scipy.interpolate import BPoly


def torus_scale(points, eps_B):
    """(scaled points, scale s): y = s (x - c) with c the bounding-box centre
    and s = (1/4 - eps_B/2) / max_i ||x_i - c||."""
    P = np.asarray(points, dtype=np.float64)
    c = 0.5 * (P.min(axis=0) + P.max(axis=0))
    R = np.sqrt(((P - c) ** 2).sum(axis=1)).max()
    s = (0.25 - 0.5 * eps_B) / R if R > 0 else 1.0
    return (P - c) * s, s


def gaussian_derivatives(r, sigma, p):
    """[K(r), K'(r), ..., K^(p-1)(r)] for K(r) = exp(-r^2/sigma^2)."""
    K = np.exp(-(r * r) / (sigma * sigma))
    P = Polynomial([1.0])
    x = Polynomial([0.0, 1.0])
    out = []
    for _ in range(p):
        out.append(P(r) * K)
        P = P.deriv() - (2.0 / (sigma * sigma)) * x * P
    return out


def regularized_gaussian(r, sigma, eps_B, p):
    """K_R(r) of the Gaussian of width sigma (on the torus scale)."""
    r = np.asarray(r, dtype=np.float64)
    r0 = 0.5 - eps_B
    kend = np.exp(-0.25 / (sigma * sigma))
    left = gaussian_derivatives(r0, sigma, p)
    right = [kend] + [0.0] * (p - 1)
    poly = BPoly.from_derivatives([r0, 0.5], [left, right])
    out = np.where(r <= r0, np.exp(-(r * r) / (sigma * sigma)), kend)
    mid = (r > r0) & (r < 0.5)
    out = np.asarray(out, dtype=np.float64)
    out[mid] = poly(r[mid])
    return out


def fourier_coefficients(sigma, d, N, eps_B, p):
    """b_l for l in I_N^d, as a d-dimensional array indexed by l mod N."""
    k1 = np.arange(N)
    k1 = np.where(k1 < N // 2, k1, k1 - N)       # FFT order: 0..N/2-1, -N/2..-1
    grids = np.meshgrid(*([k1 / N] * d), indexing="ij")
    r = np.sqrt(sum(g * g for g in grids))
    S = regularized_gaussian(r, sigma, eps_B, p)
    # b_l = N^-d sum_k S_k exp(-2 pi i l k / N): the forward DFT over k
    bh = np.fft.fftn(S) / float(N) ** d
    return bh.real


def _freqs(N, d):
    """Frequencies {-N/2..N/2}^d (N+1 per coordinate) and their weights."""
    l1 = np.arange(-N // 2, N // 2 + 1)
    c1 = np.where(np.abs(l1) == N // 2, 0.5, 1.0)
    L = np.stack([g.ravel() for g in np.meshgrid(*([l1] * d), indexing="ij")], axis=1)
    C = np.prod(np.stack([g.ravel() for g in np.meshgrid(*([c1] * d), indexing="ij")], axis=1),
                axis=1)
    return L, C


def fourier_sum_scaled(y, sigma_s, X, N, eps_B=1.0 / 16, p=5, rows=None):
    """W_RF X on already scaled nodes y (n x d), kernel width sigma_s on the
    same scale.  Returns len(rows) x b (all rows if None)."""
    y = np.asarray(y, dtype=np.float64)
    n, d = y.shape
    X2 = np.asarray(X, dtype=np.float64).reshape(n, -1)
    bh = fourier_coefficients(sigma_s, d, N, eps_B, p)
    L, C = _freqs(N, d)
    coef = C * bh[tuple((L % N).T)]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    # fhat_l = sum_j v_j exp(-2 pi i l y_j), in chunks of nodes
    fhat = np.zeros((L.shape[0], X2.shape[1]), dtype=np.complex128)
    ch = max(1, min(512, (1 << 22) // L.shape[0]))
    for j0 in range(0, n, ch):
        A = np.exp(2j * np.pi * (y[j0:j0 + ch] @ L.T))
        fhat += A.conj().T @ X2[j0:j0 + ch]
    g = coef[:, None] * fhat
    out = np.empty((rows.shape[0], X2.shape[1]))
    for i0 in range(0, rows.shape[0], ch):
        A = np.exp(2j * np.pi * (y[rows[i0:i0 + ch]] @ L.T))
        out[i0:i0 + ch] = (A @ g).real
    # W = W~ - K(0) I with K(0) = 1
    out -= X2[rows]
    return out[:, 0] if np.asarray(X).ndim == 1 else out


def fourier_sum(points, sigma, X, N, eps_B=1.0 / 16, p=5, rows=None):
    """W_RF X for raw nodes and kernel width: torus scale, then the sum."""
    y, s = torus_scale(points, eps_B)
    return fourier_sum_scaled(y, s * sigma, X, N, eps_B, p, rows)
