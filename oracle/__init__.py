"""ORACLE -- test infrastructure only.

Plain, slow, obviously correct CPU implementation of what the GPU library
computes, in FP64.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the GPU library (``paper_2007_05239_amd``) and never imports it.

Pieces (each cites the passage it follows):

* ``kernel_matvec`` / ``kernel_rows`` -- direct O(n^2) sum of the weight
  matrix with zero diagonal, Gaussian or Laplacian RBF kernel (Sec. 2 weight
  matrix; Sec. 4 kernel sum, the kernels it names and the W = W~ - K(0) I
  identity).  C, OpenMP, Neumaier sums.
* ``median_pairwise_distance`` -- the data-driven kernel width over a node
  sample (the workloads' sigma rule).
* ``degrees``, ``nadj_matvec``, ``lsym_matvec`` -- D = diag(W 1),
  L_sym = I - D^-1/2 W D^-1/2 (Sec. 2), and the layer mean
  I - L_1 = (1/T) sum_t D_t^-1/2 W_t D_t^-1/2 (Sec. 3, eq. for I - L_1).
* ``dense_nadj``, ``eigs_dense`` -- dense assembly and LAPACK ``eigh`` for
  the k largest eigenpairs of I - L_1, mapped to lambda = 1 - mu (Sec. 3,
  Algorithm 2 step 1).
* ``eigs_iterative`` -- the same through ARPACK (scipy ``eigsh``) driving
  the C direct sum, for sizes where dense assembly is too large.
* ``power_mean_dense`` -- L_p for any p != 0 through eigendecompositions,
  with the shift delta for p < 0 (Sec. 2, eqs. (1)-(2); matrix functions via
  eigendecomposition).
* ``power_mean_power_matvec`` / ``power_mean_eigs`` -- the p-th power
  L_{p,delta}^p = (1/T) sum_t (L_sym^(t) + delta I)^p applied to a block, and
  the k smallest eigenpairs of L_{p,delta} taken as the k largest of its p-th
  power (Sec. 3), through dense eigendecompositions.
* ``pksm_apply`` -- the polynomial Krylov method of Sec. 3 for one layer:
  Lanczos on L_sym^(t), then f(T_m) e_1 of the small tridiagonal matrix with
  f(lambda) = (lambda + delta)^p (Higham, Functions of Matrices, ch. 13).
* ``allen_cahn`` / ``simplex_project`` / ``potential_grad`` -- Algorithm 2
  steps 2-4 in a fixed FP64 operation order (see ``ac.c``).
* ``oracle.fourier`` -- the trigonometric sum W_RF X that Algorithm 1
  evaluates fast (Sec. 4: regularised kernel, Fourier coefficients b_l,
  f_RF through explicit non-equispaced Fourier matrices), so that the fast
  summation's window error can be measured apart from the truncation error.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no GPU code involved)."""
    if os.path.exists(_LIB_PATH) and not force:
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    objs = []
    for src, flags in (("direct.c", ["-O3", "-fopenmp"]),
                       ("ac.c", ["-O2", "-ffp-contract=off", "-fno-fast-math"])):
        obj = os.path.join(_HERE, src[:-2] + ".%d.o" % os.getpid())
        subprocess.check_call(["gcc", "-std=c99", "-fPIC", "-c", *flags,
                               os.path.join(_HERE, src), "-o", obj])
        objs.append(obj)
    subprocess.check_call(["gcc", "-shared", "-fopenmp", *objs, "-o", tmp, "-lm"])
    for o in objs:
        os.remove(o)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _ACParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("omega0", ctypes.c_double),
                ("c", ctypes.c_double), ("dt", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int)]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_kernel_rows.argtypes = [i64, ctypes.c_int, P, ctypes.c_double, i64, P,
                                           ctypes.c_int, P, i64, P, i64]
        lib.oracle_kernel_rows.restype = ctypes.c_int
        lib.oracle_kernel_rows_k.argtypes = [i64, ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                             i64, P, ctypes.c_int, P, i64, P, i64]
        lib.oracle_kernel_rows_k.restype = ctypes.c_int
        lib.oracle_simplex_project.argtypes = [ctypes.c_int, P, P]
        lib.oracle_simplex_project.restype = None
        lib.oracle_potential_grad.argtypes = [ctypes.c_int, P, P]
        lib.oracle_potential_grad.restype = None
        lib.oracle_allen_cahn.argtypes = [i64, ctypes.c_int, ctypes.c_int, P, P, i64, P,
                                          ctypes.POINTER(_ACParams), P, P,
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_double)]
        lib.oracle_allen_cahn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# weight matrix, degrees, Laplacians
# ---------------------------------------------------------------------------
KERNELS = {"gaussian": 0, "laplacian": 1}


def kernel_rows(points, sigma, X, rows=None, kernel="gaussian"):
    """y_r = sum_{j != i_r} K(x_i - x_j) X_j for the rows i_r in ``rows`` (all
    rows if None), K(y) = exp(-||y||^2 / sigma^2) (gaussian) or
    exp(-||y|| / sigma) (laplacian), Sec. 4.  X: n or n x b.  Returns
    len(rows) x b (or a vector for vector X)."""
    lib = _load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    vec = X.ndim == 1
    Xf = np.asfortranarray(X.reshape(n, -1), dtype=np.float64)
    b = Xf.shape[1]
    if rows is None:
        nr, rp = n, None
        rows_arr = None
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nr = rows_arr.shape[0]
    Y = np.zeros((nr, b), dtype=np.float64, order="F")
    rc = lib.oracle_kernel_rows_k(n, d, _p(pts), float(sigma), KERNELS[kernel], nr,
                                  None if rows_arr is None else _p(rows_arr), b,
                                  _p(Xf), n, _p(Y), max(nr, 1))
    if rc != 0:
        raise ValueError("oracle_kernel_rows: bad argument")
    return Y[:, 0] if vec else Y


def kernel_matvec(points, sigma, X, kernel="gaussian"):
    """W X with W_ij = K(x_i - x_j), W_ii = 0 (Sec. 2, Sec. 4)."""
    return kernel_rows(points, sigma, X, None, kernel)


def degrees(points, sigma, kernel="gaussian"):
    """deg(x_i) = sum_j w_ij (Sec. 2).  Raises if a node is isolated."""
    n = points.shape[0]
    d = kernel_rows(points, sigma, np.ones(n), None, kernel)
    if np.any(d <= 0.0):
        raise ValueError("isolated node: a degree is zero")
    return d


class Layer:
    """One graph layer: points, sigma, and its degrees (computed once)."""

    def __init__(self, points, sigma, kernel="gaussian"):
        self.points = np.ascontiguousarray(points, dtype=np.float64)
        self.sigma = float(sigma)
        self.kernel = kernel
        self.deg = degrees(self.points, self.sigma, kernel)
        self.dinv_sqrt = 1.0 / np.sqrt(self.deg)


def nadj_matvec(layers, X, rows=None):
    """(1/T) sum_t D_t^-1/2 W_t D_t^-1/2 X  (= (I - L_1) X; Sec. 3).  With
    ``rows`` only those rows are evaluated (each needs one O(n) pass)."""
    T = len(layers)
    X2 = X.reshape(X.shape[0], -1)
    out = None
    for L in layers:
        Z = L.dinv_sqrt[:, None] * X2
        Y = kernel_rows(L.points, L.sigma, Z, rows, L.kernel)
        sc = L.dinv_sqrt if rows is None else L.dinv_sqrt[np.asarray(rows)]
        Y = sc[:, None] * Y
        out = Y if out is None else out + Y
    out = out / T
    return out[:, 0] if X.ndim == 1 else out


def lsym_matvec(layers, X, rows=None):
    """L_1 X = X - (I - L_1) X; for one layer this is L_sym X (Sec. 2)."""
    A = nadj_matvec(layers, X, rows)
    X2 = X if rows is None else X[np.asarray(rows)]
    return X2 - A


def dense_weight(points, sigma, kernel="gaussian"):
    """Dense W with zero diagonal (Sec. 2), for small n."""
    p = np.asarray(points, dtype=np.float64)
    diff = p[:, None, :] - p[None, :, :]
    r2 = (diff ** 2).sum(-1)
    W = np.exp(-r2 / (sigma * sigma)) if kernel == "gaussian" else np.exp(-np.sqrt(r2) / sigma)
    np.fill_diagonal(W, 0.0)
    return W


def dense_nadj(layers):
    """Dense (1/T) sum_t D_t^-1/2 W_t D_t^-1/2 (Sec. 3), small n only."""
    A = None
    for L in layers:
        W = dense_weight(L.points, L.sigma, L.kernel)
        d = W.sum(1)
        if np.any(d <= 0):
            raise ValueError("isolated node")
        s = 1.0 / np.sqrt(d)
        M = s[:, None] * W * s[None, :]
        A = M if A is None else A + M
    return A / len(layers)


def _fix_signs(V):
    """Sign convention: the largest-magnitude entry of each vector is
    positive (lowest index on ties)."""
    V = V.copy()
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def eigs_dense(layers, k):
    """k smallest eigenpairs of L_1 via the k largest of I - L_1 (Sec. 3,
    Algorithm 2 step 1): lambda = 1 - mu, ascending."""
    A = dense_nadj(layers)
    mu, V = np.linalg.eigh(A)
    idx = np.argsort(-mu, kind="stable")[:k]
    lam = 1.0 - mu[idx]
    return lam, _fix_signs(V[:, idx])


def eigs_iterative(layers, k, tol=1e-12, seed=0):
    """Same eigenpairs through ARPACK (scipy eigsh) on the O(n^2) C sum."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = layers[0].points.shape[0]
    op = LinearOperator((n, n), matvec=lambda x: nadj_matvec(layers, np.asarray(x).ravel()),
                        dtype=np.float64)
    v0 = np.random.Generator(np.random.Philox(seed)).standard_normal(n)
    mu, V = eigsh(op, k=k, which="LA", tol=tol, v0=v0, ncv=max(2 * k + 1, 20))
    idx = np.argsort(-mu, kind="stable")
    return 1.0 - mu[idx], _fix_signs(V[:, idx])


def power_mean_dense(layers, p):
    """L_p = ((1/T) sum_t (L_sym^(t) + delta I)^p)^(1/p) through
    eigendecompositions; delta = log(1+|p|) for p < 0, 0 for p > 0
    (Sec. 2, eqs. (1)-(2) and the matrix-function identity)."""
    if p == 0:
        raise ValueError("p must be nonzero")
    delta = np.log1p(abs(p)) if p < 0 else 0.0
    acc = None
    for L in layers:
        W = dense_weight(L.points, L.sigma, L.kernel)
        s = 1.0 / np.sqrt(W.sum(1))
        Ls = np.eye(W.shape[0]) - s[:, None] * W * s[None, :]
        lam, V = np.linalg.eigh(Ls)
        lam = np.clip(lam, 0.0, None) + delta
        M = (V * lam ** p) @ V.T
        acc = M if acc is None else acc + M
    acc /= len(layers)
    lam, V = np.linalg.eigh(acc)
    return (V * np.clip(lam, 0.0, None) ** (1.0 / p)) @ V.T


def median_pairwise_distance(features, sample, cols=None):
    """Median of the Euclidean distances ||x_a - x_b||_2 over the pairs a < b
    of the sampled rows, over the feature columns ``cols`` (all if None); an
    even number of pairs gives the mean of the middle two.  The kernel-width
    rule of the synthetic workloads (Sec. 6 leaves sigma to a grid search).
    Each squared distance is summed over the columns in order."""
    F = np.asarray(features, dtype=np.float64)
    X = F[np.asarray(sample, dtype=np.int64)]
    if cols is not None:
        X = X[:, list(cols)]
    a, b = np.triu_indices(X.shape[0], k=1)
    r2 = np.zeros(a.shape[0])
    for k in range(X.shape[1]):
        dk = X[a, k] - X[b, k]
        r2 = r2 + dk * dk
    return float(np.median(np.sqrt(r2)))


def shift_delta(p):
    """delta = log(1 + |p|) for p < 0 and 0 for p > 0 (Sec. 2, shifted power
    mean)."""
    if p == 0:
        raise ValueError("p must be nonzero")
    return float(np.log1p(abs(p))) if p < 0 else 0.0


def lsym_dense(L):
    """Dense L_sym = I - D^-1/2 W D^-1/2 of one layer (Sec. 2), small n."""
    W = dense_weight(L.points, L.sigma, L.kernel)
    s = 1.0 / np.sqrt(W.sum(1))
    return np.eye(W.shape[0]) - s[:, None] * W * s[None, :]


def power_mean_power_dense(layers, p):
    """Dense L_{p,delta}^p = (1/T) sum_t (L_sym^(t) + delta I)^p (Sec. 3),
    every power through an eigendecomposition of L_sym^(t); its eigenvalues
    are clipped at 0 first (they are >= 0 in exact arithmetic)."""
    delta = shift_delta(p)
    acc = None
    for L in layers:
        lam, V = np.linalg.eigh(lsym_dense(L))
        lam = np.clip(lam, 0.0, None) + delta
        M = (V * lam ** p) @ V.T
        acc = M if acc is None else acc + M
    return acc / len(layers)


def power_mean_power_matvec(layers, p, X):
    """L_{p,delta}^p X (Sec. 3), small n."""
    return power_mean_power_dense(layers, p) @ X


def power_mean_eigs(layers, p, k):
    """k smallest eigenpairs of L_{p,delta} (p < 0) or L_p (p > 0): the k
    largest eigenvalues mu of the p-th power for p < 0 (f = lambda^p reverses
    the order), the k smallest for p > 0, then lambda = mu^(1/p) (Sec. 3).
    Eigenvalues ascending; sign convention of ``_fix_signs``."""
    mu, V = np.linalg.eigh(power_mean_power_dense(layers, p))
    idx = np.argsort(-mu if p < 0 else mu, kind="stable")[:k]
    lam = np.clip(mu[idx], 0.0, None) ** (1.0 / p)
    return lam, _fix_signs(V[:, idx])


def pksm_apply(Ls, p, x, tol=1e-12, max_steps=128, check_every=4):
    """Polynomial Krylov approximation of (Ls + delta I)^p x for a symmetric
    Ls with spectrum in [0, 2] (Sec. 3, PKSM; Higham, Functions of Matrices,
    ch. 13).  ``Ls`` is a dense matrix or a function x -> Ls x.

    Lanczos on Ls from v_1 = x / ||x|| (no reorthogonalisation):
      w = Ls v_j - beta_{j-1} v_{j-1};  alpha_j = v_j^T w;  w -= alpha_j v_j;
      beta_j = ||w||;  v_{j+1} = w / beta_j  (0 if beta_j = 0).
    T_m = tridiag(beta, alpha, beta) is the projection of Ls; the shift only
    moves its eigenvalues.  With T_m = Y diag(theta) Y^T,
      c_m = Y g(theta) Y^T e_1,  g(theta) = ((max(theta, 0) + delta) / delta)^p,
    the approximation is y_m = ||x|| delta^p V_m c_m.  g <= 1, so the change
    ||c_m - c_{m-s}|| (every s = check_every steps) measures the error
    relative to ||x|| ||f(Ls)||; stop when it is <= tol or at max_steps.
    Returns (y, steps, converged)."""
    delta = shift_delta(p)
    if p >= 0:
        raise ValueError("pksm_apply is for p < 0")
    mv = (lambda v: Ls @ v) if not callable(Ls) else Ls
    x = np.asarray(x, dtype=np.float64)
    nx = float(np.linalg.norm(x))
    if nx == 0.0:
        return np.zeros_like(x), 0, True
    V = [x / nx]
    alpha, beta = [], []
    c_prev = np.zeros(0)
    c = None
    converged = False
    m = 0
    for j in range(max_steps):
        w = mv(V[j])
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        a = float(V[j] @ w)
        w = w - a * V[j]
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        m = j + 1
        if m % check_every == 0 or m == max_steps:
            Tm = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
            theta, Y = np.linalg.eigh(Tm)
            g = ((np.clip(theta, 0.0, None) + delta) / delta) ** p
            c = Y @ (g * Y[0, :])
            prev = np.concatenate([c_prev, np.zeros(m - c_prev.size)])
            change = float(np.linalg.norm(c - prev))
            c_prev = c
            if change <= tol:
                converged = True
                break
        if m < max_steps:
            V.append(w / b if b > 0.0 else np.zeros_like(w))
    y = (nx * delta ** p) * (np.array(V[:m]).T @ c)
    return y, m, converged


# ---------------------------------------------------------------------------
# Allen--Cahn (Algorithm 2 steps 2-4)
# ---------------------------------------------------------------------------
def simplex_project(y):
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float64)
    x = np.empty_like(y)
    lib.oracle_simplex_project(y.shape[0], _p(y), _p(x))
    return x


def potential_grad(u):
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    T = np.empty_like(u)
    lib.oracle_potential_grad(u.shape[0], _p(u), _p(T))
    return T


def allen_cahn(evals, evecs, labels, m, eps=5e-3, omega0=1000.0, c=None, dt=0.01,
               tol=1e-6, max_iter=300):
    """Returns (U n x m, pred n, iterations, min top-two margin)."""
    lib = _load()
    if c is None:
        c = omega0 + 3.0 / eps
    evecs = np.asfortranarray(evecs, dtype=np.float64)
    n, k = evecs.shape
    ev = np.ascontiguousarray(evals, dtype=np.float64)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    U = np.empty((n, m), dtype=np.float64)
    pred = np.empty(n, dtype=np.int32)
    it = ctypes.c_int(0)
    mm = ctypes.c_double(0.0)
    prm = _ACParams(eps, omega0, c, dt, tol, max_iter)
    rc = lib.oracle_allen_cahn(n, k, m, _p(ev), _p(evecs), n, _p(lab), ctypes.byref(prm),
                               _p(U), _p(pred), ctypes.byref(it), ctypes.byref(mm))
    if rc != 0:
        raise ValueError("oracle_allen_cahn: bad argument")
    return U, pred, it.value, mm.value
