"""Thin ctypes binding of libmlg.so (include/mlg.h).

Argument marshalling only: every computation runs in the HIP library.  Arrays
may be numpy arrays (host) or torch CUDA/HIP tensors (device, passed with
MLG_DEVICE_PTRS).  There is no CPU fallback: if libmlg.so is missing or does
not load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlg.so")

MLG_OK = 0
MLG_WARN_NOT_CONVERGED = 1
MLG_ERR_ARG = -1
MLG_ERR_RANGE = -2
MLG_ERR_ISOLATED = -3
MLG_ERR_NOMEM = -4
MLG_ERR_HIP = -5
MLG_ERR_NOT_IMPL = -6

MLG_DEVICE_PTRS = 1
MLG_ASYNC = 4
MLG_SKIP_DEGREES = 2
MLG_METHOD_DIRECT = 0
MLG_METHOD_NFFT = 1
MLG_KERNEL_GAUSSIAN = 0
MLG_KERNEL_LAPLACIAN = 1
MLG_OP_NADJ = 0
MLG_OP_LSYM = 1
MLG_OP_W = 2

STAGES = ["scatter_in", "spread", "gather", "fft", "interp", "gather_out", "direct", "unused"]

EXPORTED = ["mlg_last_error", "mlg_version", "mlg_graph_create", "mlg_graph_create_grouped",
            "mlg_median_pairwise_distance", "mlg_graph_destroy",
            "mlg_graph_degrees", "mlg_graph_synchronize", "mlg_kernel_matvec", "mlg_laplacian_matvec",
            "mlg_lanczos_eigs", "mlg_power_mean_matvec", "mlg_allen_cahn_ssl",
            "mlg_profile_stages", "mlg_graph_layer_info", "mlg_autotune_layer",
            "mlg_kernel_matvec_noalloc"]

MLG_NOALLOC_SCRATCH_BYTES = 64 << 20


class MlgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mlg status %d: %s" % (code, msg))
        self.code = code


class KParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("precision", ctypes.c_int), ("N", ctypes.c_int),
                ("window", ctypes.c_int), ("eps_B", ctypes.c_double), ("p_reg", ctypes.c_int),
                ("bin", ctypes.c_int), ("kernel", ctypes.c_int)]


class EigInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("nconv", ctypes.c_int), ("max_resid", ctypes.c_double),
                ("inner_steps", ctypes.c_int), ("inner_unconverged", ctypes.c_int)]


class PksmParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_steps", ctypes.c_int)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int), ("N", ctypes.c_int), ("bin", ctypes.c_int),
                ("tried", ctypes.c_int), ("passed", ctypes.c_int), ("err", ctypes.c_double),
                ("ms", ctypes.c_double)]


class ACParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("omega0", ctypes.c_double), ("c", ctypes.c_double),
                ("dt", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int)]


def kparams(method="nfft", precision=32, N=64, window=0, eps_B=1.0 / 16, p_reg=5, bin=1,
            kernel="gaussian"):
    m = MLG_METHOD_NFFT if method == "nfft" else MLG_METHOD_DIRECT
    kk = MLG_KERNEL_LAPLACIAN if kernel == "laplacian" else MLG_KERNEL_GAUSSIAN
    return KParams(m, precision, N, window, eps_B, p_reg, bin, kk)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmlg.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    sig = {
        "mlg_last_error": ([], ctypes.c_char_p),
        "mlg_version": ([], ctypes.c_char_p),
        "mlg_graph_create": ([ctypes.POINTER(P), i64, I, P, P, P, P, I, P], I),
        "mlg_graph_destroy": ([P], I),
        "mlg_graph_create_grouped": ([ctypes.POINTER(P), i64, I, P, I, P, P, P, P, I, P], I),
        "mlg_median_pairwise_distance": ([i64, I, P, I, P, I, P, ctypes.POINTER(ctypes.c_double),
                                          I, P], I),
        "mlg_graph_degrees": ([P, I, P, I], I),
        "mlg_kernel_matvec": ([i64, I, P, ctypes.c_double, ctypes.POINTER(KParams), I, P, i64, P,
                               i64, I, P], I),
        "mlg_kernel_matvec_noalloc": ([i64, I, P, ctypes.c_double, ctypes.POINTER(KParams), I, P,
                                       i64, P, i64, P], I),
        "mlg_laplacian_matvec": ([P, I, I, I, P, i64, P, i64, I], I),
        "mlg_graph_synchronize": ([P], I),
        "mlg_lanczos_eigs": ([P, I, ctypes.c_double, I, I, ctypes.c_double, I, ctypes.c_uint64, P,
                              P, P, i64, ctypes.POINTER(EigInfo), ctypes.POINTER(PksmParams), I],
                             I),
        "mlg_power_mean_matvec": ([P, I, ctypes.c_double, I, P, i64, P, i64,
                                   ctypes.POINTER(PksmParams), ctypes.POINTER(ctypes.c_int), I], I),
        "mlg_allen_cahn_ssl": ([i64, I, I, P, P, i64, P, ctypes.POINTER(ACParams), P, P,
                                ctypes.POINTER(ctypes.c_int), I, P], I),
        "mlg_profile_stages": ([P, I, I, I, P, i64, P, i64, I, P, I], I),
        "mlg_graph_layer_info": ([P, I, P, P], I),
        "mlg_autotune_layer": ([i64, I, P, ctypes.c_double, I, I, ctypes.c_double, I,
                                ctypes.c_uint64, I, P, ctypes.POINTER(KParams),
                                ctypes.POINTER(TuneInfo)], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def version():
    return _lib.mlg_version().decode()


def _check(rc, allow_warn=False):
    if rc == MLG_OK or (allow_warn and rc == MLG_WARN_NOT_CONVERGED):
        return rc
    raise MlgError(rc, _lib.mlg_last_error().decode())


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _sync():
    import torch
    torch.cuda.synchronize()


def _ptr(a):
    """(pointer, is_device) of a numpy array or torch tensor."""
    if _is_torch(a):
        return ctypes.c_void_p(a.data_ptr()), bool(a.is_cuda)
    return a.ctypes.data_as(ctypes.c_void_p), False


def _colmajor(X):
    """Column-major view requirements: returns (array, ld, b)."""
    if _is_torch(X):
        import torch
        if X.dim() == 1:
            X = X.reshape(-1, 1)
        Xt = X.t().contiguous()          # b x n row-major == n x b column-major
        return Xt, X.shape[0], X.shape[1]
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    X = np.asfortranarray(X)
    return X, X.shape[0], X.shape[1]


def autotune_layer(points, sigma, precision=32, b=16, tol=1e-4, nrows=128, seed=0):
    """NFFT window, bandwidth and bin for one layer (mlg_autotune_layer): returns
    (KParams, info dict).  points n x d (numpy or torch CUDA).  Raises
    MlgError (MLG_ERR_RANGE) if no candidate meets tol; the exception then
    carries the info of the most accurate candidate as `.info`."""
    if _is_torch(points):
        pts = points.contiguous()
        flags = MLG_DEVICE_PTRS if pts.is_cuda else 0
        if pts.is_cuda:
            _sync()
        ptr = _ptr(pts)[0]
    else:
        pts = np.ascontiguousarray(points, dtype=np.float64)
        flags = 0
        ptr = pts.ctypes.data
    n, d = int(pts.shape[0]), int(pts.shape[1])
    kp = KParams()
    info = TuneInfo()
    rc = _lib.mlg_autotune_layer(n, d, ptr, float(sigma), int(precision), int(b), float(tol),
                                 int(nrows), int(seed) & (2 ** 64 - 1), flags, None,
                                 ctypes.byref(kp), ctypes.byref(info))
    out = {f: getattr(info, f) for f, _ in TuneInfo._fields_}
    if rc != MLG_OK:
        e = MlgError(rc, _lib.mlg_last_error().decode())
        e.info = out
        raise e
    return kp, out


def stride_groups(D, per_layer):
    """Feature groups of `per_layer` columns taken at stride D // per_layer:
    (0, s, 2s, ...), (1, s + 1, ...), ...; leftover columns (D not a multiple)
    form a last, smaller group.  For D = 102: per_layer 2 gives (0, 51), ...,
    (50, 101) and per_layer 3 gives (0, 34, 68), ..., (33, 67, 101) -- the
    band pairings of Sec. 8.3 (0-based)."""
    if per_layer < 1 or D < 1:
        raise ValueError("need D >= 1 and per_layer >= 1")
    s = D // per_layer
    if s == 0:
        return [tuple(range(D))]
    groups = [tuple(i + k * s for k in range(per_layer)) for i in range(s)]
    used = s * per_layer
    if used < D:
        groups.append(tuple(range(used, D)))
    return groups


def median_pairwise_distance(features, sample, cols=None):
    """Median of the pairwise distances of the sampled rows over `cols`
    (mlg_median_pairwise_distance); features n x D (numpy or torch CUDA)."""
    if _is_torch(features):
        F = features.contiguous()
        flags = MLG_DEVICE_PTRS if F.is_cuda else 0
        if F.is_cuda:
            _sync()
    else:
        F = np.ascontiguousarray(features, dtype=np.float64)
        flags = 0
    n, D = int(F.shape[0]), int(F.shape[1])
    d = D if cols is None else len(cols)
    colarr = None if cols is None else (ctypes.c_int * d)(*[int(c) for c in cols])
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    out = ctypes.c_double(0.0)
    _check(_lib.mlg_median_pairwise_distance(n, D, _ptr(F)[0], d, colarr, int(smp.shape[0]),
                                             smp.ctypes.data_as(ctypes.c_void_p),
                                             ctypes.byref(out), flags, None))
    return out.value


class Graph:
    """A multilayer graph (mlg_graph_create); one layer per point set."""

    @classmethod
    def from_features(cls, features, groups, sigmas, params=None, degrees=True):
        """Feature grouping (mlg_graph_create_grouped): layer t uses the
        columns groups[t] of the n x D feature matrix."""
        self = cls.__new__(cls)
        if _is_torch(features):
            F = features.contiguous()
            dev = bool(F.is_cuda)
            if dev:
                _sync()
        else:
            F = np.ascontiguousarray(features, dtype=np.float64)
            dev = False
        self.n = int(F.shape[0])
        self.T = len(groups)
        D = int(F.shape[1])
        if params is None:
            params = [kparams() for _ in groups]
        elif isinstance(params, KParams):
            params = [params] * self.T
        dims = (ctypes.c_int * self.T)(*[len(g) for g in groups])
        flat = [int(c) for g in groups for c in g]
        cols = (ctypes.c_int * len(flat))(*flat)
        sarr = (ctypes.c_double * self.T)(*[float(x) for x in sigmas])
        karr = (KParams * self.T)(*params)
        h = ctypes.c_void_p()
        flags = (MLG_DEVICE_PTRS if dev else 0) | (0 if degrees else MLG_SKIP_DEGREES)
        _check(_lib.mlg_graph_create_grouped(ctypes.byref(h), self.n, D, _ptr(F)[0], self.T, dims,
                                             cols, sarr, karr, flags, None))
        self._h = h
        self._keep = []
        return self

    def __init__(self, layers, sigmas, params=None, device=False, degrees=True):
        self.n = int(layers[0].shape[0])
        self.T = len(layers)
        if params is None:
            params = [kparams() for _ in layers]
        elif isinstance(params, KParams):
            params = [params] * self.T
        ds = (ctypes.c_int * self.T)(*[int(L.shape[1]) for L in layers])
        self._keep = []
        ptrs = []
        dev = False
        for L in layers:
            if _is_torch(L):
                L = L.contiguous()
                dev = bool(L.is_cuda)
            else:
                L = np.ascontiguousarray(L, dtype=np.float64)
            self._keep.append(L)
            ptrs.append(_ptr(L)[0].value)
        if dev:
            _sync()
        parr = (ctypes.c_void_p * self.T)(*ptrs)
        sarr = (ctypes.c_double * self.T)(*[float(s) for s in sigmas])
        karr = (KParams * self.T)(*params)
        h = ctypes.c_void_p()
        flags = (MLG_DEVICE_PTRS if dev else 0) | (0 if degrees else MLG_SKIP_DEGREES)
        _check(_lib.mlg_graph_create(ctypes.byref(h), self.n, self.T, ds, parr, sarr, karr,
                                     flags, None))
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.mlg_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def degrees(self, layer):
        out = np.empty(self.n)
        _check(_lib.mlg_graph_degrees(self._h, layer, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def layer_info(self, layer):
        ip = (ctypes.c_int * 6)()
        dp = (ctypes.c_double * 2)()
        _check(_lib.mlg_graph_layer_info(self._h, layer, ip, dp))
        return dict(d=ip[0], N=ip[1], window=ip[2], bin=ip[3], precision=ip[4], method=ip[5],
                    sigma_scaled=dp[0], scale=dp[1])

    def laplacian_matvec(self, layer, op, X, out=None):
        """Y = op X; X n x b (numpy -> numpy, torch CUDA -> torch CUDA)."""
        Xc, n, b = _colmajor(X)
        if _is_torch(Xc):
            import torch
            Y = torch.empty((b, n), dtype=torch.float64, device=Xc.device)
            _sync()
            _check(_lib.mlg_laplacian_matvec(self._h, layer, op, b, _ptr(Xc)[0], n, _ptr(Y)[0], n,
                                             MLG_DEVICE_PTRS))
            return Y.t()
        Y = np.zeros((n, b), order="F")
        _check(_lib.mlg_laplacian_matvec(self._h, layer, op, b, _ptr(Xc)[0], n, _ptr(Y)[0], n, 0))
        return Y

    def laplacian_matvec_into(self, layer, op, Xc, Yc, sync=True, wait=True):
        """Device-only form: Xc, Yc are b x n contiguous CUDA tensors, i.e. the
        column-major n x b blocks the C ABI takes; no copies are made.  sync:
        wait for torch's pending work first; wait=False: enqueue only
        (MLG_ASYNC), Yc is ready after synchronize()."""
        b, n = Xc.shape
        if sync:
            _sync()
        flags = MLG_DEVICE_PTRS | (0 if wait else MLG_ASYNC)
        _check(_lib.mlg_laplacian_matvec(self._h, layer, op, b, _ptr(Xc)[0], n, _ptr(Yc)[0], n,
                                         flags))
        return Yc

    def synchronize(self):
        """Wait for the products enqueued with wait=False (mlg_graph_synchronize)."""
        _check(_lib.mlg_graph_synchronize(self._h))

    def profile_stages(self, layer, op, X, reps=5, return_y=False):
        """Average ms per matvec in each stage (dict), device tensors only;
        with return_y, also the product (n x b), computed without the HIP
        graph and with the layers one after another."""
        import torch
        Xc, n, b = _colmajor(X)
        Y = torch.empty((b, n), dtype=torch.float64, device=Xc.device)
        ms = (ctypes.c_double * 8)()
        _sync()
        _check(_lib.mlg_profile_stages(self._h, layer, op, b, _ptr(Xc)[0], n, _ptr(Y)[0], n, reps,
                                       ms, MLG_DEVICE_PTRS))
        st = dict(zip(STAGES, list(ms)))
        return (st, Y.t()) if return_y else st

    def lanczos_eigs(self, layer, k, block=4, tol=1e-10, max_restarts=200, seed=0, p=1.0,
                     V0=None, device=False, inner_tol=0.0, inner_steps=0):
        """k smallest eigenpairs (lambda ascending, n x k vectors, info dict);
        p = 1 (L_sym / L_1) or p < 0 (L_{p,delta} through the Krylov power)."""
        info = EigInfo()
        pk = ctypes.byref(PksmParams(inner_tol, inner_steps))
        if device:
            import torch
            ev = torch.empty(k, dtype=torch.float64, device="cuda")
            V = torch.empty((k, self.n), dtype=torch.float64, device="cuda")
            v0p = None
            if V0 is not None:
                V0c, _, _ = _colmajor(V0)
                v0p = _ptr(V0c)[0]
            _sync()
            rc = _lib.mlg_lanczos_eigs(self._h, layer, p, k, block, tol, max_restarts, seed, v0p,
                                       _ptr(ev)[0], _ptr(V)[0], self.n, ctypes.byref(info), pk,
                                       MLG_DEVICE_PTRS)
            _check(rc, allow_warn=True)
            evals, evecs = ev, V.t()
        else:
            evals = np.empty(k)
            evecs = np.zeros((self.n, k), order="F")
            v0p = None
            if V0 is not None:
                V0c, _, _ = _colmajor(V0)
                self._v0 = V0c
                v0p = _ptr(V0c)[0]
            rc = _lib.mlg_lanczos_eigs(self._h, layer, p, k, block, tol, max_restarts, seed, v0p,
                                       _ptr(evals)[0], _ptr(evecs)[0], self.n, ctypes.byref(info),
                                       pk, 0)
            _check(rc, allow_warn=True)
        return evals, evecs, dict(iters=info.iters, restarts=info.restarts, matvecs=info.matvecs,
                                  nconv=info.nconv, max_resid=info.max_resid,
                                  inner_steps=info.inner_steps,
                                  inner_unconverged=info.inner_unconverged,
                                  converged=(rc == MLG_OK))

    def power_mean_matvec(self, layer, p, X, tol=0.0, max_steps=0):
        """Y = (L_sym^(t) + delta I)^p X (layer t) or the layer mean of these
        terms (layer -1), p < 0 (mlg_power_mean_matvec).  Returns (Y, info)
        with info = dict(steps, converged)."""
        Xc, n, b = _colmajor(X)
        pk = ctypes.byref(PksmParams(tol, max_steps))
        steps = ctypes.c_int(0)
        if _is_torch(Xc):
            import torch
            Y = torch.empty((b, n), dtype=torch.float64, device=Xc.device)
            _sync()
            rc = _lib.mlg_power_mean_matvec(self._h, layer, p, b, _ptr(Xc)[0], n, _ptr(Y)[0], n,
                                            pk, ctypes.byref(steps), MLG_DEVICE_PTRS)
            Y = Y.t()
        else:
            Y = np.zeros((n, b), order="F")
            rc = _lib.mlg_power_mean_matvec(self._h, layer, p, b, _ptr(Xc)[0], n, _ptr(Y)[0], n,
                                            pk, ctypes.byref(steps), 0)
        _check(rc, allow_warn=True)
        return Y, dict(steps=steps.value, converged=(rc == MLG_OK))


def kernel_matvec(points, sigma, X, params=None):
    """Y = W X (zero diagonal) for one point set (mlg_kernel_matvec)."""
    if params is None:
        params = kparams()
    Xc, n, b = _colmajor(X)
    if _is_torch(Xc):
        import torch
        pts = points.contiguous()
        Y = torch.empty((b, n), dtype=torch.float64, device=Xc.device)
        _sync()
        _check(_lib.mlg_kernel_matvec(n, pts.shape[1], _ptr(pts)[0], float(sigma),
                                      ctypes.byref(params), b, _ptr(Xc)[0], n, _ptr(Y)[0], n,
                                      MLG_DEVICE_PTRS, None))
        return Y.t()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    Y = np.zeros((n, b), order="F")
    _check(_lib.mlg_kernel_matvec(n, pts.shape[1], _ptr(pts)[0], float(sigma),
                                  ctypes.byref(params), b, _ptr(Xc)[0], n, _ptr(Y)[0], n, 0, None))
    return Y


def kernel_matvec_noalloc(points, sigma, X, Y, params, stream=None):
    """Enqueue Y = W X (direct summation, zero diagonal) without any device
    allocation (mlg_kernel_matvec_noalloc).  points: n x d torch CUDA tensor
    (row-major, contiguous); X, Y: n x b column-major device blocks given as
    b x n contiguous torch tensors (Y is written).  Returns without waiting:
    Y is ready once `stream` (default: the current torch stream) reaches the
    call."""
    import torch
    assert points.is_cuda and points.is_contiguous() and X.is_contiguous() and Y.is_contiguous()
    b, n = X.shape
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.mlg_kernel_matvec_noalloc(n, points.shape[1], _ptr(points)[0], float(sigma),
                                          ctypes.byref(params), b, _ptr(X)[0], n, _ptr(Y)[0], n,
                                          ctypes.c_void_p(stream)))


def allen_cahn_ssl(evals, evecs, labels, m, eps=5e-3, omega0=1000.0, c=None, dt=0.01, tol=1e-6,
                   max_iter=300):
    """Algorithm 2 steps 2-4 on given eigenpairs: returns (U, pred, iters)."""
    if c is None:
        c = omega0 + 3.0 / eps
    prm = ACParams(eps, omega0, c, dt, tol, max_iter)
    it = ctypes.c_int(0)
    if _is_torch(evecs):
        import torch
        Ec, n, k = _colmajor(evecs)
        ev = evals.contiguous().to(torch.float64)
        lab = labels.contiguous().to(torch.int32)
        U = torch.empty((n, m), dtype=torch.float64, device=Ec.device)
        pred = torch.empty(n, dtype=torch.int32, device=Ec.device)
        _sync()
        _check(_lib.mlg_allen_cahn_ssl(n, k, m, _ptr(ev)[0], _ptr(Ec)[0], n, _ptr(lab)[0],
                                       ctypes.byref(prm), _ptr(U)[0], _ptr(pred)[0],
                                       ctypes.byref(it), MLG_DEVICE_PTRS, None))
        return U, pred, it.value
    Ec, n, k = _colmajor(evecs)
    ev = np.ascontiguousarray(evals, dtype=np.float64)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    U = np.empty((n, m))
    pred = np.empty(n, dtype=np.int32)
    _check(_lib.mlg_allen_cahn_ssl(n, k, m, _ptr(ev)[0], _ptr(Ec)[0], n, _ptr(lab)[0],
                                   ctypes.byref(prm), _ptr(U)[0], _ptr(pred)[0], ctypes.byref(it),
                                   0, None))
    return U, pred, it.value
