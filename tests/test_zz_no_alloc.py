"""The allocation-free direct product (mlg_kernel_matvec_noalloc) against the
allocating entry point (mlg_kernel_matvec, direct method) through the C ABI:
two calls in a row on one stream, the second with a smaller input, both
compared bit for bit with the allocating call and with the FP64 oracle at the
parity gates (1e-12 FP64, 1e-5 FP32 direct tiles).  Argument and size-limit
errors come back before any device work."""
import ctypes

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


def _case(n, d, b, seed):
    pts = gen.gaussian_mixture(n, d, 4, 0.08, seed)[0]
    X = gen.test_vectors(n, b, seed + 1)
    return pts, X


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec,gate,kernel", [(64, 1e-12, "gaussian"), (32, 1e-5, "gaussian"),
                                              (64, 1e-12, "laplacian")])
def test_noalloc_matches_allocating_entry(mlg, prec, gate, kernel):
    import torch
    sigma = 0.15
    kp = mlg.kparams("direct", precision=prec, kernel=kernel)
    cases = [(5000, 3, 16, 71), (3001, 2, 5, 81)]   # second call smaller
    host, outs = [], []
    for n, d, b, seed in cases:
        pts, X = _case(n, d, b, seed)
        host.append((pts, X))
        print("noalloc FP%d %s n=%d d=%d b=%d" % (prec, kernel, n, d, b), flush=True)
        P = _dev(pts)
        Xt = _dev(X.T)                          # b x n row-major = n x b column-major
        Yt = torch.full((b, n), float("nan"), dtype=torch.float64, device="cuda")
        mlg.kernel_matvec_noalloc(P, sigma, Xt, Yt, kp)
        outs.append((P, Xt, Yt))
    torch.cuda.synchronize()
    for (pts, X), (P, Xt, Yt) in zip(host, outs):
        Y = Yt.cpu().numpy().T
        ref_lib = mlg.kernel_matvec(pts, sigma, X, kp)
        assert np.array_equal(Y, ref_lib)
        ref = oracle.kernel_matvec(pts, sigma, X, kernel)
        err = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= gate, err


def test_noalloc_argument_errors(mlg):
    import torch
    lib = mlg.lib()
    n, b = 4096, 16
    P = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    X = torch.zeros((b, n), dtype=torch.float64, device="cuda")
    Y = torch.zeros((b, n), dtype=torch.float64, device="cuda")
    kd = mlg.kparams("direct", precision=64)
    kn = mlg.kparams("nfft", precision=32)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    # the NFFT method allocates plans: not offered here
    assert lib.mlg_kernel_matvec_noalloc(n, 3, ptr(P), 0.1, ctypes.byref(kn), b, ptr(X), n,
                                         ptr(Y), n, None) == mlg.MLG_ERR_NOT_IMPL
    assert lib.mlg_kernel_matvec_noalloc(n, 3, ptr(P), 0.0, ctypes.byref(kd), b, ptr(X), n,
                                         ptr(Y), n, None) == mlg.MLG_ERR_RANGE
    assert lib.mlg_kernel_matvec_noalloc(n, 3, ptr(P), 0.1, ctypes.byref(kd), b, ptr(X), n - 1,
                                         ptr(Y), n, None) == mlg.MLG_ERR_ARG
    assert lib.mlg_kernel_matvec_noalloc(n, 3, None, 0.1, ctypes.byref(kd), b, ptr(X), n,
                                         ptr(Y), n, None) == mlg.MLG_ERR_ARG
    # beyond the scratch limit: rejected with a message, nothing enqueued
    big = 1 << 22
    assert lib.mlg_kernel_matvec_noalloc(big, 3, ptr(P), 0.1, ctypes.byref(kd), 64, ptr(X), big,
                                         ptr(Y), big, None) == mlg.MLG_ERR_RANGE
    assert b"scratch" in lib.mlg_last_error()
