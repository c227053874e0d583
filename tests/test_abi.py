"""The C-ABI library loads and exports every function include/mlg.h declares;
argument checks that fail before any device work return their status codes.
No compute call is made here (CPU-only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlg.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlg_[a-z_]+)\s*\(", txt)))


def test_header_declares_boundary_calls():
    names = declared_functions()
    for need in ["mlg_kernel_matvec", "mlg_laplacian_matvec", "mlg_lanczos_eigs",
                 "mlg_allen_cahn_ssl", "mlg_graph_create", "mlg_graph_destroy"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2007_05239_amd.mlg as mlg
    out = subprocess.run(["nm", "-D", "--defined-only", mlg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mlg_[a-z_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert sorted(mlg.EXPORTED) == sorted(declared_functions())


def test_version_and_empty_error():
    import paper_2007_05239_amd.mlg as mlg
    assert "gfx950" in mlg.version()


def test_argument_errors_before_device_work():
    import paper_2007_05239_amd.mlg as mlg
    lib = mlg.lib()
    h = ctypes.c_void_p()
    # null output handle
    assert lib.mlg_graph_create(None, 10, 1, None, None, None, None, 0, None) == mlg.MLG_ERR_ARG
    d = (ctypes.c_int * 1)(3)
    pts = np.zeros((10, 3))
    parr = (ctypes.c_void_p * 1)(pts.ctypes.data)
    sig = (ctypes.c_double * 1)(0.5)
    kp = (mlg.KParams * 1)(mlg.kparams())
    # n < 2
    assert lib.mlg_graph_create(ctypes.byref(h), 1, 1, d, parr, sig, kp, 0, None) == mlg.MLG_ERR_ARG
    # sigma <= 0
    sig0 = (ctypes.c_double * 1)(0.0)
    assert lib.mlg_graph_create(ctypes.byref(h), 10, 1, d, parr, sig0, kp, 0, None) == mlg.MLG_ERR_RANGE
    # NFFT with d = 4
    d4 = (ctypes.c_int * 1)(4)
    assert lib.mlg_graph_create(ctypes.byref(h), 10, 1, d4, parr, sig, kp, 0, None) == mlg.MLG_ERR_RANGE
    # bad precision
    kbad = (mlg.KParams * 1)(mlg.kparams(precision=16))
    assert lib.mlg_graph_create(ctypes.byref(h), 10, 1, d, parr, sig, kbad, 0, None) == mlg.MLG_ERR_ARG
    assert "precision" in lib.mlg_last_error().decode()
    # Allen--Cahn argument checks
    prm = mlg.ACParams(5e-3, 1000.0, 1600.0, 0.01, 1e-6, 300)
    it = ctypes.c_int()
    assert lib.mlg_allen_cahn_ssl(10, 2, 1, None, None, 10, None, ctypes.byref(prm), None, None,
                                  ctypes.byref(it), 0, None) == mlg.MLG_ERR_ARG
    # null graph
    assert lib.mlg_laplacian_matvec(None, 0, 0, 1, None, 1, None, 1, 0) == mlg.MLG_ERR_ARG
    # autotuner: null outputs, bad precision, tolerance, sample size and dimension
    kpo, tio = mlg.KParams(), mlg.TuneInfo()
    at = lib.mlg_autotune_layer
    assert at(10, 3, pts.ctypes.data, 0.5, 32, 4, 1e-4, 4, 0, 0, None, None, ctypes.byref(tio)) == mlg.MLG_ERR_ARG
    assert at(10, 3, pts.ctypes.data, 0.5, 16, 4, 1e-4, 4, 0, 0, None, ctypes.byref(kpo), ctypes.byref(tio)) == mlg.MLG_ERR_ARG
    assert at(10, 3, pts.ctypes.data, 0.5, 32, 4, 0.0, 4, 0, 0, None, ctypes.byref(kpo), ctypes.byref(tio)) == mlg.MLG_ERR_ARG
    assert at(10, 3, pts.ctypes.data, 0.5, 32, 4, 1e-4, 11, 0, 0, None, ctypes.byref(kpo), ctypes.byref(tio)) == mlg.MLG_ERR_ARG
    assert at(10, 4, pts.ctypes.data, 0.5, 32, 4, 1e-4, 4, 0, 0, None, ctypes.byref(kpo), ctypes.byref(tio)) == mlg.MLG_ERR_RANGE
    assert at(10, 3, pts.ctypes.data, -1.0, 32, 4, 1e-4, 4, 0, 0, None, ctypes.byref(kpo), ctypes.byref(tio)) == mlg.MLG_ERR_RANGE
    assert lib.mlg_graph_destroy(None) == mlg.MLG_OK


def test_stride_groups():
    import paper_2007_05239_amd.mlg as mlg
    g2 = mlg.stride_groups(102, 2)
    assert len(g2) == 51 and g2[0] == (0, 51) and g2[-1] == (50, 101)
    g3 = mlg.stride_groups(102, 3)
    assert len(g3) == 34 and g3[0] == (0, 34, 68) and g3[-1] == (33, 67, 101)
    g = mlg.stride_groups(7, 3)
    assert g == [(0, 2, 4), (1, 3, 5), (6,)]
    assert sorted(c for grp in mlg.stride_groups(13, 2) for c in grp) == list(range(13))
