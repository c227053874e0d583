"""Write the stored expected values of the full-size parity checks.

Every number written here comes from the CPU oracle (``oracle/``) on the
seeded synthetic workloads of ``workloads/gen.py``; nothing is taken from the
GPU library.  Run once on the host (hours of CPU time: the oracle is the
plain O(n^2) direct sum); the tests and the benchmark only read the results.

  ball_eigs      the 20 smallest eigenvalues of L_sym of the 10^5-point ball
                 (sigma 0.05): ARPACK (scipy eigsh, tol 1e-12) driving the
                 oracle's direct sum, lambda = 1 - mu (Sec. 3; Algorithm 2
                 step 1).  -> ball_n100000_eigs.json
  image_rows     4096 sampled rows of L_1 X for the 1000 x 1000 image graph
                 (three layers, b = 16 seeded N(0,1) vectors), every layer's
                 degrees over all 10^6 nodes from the oracle (Sec. 2 degree
                 and L_sym; Sec. 3 eq. for I - L_1).
                 -> image1000_L1_rows4096_b16.npz

Usage:  python tests/golden/make_golden.py {ball_eigs|image_rows} [--cache DIR]
The optional cache keeps each layer's oracle degrees between runs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import gen  # noqa: E402

# row sample and test block of the image rows (shared with the readers)
IMAGE_ROWS = 4096
IMAGE_B = 16
IMAGE_ROW_SEED_OFFSET = 500
IMAGE_X_SEED_OFFSET = 300


def image_sample(n, base_seed):
    """Sorted distinct row indices of the stored image rows."""
    return np.sort(gen.rng(base_seed + IMAGE_ROW_SEED_OFFSET).choice(n, size=IMAGE_ROWS,
                                                                    replace=False))


def _layer(points, sigma, cache, tag):
    """oracle.Layer with its degrees, optionally kept in `cache`."""
    path = None if cache is None else os.path.join(cache, "deg_%s.npy" % tag)
    if path is not None and os.path.exists(path):
        L = oracle.Layer.__new__(oracle.Layer)
        L.points = np.ascontiguousarray(points, dtype=np.float64)
        L.sigma = float(sigma)
        L.kernel = "gaussian"
        L.deg = np.load(path)
        if np.any(L.deg <= 0.0):
            raise ValueError("isolated node in cached degrees")
        L.dinv_sqrt = 1.0 / np.sqrt(L.deg)
        return L
    t0 = time.time()
    L = oracle.Layer(points, sigma)
    print("  degrees of %s: %.0f s" % (tag, time.time() - t0), flush=True)
    if path is not None:
        os.makedirs(cache, exist_ok=True)
        np.save(path, L.deg)
    return L


def ball_eigs(cache):
    c = gen.config2()
    k = c["k"]
    t0 = time.time()
    L = _layer(c["layers"][0], c["sigma"][0], cache, "ball_n%d" % c["n"])
    lam, _ = oracle.eigs_iterative([L], k, tol=1e-12, seed=c["base_seed"] + 600)
    out = {
        "_about": "20 smallest eigenvalues of L_sym, 1e5 points uniform in a 3-D ball of "
                  "radius 0.25, sigma 0.05 (workloads.gen.config2). Written by "
                  "tests/golden/make_golden.py from the CPU oracle only: ARPACK (eigsh, "
                  "which='LA', tol 1e-12) on D^-1/2 W D^-1/2 through the FP64 direct sum; "
                  "lambda = 1 - mu (Sec. 3; Algorithm 2 step 1).",
        "n": c["n"], "sigma": c["sigma"][0], "k": k,
        "eigenvalues": [float(v) for v in lam],
        "cpu_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(HERE, "ball_n%d_eigs.json" % c["n"])
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


def image_rows(cache):
    c = gen.config3()
    n = c["n"]
    t0 = time.time()
    layers = [_layer(P, s, cache, "image%d_layer%d" % (n, t))
              for t, (P, s) in enumerate(zip(c["layers"], c["sigma"]))]
    rows = image_sample(n, c["base_seed"])
    X = gen.test_vectors(n, IMAGE_B, c["base_seed"] + IMAGE_X_SEED_OFFSET)
    Y = oracle.lsym_matvec(layers, X, rows)
    path = os.path.join(HERE, "image%d_L1_rows%d_b%d.npz" % (int(round(n ** 0.5)), IMAGE_ROWS,
                                                            IMAGE_B))
    np.savez(path, rows=rows.astype(np.int64), L1X=np.ascontiguousarray(Y),
             dinv_sqrt_rows=np.stack([L.dinv_sqrt[rows] for L in layers], axis=1),
             sigma=np.asarray(c["sigma"]))
    print("wrote %s (%.0f s)" % (path, time.time() - t0), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["ball_eigs", "image_rows"])
    ap.add_argument("--cache", default=None)
    a = ap.parse_args()
    {"ball_eigs": ball_eigs, "image_rows": image_rows}[a.what](a.cache)


if __name__ == "__main__":
    main()
