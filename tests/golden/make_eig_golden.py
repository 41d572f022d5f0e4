"""Write the FP64 oracle eigenvalue references of the two larger workloads.

* sigmoid-64 ([64, 64, 10] sigmoid, N = 10000, P = 4810): H by basis
  Hessian-vector products and OPG = J^T J / N (Sec. 3, 5.1), then LAPACK eigh.
  Stored: the 101 algebraically largest eigenvalues of each (descending), the
  Frobenius norms, and the unit eigenvectors of the 8 largest (largest-|.|
  component positive).
* MNIST-shaped ([784, 100, 10] ReLU, N = 60000, P = 79510): the paper's own
  procedure (Sec. 5.3): ARPACK Lanczos (which='LA') on the matrix-free oracle
  Hessian-vector product.  Stored: the 101 largest eigenvalues, descending.

Only oracle/ computes.  Run from the repository root:
    python tests/golden/make_eig_golden.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import eig, mlp  # noqa: E402
from paper_1905_05559_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "eig_sigmoid64_mnist.npz")
KEEP = 101
NVEC = 8


def sigmoid64(out):
    w = workloads.sigmoid_64()
    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    X, Y = w.X.astype(np.float64), w.Y.astype(np.float64)
    t = time.time()
    H = mlp.hessian(om, X, Y, block=128)
    G = mlp.opg(om, X, Y)
    print("sigmoid-64 H and OPG formed: %.1f s" % (time.time() - t), flush=True)
    for tag, M in (("H", H), ("G", G)):
        Ms = 0.5 * (M + M.T)
        lam, Q = eig.topk_eigh(Ms, KEEP)
        out["sig_%s_lam" % tag] = lam
        out["sig_%s_fro" % tag] = np.array(np.linalg.norm(Ms))
        out["sig_%s_Q%d" % (tag, NVEC)] = Q[:NVEC]
        print("sigmoid-64 %s: lambda_1 %.6e, lambda_100 %.6e, ||M||_F %.6e" % (tag, lam[0], lam[99],
                                                                            np.linalg.norm(Ms)), flush=True)


def mnist(out):
    w = workloads.mnist_relu()
    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    X, Y = w.X.astype(np.float64), w.Y.astype(np.float64)
    t = time.time()
    count = [0]

    def matvec(v):
        count[0] += 1
        return mlp.hvp(om, X, Y, v[None, :])[0]

    lam, _ = eig.topk_lanczos(matvec, w.P, KEEP, tol=1e-10)
    out["mnist_H_lam"] = lam
    print("MNIST-shaped H: %d oracle HVPs, %.1f s; lambda_1 %.6e, lambda_100 %.6e"
          % (count[0], time.time() - t, lam[0], lam[99]), flush=True)


def main():
    out = {}
    sigmoid64(out)
    mnist(out)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
