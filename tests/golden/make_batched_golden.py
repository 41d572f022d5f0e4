"""Write the FP64 oracle references of the batched-network verification subset.

The subset is 16 networks of the 256-network distribution (workloads.batched_model):
the 4 smallest and the 4 largest by P, and 8 others drawn with a fixed seed.  For each
network and each of two 64-column blocks of H and of the OPG (a seeded block, and the
last 64 columns, which end with the output biases) it stores

  * the 64 x 64 diagonal block M[cols, cols] (every entry), and
  * a 32-row Gaussian sketch S M[:, cols] of the whole column block, with
    S = sketch_matrix(P, seed) (rows drawn from numpy PCG64).

A device result R[:, cols] is then compared through S R[:, cols]: any error of
significant Frobenius norm in the block, wherever it sits, moves the sketch.

Only oracle/ computes (H columns by basis Hessian-vector products, OPG columns from
J; Sec. 3 and 5.1).  Run from the repository root:
    python tests/golden/make_batched_golden.py
It takes about half an hour on 8 cores (the largest networks dominate).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import mlp  # noqa: E402
from paper_1905_05559_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "batched_cfg4_subset.npz")
NMODELS = 256
BLOCK = 64
SKETCH_ROWS = 32


def widths_of(m: int):
    """P of batch model m without drawing its data (same draws as batched_model)."""
    w = workloads.batched_model(m)
    return w.P


def subset():
    Ps = sorted((widths_of(m), m) for m in range(NMODELS))
    small = [m for _, m in Ps[:4]]
    large = [m for _, m in Ps[-4:]]
    rest = [m for _, m in Ps[4:-4]]
    rng = np.random.Generator(np.random.PCG64(2024))
    others = sorted(int(x) for x in rng.choice(rest, size=8, replace=False))
    return small + others + large


def blocks_of(m: int, P: int):
    rng = np.random.Generator(np.random.PCG64(7000 + m))
    c0 = int(rng.integers(0, P - 2 * BLOCK))
    return [(c0, c0 + BLOCK), (P - BLOCK, P)]


def sketch_matrix(P: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((SKETCH_ROWS, P))


def main():
    models = subset()
    out = {"models": np.array(models, dtype=np.int64)}
    t_all = time.time()
    for m in models:
        t0 = time.time()
        w = workloads.batched_model(m)
        om = mlp.model_from(w.T, w.acts, w.W, w.b)
        X, Y = w.X.astype(np.float64), w.Y.astype(np.float64)
        S = sketch_matrix(w.P, 9000 + m)
        for bi, (c0, c1) in enumerate(blocks_of(m, w.P)):
            Hc = mlp.hessian_cols(om, X, Y, c0, c1, block=BLOCK)
            Gc = mlp.opg_cols(om, X, Y, list(range(c0, c1)))
            key = "m%d_b%d" % (m, bi)
            out[key + "_cols"] = np.array([c0, c1], dtype=np.int64)
            out[key + "_H_diag"] = Hc[c0:c1, :]
            out[key + "_G_diag"] = Gc[c0:c1, :]
            out[key + "_H_sketch"] = S @ Hc
            out[key + "_G_sketch"] = S @ Gc
        print("model %d T=%s N=%d P=%d: %.1f s" % (m, w.T, w.N, w.P, time.time() - t0), flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote %s (%.1f s)" % (OUT, time.time() - t_all))


if __name__ == "__main__":
    main()
