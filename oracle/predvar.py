"""Oracle: damped curvature query (Laplace-style predictive variance).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper motivates the inverse Hessian for uncertainty quantification (Sec. 1)
and gives the full-rank form Q Lam Q^T + lam~ (I - Q Q^T) with its derivation
(Sec. 4.2, Appendix A.2), but defines no query vector.  Reading used here: for a
query x_q and class c the query vector is the logit gradient
g_q = d z^(L)_c(x_q) / d omega, and the query returns

    s_q = g_q^T (Q^T diag(lam) Q + delta I)^{-1} g_q
        = sum_k (q_k . g_q)^2 / (lam_k + delta) + (|g_q|^2 - sum_k (q_k . g_q)^2) / delta,

the second line following from the orthonormality argument of Appendix A.2
(the complement of span(Q) carries eigenvalue delta).  c defaults to the arg-max
of the prediction (lowest index on ties).
"""
from __future__ import annotations

import numpy as np

from . import mlp


def default_classes(model: mlp.Model, Xq) -> np.ndarray:
    z = mlp.logits_forward(model, Xq)
    return np.argmax(z, axis=1)  # lowest index on ties


def logit_grad(model: mlp.Model, Xq, cls) -> np.ndarray:
    """Rows g_q = gradient of Z^(L)[q, cls_q] with respect to omega (nq x P).

    Backpropagation exactly as for C_n but seeded with the unit vector e_c at the
    output pre-activation instead of Yhat - y.
    """
    L = model.L
    Z, A = mlp.forward(model, Xq)
    nq = Xq.shape[0]
    delta = [None] * (L + 1)
    delta[L] = np.zeros((nq, model.T[-1]))
    delta[L][np.arange(nq), np.asarray(cls)] = 1.0
    for l in range(L - 1, 1, -1):
        delta[l] = mlp.sigma_d1(model.acts[l - 2], Z[l]) * (delta[l + 1] @ model.W[l - 1])
    return np.concatenate([mlp.khatri_rao_rows(delta[l], A[l - 1]) for l in range(2, L + 1)], axis=1)


def predvar_identity(lam, Q, delta: float, G) -> np.ndarray:
    """s_q from the projection identity (any P)."""
    lam = np.asarray(lam, dtype=np.float64)
    proj = np.asarray(G, dtype=np.float64) @ np.asarray(Q, dtype=np.float64).T   # nq x K
    g2 = np.sum(np.asarray(G, dtype=np.float64) ** 2, axis=1)
    p2 = proj ** 2
    return np.sum(p2 / (lam[None, :] + delta), axis=1) + (g2 - np.sum(p2, axis=1)) / delta


def predvar_dense(lam, Q, delta: float, G) -> np.ndarray:
    """s_q = g^T (Q^T diag(lam) Q + delta I)^{-1} g by a dense solve (small P only)."""
    Q = np.asarray(Q, dtype=np.float64)
    P = Q.shape[1]
    M = Q.T @ (np.asarray(lam)[:, None] * Q) + delta * np.eye(P)
    G = np.asarray(G, dtype=np.float64)
    S = np.linalg.solve(M, G.T)
    return np.sum(G.T * S, axis=0)
