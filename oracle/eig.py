"""Oracle: leading eigenpairs of H or of the OPG -- TEST INFRASTRUCTURE ONLY.

"Top-K" means the K algebraically largest eigenvalues, sorted descending
(Sec. 4.1 assumes lambda_1 >= ... >= lambda_K; Sec. 5.3 asks the Lanczos solver for
which='LA' and sorts descending).  Eigenvectors are unique only up to sign, so
every eigenvector is normalised so that its largest-magnitude component is
positive (lowest index on ties).
"""
from __future__ import annotations

import numpy as np


def sign_normalize(Q: np.ndarray) -> np.ndarray:
    """Rows of Q (K x P): flip each row so its largest-|.| entry is positive."""
    Q = np.array(Q, dtype=np.float64, copy=True)
    for k in range(Q.shape[0]):
        idx = int(np.argmax(np.abs(Q[k])))  # argmax returns the lowest index on ties
        if Q[k, idx] < 0:
            Q[k] = -Q[k]
    return Q


def topk_eigh(M: np.ndarray, K: int):
    """K algebraically largest eigenpairs of a symmetric matrix via LAPACK (dense).

    Returns (lam (K,) descending, Q (K x P) rows = eigenvectors).
    """
    w, V = np.linalg.eigh(np.asarray(M, dtype=np.float64))
    order = np.argsort(w)[::-1][:K]
    return w[order].copy(), sign_normalize(V[:, order].T)


def topk_lanczos(matvec, P: int, K: int, tol: float = 0.0):
    """The paper's own procedure (Sec. 5.3): ARPACK Lanczos on a matrix-free operator."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    op = LinearOperator((P, P), matvec=lambda v: matvec(np.ravel(v)), dtype=np.float64)
    w, V = eigsh(op, k=K, which="LA", tol=tol)
    order = np.argsort(w)[::-1]
    return w[order].copy(), sign_normalize(V[:, order].T)


def residuals(M_apply, lam: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """||M q_k - lam_k q_k||_2 for each row q_k of Q; M_apply maps (P x K) -> (P x K)."""
    R = M_apply(Q.T) - Q.T * lam[None, :]
    return np.linalg.norm(R, axis=0)


def low_rank_quadratic(lam, Q, x):
    """x^T (Q^T diag(lam) Q) x without forming the P x P matrix (Sec. 5.5)."""
    p = Q @ x
    return float(p @ (lam * p))


def low_rank_apply(lam, Q, x):
    """H~ x = Q^T diag(lam) (Q x) without forming the P x P matrix (Sec. 5.5)."""
    return Q.T @ (lam * (Q @ x))


def full_rank_apply(lam, Q, x, lam_tilde=None):
    """H~~ x = Q^T diag(lam) Q x + lam~ (x - Q^T Q x), lam~ = lam_K by default (Sec. 5.6)."""
    lt = lam[-1] if lam_tilde is None else lam_tilde
    p = Q @ x
    return Q.T @ (lam * p) + lt * (x - Q.T @ p)


def full_rank_inverse_apply(lam, Q, x, lam_tilde=None):
    """H~~^{-1} x.  H~~ has eigenvalues lam_k on the rows of Q and lam~ on their orthogonal
    complement (App. A.2), so its inverse replaces them by 1/lam_k and 1/lam~."""
    lt = lam[-1] if lam_tilde is None else lam_tilde
    p = Q @ x
    return Q.T @ (p / lam) + (x - Q.T @ p) / lt


def full_rank_quadratic(lam, Q, x, lam_tilde=None):
    """x^T [Q^T diag(lam) Q + lam~ (I - Q^T Q)] x with lam~ = lam_K by default (Sec. 5.6)."""
    lt = lam[-1] if lam_tilde is None else lam_tilde
    p = Q @ x
    return float(p @ (lam * p) + lt * (x @ x) - lt * (p @ p))
