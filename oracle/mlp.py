"""Oracle: MLP cost, per-example gradients, OPG and exact Hessian (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation (Sec. 2 of the paper): layers l = 1..L with widths T_l; W^(l-1) is
T_l x T_{l-1}, b^(l) has T_l entries; A^(1) = X; Z^(l) = A^(l-1) W^(l-1)^T + b^(l);
A^(l) = sigma^(l)(Z^(l)) for hidden layers and Yhat = softmax(Z^(L)).  The cost is
the mean over N examples of the per-example cross-entropy C_n (Sec. 2, the cost
definition).  omega is the flat parameter vector of the flatten definition in
Sec. 2: W^(1) row-major, then b^(2), then W^(2), b^(3), ...

All arrays are float64 unless the caller passes complex values (the
complex-step pin uses the same code path with a complex omega).

Readings of the paper (see the list in the design notes):
  * J is N x P with row n equal to the gradient of C_n (no 1/N factor); the OPG
    is J^T J / N (Sec. 3, OPG definition and its Jacobian form).
  * H and the OPG are exact full-N means; the paper's mini-batch loops drop the
    remainder when N is not a multiple of the batch size, here nothing is dropped.
  * ReLU'(0) = 0 and ReLU'' = 0.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np


@dataclass
class Model:
    T: List[int]
    acts: List[str]             # hidden activations, layers 2..L-1
    W: List[np.ndarray]         # W[k] = W^(k+1): (T[k+1], T[k])
    b: List[np.ndarray]         # b[k] = b^(k+2): (T[k+1],)

    @property
    def L(self) -> int:
        return len(self.T)


def model_from(T, acts, W, b) -> Model:
    """Promote stored arrays to float64 (first step of the oracle)."""
    return Model(list(T), list(acts), [np.asarray(w, dtype=np.float64) for w in W],
                 [np.asarray(v, dtype=np.float64) for v in b])


# ---------------------------------------------------------------------------
# Flat parameter layout (Sec. 2, flatten definition).
# ---------------------------------------------------------------------------

def num_params(T: Sequence[int]) -> int:
    """P = T_1 T_2 + T_2 + ... + T_{L-1} T_L + T_L (Sec. 2)."""
    return int(sum(T[k] * T[k + 1] + T[k + 1] for k in range(len(T) - 1)))


def layer_offsets(T: Sequence[int]):
    """For k = 0..L-2 (weight W^(k+1), bias b^(k+2)): (offset of W, offset of b)."""
    offs, o = [], 0
    for k in range(len(T) - 1):
        offs.append((o, o + T[k + 1] * T[k]))
        o += T[k + 1] * T[k] + T[k + 1]
    return offs


def flatten(W: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> np.ndarray:
    """omega = flatten over l of (W^(l-1), b^(l)), each W row-wise."""
    parts = []
    for w, v in zip(W, b):
        parts.append(np.reshape(w, -1))
        parts.append(np.reshape(v, -1))
    return np.concatenate(parts)


def unflatten(omega: np.ndarray, T: Sequence[int]):
    """Inverse of flatten: lists of W^(l-1) (T_l x T_{l-1}) and b^(l)."""
    W, b = [], []
    for k, (ow, ob) in enumerate(layer_offsets(T)):
        W.append(np.reshape(omega[ow:ob], (T[k + 1], T[k])))
        b.append(omega[ob:ob + T[k + 1]])
    return W, b


def with_omega(model: Model, omega: np.ndarray) -> Model:
    W, b = unflatten(omega, model.T)
    return Model(model.T, model.acts, W, b)


# ---------------------------------------------------------------------------
# Activations and their first two derivatives.
# ---------------------------------------------------------------------------

def sigma(act: str, z):
    if act == "tanh":
        return np.tanh(z)
    if act == "sigmoid":
        return 1.0 / (1.0 + np.exp(-z))
    if act == "relu":
        return z * (np.real(z) > 0)
    raise ValueError(act)


def sigma_d1(act: str, z):
    if act == "tanh":
        t = np.tanh(z)
        return 1.0 - t * t
    if act == "sigmoid":
        s = 1.0 / (1.0 + np.exp(-z))
        return s * (1.0 - s)
    if act == "relu":
        return (np.real(z) > 0).astype(np.float64)
    raise ValueError(act)


def sigma_d2(act: str, z):
    if act == "tanh":
        t = np.tanh(z)
        return -2.0 * t * (1.0 - t * t)
    if act == "sigmoid":
        s = 1.0 / (1.0 + np.exp(-z))
        return s * (1.0 - s) * (1.0 - 2.0 * s)
    if act == "relu":
        return np.zeros(np.shape(z))
    raise ValueError(act)


def softmax_rows(z):
    """Row softmax exp(z - max) / sum (Sec. 2); the max uses the real part."""
    zmax = np.max(np.real(z), axis=1, keepdims=True)
    e = np.exp(z - zmax)
    return e / np.sum(e, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# Forward pass, cost, per-example backprop (Sec. 2 and Sec. 3).
# ---------------------------------------------------------------------------

def forward(model: Model, X):
    """Returns (Z, A) with Z[l] = Z^(l) and A[l] = A^(l) for l = 1..L (index 0, 1 unused).

    A[L] is the softmax output Yhat.  Model function of Sec. 2.
    """
    L = model.L
    Z = [None] * (L + 1)
    A = [None] * (L + 1)
    A[1] = X
    for l in range(2, L + 1):
        Z[l] = A[l - 1] @ model.W[l - 2].T + model.b[l - 2]
        A[l] = softmax_rows(Z[l]) if l == L else sigma(model.acts[l - 2], Z[l])
    return Z, A


def cost(model: Model, X, Y) -> float:
    """C = (1/N) sum_n -sum_m y_{n,m} log yhat_{n,m} (Sec. 2, cost definition)."""
    Z, _ = forward(model, X)
    zL = Z[model.L]
    zmax = np.max(zL, axis=1, keepdims=True)
    lse = zmax[:, 0] + np.log(np.sum(np.exp(zL - zmax), axis=1))
    return float(np.mean(lse - np.sum(Y * zL, axis=1)))


def backprop(model: Model, X, Y):
    """Per-example error signals delta^(l) = dC_n/dZ^(l) (rows n), l = 2..L.

    delta^(L) = Yhat - Y (softmax with cross-entropy), E^(l) = delta^(l+1) W^(l),
    delta^(l) = sigma'(Z^(l)) * E^(l).  Returns (Z, A, delta, E).
    """
    L = model.L
    Z, A = forward(model, X)
    delta = [None] * (L + 1)
    E = [None] * (L + 1)
    delta[L] = A[L] - Y
    for l in range(L - 1, 1, -1):
        E[l] = delta[l + 1] @ model.W[l - 1]
        delta[l] = sigma_d1(model.acts[l - 2], Z[l]) * E[l]
    return Z, A, delta, E


def khatri_rao_rows(delta_l, a_prev):
    """Per-example gradient block of one layer: rows [vec(delta_n a_n^T), delta_n].

    The gradient of C_n with respect to W^(l-1) is the outer product of delta^(l)_n
    and A^(l-1)_n, flattened row-wise; with respect to b^(l) it is delta^(l)_n.
    """
    N = delta_l.shape[0]
    outer = delta_l[:, :, None] * a_prev[:, None, :]
    return np.concatenate([outer.reshape(N, -1), delta_l], axis=1)


def jacobian(model: Model, X, Y):
    """J (N x P): row n is the flat gradient of C_n (Sec. 3, the matrix J)."""
    _, A, delta, _ = backprop(model, X, Y)
    return np.concatenate([khatri_rao_rows(delta[l], A[l - 1]) for l in range(2, model.L + 1)],
                          axis=1)


def gradient(model: Model, X, Y):
    """Gradient of C: the mean of the per-example gradients."""
    return np.mean(jacobian(model, X, Y), axis=0)


def opg(model: Model, X, Y):
    """OPG = (1/N) sum_n grad C_n grad C_n^T = J^T J / N (Sec. 3)."""
    J = jacobian(model, X, Y)
    return J.T @ J / J.shape[0]


def param_index(T, k: int, i: int, j: int) -> int:
    """Flat index of W^(k+1)[i, j] (j < T[k]) or of b^(k+2)[i] (j == T[k])."""
    ow, ob = layer_offsets(T)[k]
    return ow + i * T[k] + j if j < T[k] else ob + i


def jacobian_cols(model: Model, X, Y, cols: Sequence[int]):
    """Selected columns J[:, cols], each computed from delta and A alone."""
    _, A, delta, _ = backprop(model, X, Y)
    T = model.T
    offs = layer_offsets(T)
    out = np.empty((X.shape[0], len(cols)))
    for c, p in enumerate(cols):
        for k, (ow, ob) in enumerate(offs):
            if ow <= p < ob + T[k + 1]:
                l = k + 2
                if p < ob:
                    i, j = divmod(p - ow, T[k])
                    out[:, c] = delta[l][:, i] * A[l - 1][:, j]
                else:
                    out[:, c] = delta[l][:, p - ob]
                break
    return out


def opg_tile(model: Model, X, Y, rows: Sequence[int], cols: Sequence[int]):
    """OPG[rows, cols] = J[:, rows]^T J[:, cols] / N from those columns of J only."""
    Jr = jacobian_cols(model, X, Y, rows)
    Jc = jacobian_cols(model, X, Y, cols)
    return Jr.T @ Jc / X.shape[0]


def opg_cols(model: Model, X, Y, cols: Sequence[int]):
    """Columns OPG[:, cols] = J^T J[:, cols] / N without forming J (Sec. 3).

    For a weight vector v = J[:, c], J^T v is sum_n v_n grad C_n; its block for layer l
    is (delta^(l) * v)^T [A^(l-1), 1] (the per-example outer products of the gradient
    definition, summed).  Returns P x len(cols).
    """
    _, A, delta, _ = backprop(model, X, Y)
    Jc = jacobian_cols(model, X, Y, cols)
    N = X.shape[0]
    out = np.empty((num_params(model.T), len(cols)))
    for c in range(len(cols)):
        parts = []
        for l in range(2, model.L + 1):
            dv = delta[l] * Jc[:, c:c + 1]                   # rows v_n delta^(l)_n
            parts.append((dv.T @ A[l - 1]).reshape(-1))      # W^(l-1) block, row-major
            parts.append(dv.sum(axis=0))                     # b^(l) block
        out[:, c] = np.concatenate(parts)
    return out / N


# ---------------------------------------------------------------------------
# Hessian-vector products by the R-operator (Appendix A.1, Sec. 5.1).
# ---------------------------------------------------------------------------

def hvp(model: Model, X, Y, V):
    """H v for each row v of V (B x P): forward-over-reverse R-operator.

    The paper obtains Hv by differentiating (grad C) . v once more (Appendix A.1);
    the same quantity is the directional derivative of the gradient along v,
    computed here by propagating R{.} = d/dt (.)(omega + t v) at t = 0 through the
    forward pass and the per-example backward pass:
      R{Z^(l)} = R{A^(l-1)} W^(l-1)^T + A^(l-1) V_W^(l-1)^T + V_b^(l),  R{A^(1)} = 0
      R{A^(l)} = sigma'(Z^(l)) R{Z^(l)}
      R{Yhat}  = Yhat * (R{Z^(L)} - sum(Yhat * R{Z^(L)}))
      R{delta^(L)} = R{Yhat}
      R{delta^(l)} = sigma''(Z) R{Z} E^(l) + sigma'(Z) (R{delta^(l+1)} W^(l) + delta^(l+1) V_W^(l))
      (Hv)_{W^(l-1)} = (1/N) sum_n R{delta^(l)}_n A^(l-1)_n^T + delta^(l)_n R{A^(l-1)}_n^T
      (Hv)_{b^(l)}   = (1/N) sum_n R{delta^(l)}_n
    Returns HV with the same shape as V (rows are H v_b; H is symmetric so this
    also equals v_b^T H, the orientation of Appendix A.1).
    """
    V = np.atleast_2d(np.asarray(V, dtype=np.float64))
    Bn, P = V.shape
    T, L = model.T, model.L
    N = X.shape[0]
    Z, A, delta, E = backprop(model, X, Y)
    # unflatten each direction: VW[l] (B, T_l, T_{l-1}), Vb[l] (B, T_l)
    VW = [None] * (L + 1)
    Vb = [None] * (L + 1)
    for k, (ow, ob) in enumerate(layer_offsets(T)):
        l = k + 2
        VW[l] = V[:, ow:ob].reshape(Bn, T[l - 1], T[l - 2])
        Vb[l] = V[:, ob:ob + T[l - 1]]
    RZ = [None] * (L + 1)
    RA = [None] * (L + 1)      # R{A^(1)} = 0: the input does not depend on omega
    for l in range(2, L + 1):
        # R{Z^(l)}[n, b, :] for every example n and direction b
        RZ[l] = (np.einsum("bij,nj->nbi", VW[l], A[l - 1], optimize=True)
                 + Vb[l][None, :, :])
        if RA[l - 1] is not None:
            RZ[l] = RZ[l] + RA[l - 1] @ model.W[l - 2].T
        if l < L:
            RA[l] = sigma_d1(model.acts[l - 2], Z[l])[:, None, :] * RZ[l]
    yhat = A[L][:, None, :]
    RD = [None] * (L + 1)
    RD[L] = yhat * (RZ[L] - np.sum(yhat * RZ[L], axis=2, keepdims=True))
    for l in range(L - 1, 1, -1):
        act = model.acts[l - 2]
        RD[l] = (sigma_d2(act, Z[l])[:, None, :] * RZ[l] * E[l][:, None, :]
                 + sigma_d1(act, Z[l])[:, None, :]
                 * (RD[l + 1] @ model.W[l - 1]
                    + np.einsum("bij,ni->nbj", VW[l + 1], delta[l + 1], optimize=True)))
    out = np.empty((Bn, P))
    for k, (ow, ob) in enumerate(layer_offsets(T)):
        l = k + 2
        gW = np.einsum("nbi,nj->bij", RD[l], A[l - 1], optimize=True)
        if RA[l - 1] is not None:
            gW = gW + np.einsum("ni,nbj->bij", delta[l], RA[l - 1], optimize=True)
        gW = gW / N
        out[:, ow:ob] = gW.reshape(Bn, -1)
        out[:, ob:ob + T[l - 1]] = np.sum(RD[l], axis=0) / N
    return out


def hessian_cols(model: Model, X, Y, c0: int, c1: int, block: int = 64):
    """Columns c0..c1-1 of H: Hessian-vector products with basis vectors (Sec. 5.1).

    Columns are independent, so they are formed a few at a time.  Returns P x (c1-c0).
    """
    P = num_params(model.T)
    out = np.empty((P, c1 - c0))
    for s in range(c0, c1, block):
        e = min(c1, s + block)
        Vb = np.zeros((e - s, P))
        Vb[np.arange(e - s), np.arange(s, e)] = 1.0
        out[:, s - c0:e - c0] = hvp(model, X, Y, Vb).T
    return out


def hessian(model: Model, X, Y, block: int = 64):
    """Exact H (P x P), column by column from basis HVPs; NOT symmetrised."""
    P = num_params(model.T)
    return hessian_cols(model, X, Y, 0, P, block)


def logits_forward(model: Model, X):
    """Output pre-activations Z^(L) (used by the predictive-variance query)."""
    Z, _ = forward(model, X)
    return Z[model.L]
