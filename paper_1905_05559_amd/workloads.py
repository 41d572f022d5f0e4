"""Seeded synthetic workloads for the Hessian / OPG hot path.

This module only draws inputs: network widths, Glorot-uniform weights, zero
biases, inputs X and one-hot labels Y.  It holds none of the method's
arithmetic, so both the FP64 oracle and the device library can be fed from it
without sharing any computation.

Model structure follows Sec. 2 of the paper: widths T_1..T_L, weight matrices
W^(l-1) of shape T_l x T_{l-1} (row-major), bias vectors b^(l), hidden
activations sigma^(l) for l = 2..L-1 and a softmax output layer.  The cost is the
mean softmax cross-entropy over N examples with one-hot targets.

Draw order for one model (all from one numpy PCG64 generator):
  for l = 2..L:  W^(l-1) ~ U(-r, r), r = sqrt(6 / (T_{l-1} + T_l)), drawn as a
                 T_l x T_{l-1} row-major matrix;  b^(l) = 0
  then X (distribution per workload), then integer labels -> one-hot Y.
Values are drawn in float64 and cast once to the storage dtype.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

ACTS = ("tanh", "sigmoid", "relu")


@dataclass
class Workload:
    """One network plus one data set, all arrays on the host."""

    name: str
    T: List[int]                 # widths T_1..T_L
    acts: List[str]              # hidden activations for l = 2..L-1 (len L-2)
    W: List[np.ndarray]          # W[k] = W^(k+1), shape (T[k+1], T[k])
    b: List[np.ndarray]          # b[k] = b^(k+2), shape (T[k+1],)
    X: np.ndarray                # (N, T_1)
    Y: np.ndarray                # (N, T_L) one-hot
    labels: np.ndarray           # (N,) int64
    dtype: str = "float64"       # storage dtype of W, b, X, Y
    meta: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return len(self.T)

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def P(self) -> int:
        return int(sum(self.T[k + 1] * self.T[k] + self.T[k + 1] for k in range(self.L - 1)))


def _glorot(rng: np.random.Generator, fan_out: int, fan_in: int) -> np.ndarray:
    r = np.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-r, r, size=(fan_out, fan_in))


def _draw_params(rng, T):
    Ws, bs = [], []
    for k in range(len(T) - 1):
        Ws.append(_glorot(rng, T[k + 1], T[k]))
        bs.append(np.zeros(T[k + 1]))
    return Ws, bs


def _one_hot(labels: np.ndarray, C: int) -> np.ndarray:
    Y = np.zeros((labels.shape[0], C))
    Y[np.arange(labels.shape[0]), labels] = 1.0
    return Y


def _finish(name, T, acts, Ws, bs, X, labels, dtype, meta=None) -> Workload:
    Y = _one_hot(labels, T[-1])
    cast = lambda a: np.ascontiguousarray(a.astype(dtype))
    return Workload(name=name, T=list(map(int, T)), acts=list(acts),
                    W=[cast(w) for w in Ws], b=[cast(v) for v in bs],
                    X=cast(X), Y=cast(Y), labels=labels.astype(np.int64),
                    dtype=dtype, meta=meta or {})


def mlp_gaussian(T: Sequence[int], acts: Sequence[str], N: int, seed: int,
                 dtype: str = "float64", name: str = "custom") -> Workload:
    """Glorot weights, zero biases, x ~ N(0, 1), labels uniform over T_L classes."""
    assert len(acts) == len(T) - 2 and all(a in ACTS for a in acts)
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws, bs = _draw_params(rng, T)
    X = rng.standard_normal((N, T[0]))
    labels = rng.integers(0, T[-1], size=N)
    return _finish(name, T, acts, Ws, bs, X, labels, dtype)


def mlp_sparse_uniform(T: Sequence[int], acts: Sequence[str], N: int, seed: int,
                       zero_frac: float = 0.8, dtype: str = "float32",
                       name: str = "custom") -> Workload:
    """MNIST-shaped stand-in: x_{n,j} = 0 with probability zero_frac, else U[0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws, bs = _draw_params(rng, T)
    mask = rng.random((N, T[0])) < zero_frac
    vals = rng.random((N, T[0]))
    X = np.where(mask, 0.0, vals)
    labels = rng.integers(0, T[-1], size=N)
    return _finish(name, T, acts, Ws, bs, X, labels, dtype)


# ---------------------------------------------------------------------------
# The five named workloads.
# ---------------------------------------------------------------------------

def tiny_tanh(N: int = 64) -> Workload:
    """[4, 8, 3] tanh MLP, P = 67, N = 64, FP64 storage, seed 1."""
    return mlp_gaussian([4, 8, 3], ["tanh"], N, seed=1, dtype="float64", name="mlp4-8-3-tanh-n64")


def sigmoid_64(N: int = 10000, dtype: str = "float32") -> Workload:
    """[64, 64, 10] sigmoid MLP, P = 4810, N = 10000, FP32 storage, seed 2."""
    return mlp_gaussian([64, 64, 10], ["sigmoid"], N, seed=2, dtype=dtype,
                        name="mlp64-64-10-sigmoid-n%d" % N)


def mnist_relu(N: int = 60000) -> Workload:
    """MNIST-shaped synthetic [784, 100, 10] ReLU MLP, P = 79510, N = 60000, seed 3."""
    return mlp_sparse_uniform([784, 100, 10], ["relu"], N, seed=3, dtype="float32",
                              name="mnist-shaped-784-100-10-relu-n%d" % N)


def batched_model(m: int) -> Workload:
    """Model m of the 256-model batch: seed 4000 + m.

    T_1 ~ U{8..128}; 1 or 2 hidden tanh layers (p = 1/2 each) of width U{16..256};
    T_L ~ U{2..20}; N ~ U{100..5000}; x ~ N(0, 1); FP32 storage.
    """
    rng = np.random.Generator(np.random.PCG64(4000 + m))
    T1 = int(rng.integers(8, 129))
    nh = 1 + int(rng.random() < 0.5)
    hidden = [int(h) for h in rng.integers(16, 257, size=nh)]
    T_L = int(rng.integers(2, 21))
    N = int(rng.integers(100, 5001))
    T = [T1] + hidden + [T_L]
    Ws, bs = _draw_params(rng, T)
    X = rng.standard_normal((N, T1))
    labels = rng.integers(0, T_L, size=N)
    return _finish("batch-model-%d" % m, T, ["tanh"] * nh, Ws, bs, X, labels, "float32",
                   meta={"model_index": m})


def queries_like_mnist(nq: int, seed: int, T1: int = 784, zero_frac: float = 0.8) -> np.ndarray:
    """Query inputs for predictive-variance requests, drawn like the MNIST-shaped X."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = rng.random((nq, T1)) < zero_frac
    vals = rng.random((nq, T1))
    return np.where(mask, 0.0, vals).astype(np.float32)


def gaussian_directions(B: int, P: int, seed: int, dtype: str = "float32") -> np.ndarray:
    """B seeded Gaussian directions in R^P (rows), for dense Hessian-vector products."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((B, P)).astype(dtype))


def start_block(P: int, b: int, seed: int) -> np.ndarray:
    """Seeded Gaussian start block (P x b, float64) for subspace iteration."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((P, b))


def serving_mix(n_requests: int, seed: int = 5, rate: float = 2000.0):
    """Poisson request stream: (arrival_s, kind, arg) tuples.

    kinds: 'full' (H + OPG of a batch-distribution model) 0.25 %, 'topk' (top-32 of H,
    matrix-free) 2.5 %, 'predvar' (query batch against the resident MNIST-shaped
    model) 97.25 % with batch size log-uniform on {1..1024}.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    u = rng.random(n_requests)
    reqs = []
    for k in range(n_requests):
        if u[k] < 0.0025:
            reqs.append((float(t[k]), "full", int(rng.integers(0, 256))))
        elif u[k] < 0.0275:
            reqs.append((float(t[k]), "topk", int(rng.integers(0, 256))))
        else:
            b = int(np.clip(np.floor(np.exp(rng.uniform(0.0, np.log(1025.0)))), 1, 1024))
            reqs.append((float(t[k]), "predvar", b))
    return reqs
