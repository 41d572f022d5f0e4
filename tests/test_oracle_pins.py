"""Pins for the FP64 oracle: values fixed by the paper or by mathematics.

Every check here compares the oracle with something other than itself:
values printed in the paper, finite differences, the complex-step derivative,
closed forms written out independently with np.kron, null spaces that follow
from the softmax shift invariance, LAPACK/ARPACK, or exact identities.
"""
import json
import os

import numpy as np
import pytest

from oracle import eig, mlp, predvar
from paper_1905_05559_amd import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _model(w: workloads.Workload):
    return mlp.model_from(w.T, w.acts, w.W, w.b), w.X.astype(np.float64), w.Y.astype(np.float64)


def _small(T, acts, N, seed):
    return _model(workloads.mlp_gaussian(T, acts, N, seed))


def _fd_grad(model, X, Y, h=1e-5):
    om = mlp.flatten(model.W, model.b)
    g = np.empty_like(om)
    for p in range(om.size):
        e = np.zeros_like(om)
        e[p] = h
        g[p] = (mlp.cost(mlp.with_omega(model, om + e), X, Y)
                - mlp.cost(mlp.with_omega(model, om - e), X, Y)) / (2 * h)
    return g


def _complex_step_hessian(model, X, Y, h=1e-30):
    """H[:, j] = Im grad C(omega + i h e_j) / h (Squire & Trapp 1998)."""
    om = mlp.flatten(model.W, model.b).astype(np.complex128)
    P = om.size
    H = np.empty((P, P))
    for j in range(P):
        e = np.zeros(P, dtype=np.complex128)
        e[j] = 1j * h
        H[:, j] = np.imag(mlp.gradient(mlp.with_omega(model, om + e), X, Y)) / h
    return H


def _relf(A, R):
    return np.linalg.norm(A - R) / np.linalg.norm(R)


# ---------------------------------------------------------------------------
# Values printed in the paper.
# ---------------------------------------------------------------------------

def test_paper_per_example_gradient_demo():
    g = json.load(open(os.path.join(GOLD, "paper_sec3_1_per_example.json")))
    X = np.array(g["X"])
    w = np.array(g["w"])
    # a one-output linear layer (no hidden layer, zero bias) is the paper's model
    model = mlp.Model([4, 1], [], [w[None, :]], [np.zeros(1)])
    z = mlp.logits_forward(model, X)[:, 0]
    np.testing.assert_array_equal(z, g["outputs"])
    G = predvar.logit_grad(model, X, [0, 0])
    np.testing.assert_array_equal(G[:, :4], g["per_example_gradients"])
    np.testing.assert_array_equal(G[:, :4].sum(axis=0), g["batched_gradient"])
    # Khatri-Rao rows with delta = 1 reproduce the per-example gradients too
    KR = mlp.khatri_rao_rows(np.ones((2, 1)), X)
    np.testing.assert_array_equal(KR[:, :4], g["per_example_gradients"])


def test_paper_flatten_shapes():
    g = json.load(open(os.path.join(GOLD, "paper_sec3_2_shapes.json")))
    assert mlp.num_params(g["T"]) == g["P"]
    (ow, ob), = mlp.layer_offsets(g["T"])
    assert ob - ow == g["weight_block_rows"]
    assert mlp.num_params(g["T"]) - ob == g["bias_block_rows"]
    # flatten / unflatten round trip in the paper's row-wise order
    rng = np.random.default_rng(0)
    W = [rng.standard_normal((32, 64))]
    b = [rng.standard_normal(32)]
    om = mlp.flatten(W, b)
    assert om[5] == W[0][0, 5] and om[64 + 3] == W[0][1, 3] and om[2048 + 7] == b[0][7]
    W2, b2 = mlp.unflatten(om, g["T"])
    np.testing.assert_array_equal(W2[0], W[0])
    np.testing.assert_array_equal(b2[0], b[0])


def test_param_counts_of_workloads():
    assert mlp.num_params([4, 8, 3]) == 67
    assert mlp.num_params([64, 64, 10]) == 4810
    assert mlp.num_params([784, 100, 10]) == 79510


# ---------------------------------------------------------------------------
# Derivatives against finite differences and the complex step.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("T,acts", [([4, 8, 3], ["tanh"]), ([3, 5, 4, 3], ["sigmoid", "tanh"]),
                                    ([4, 6, 3], ["relu"])])
def test_gradient_matches_central_fd(T, acts):
    model, X, Y = _small(T, acts, 16, 7)
    g = mlp.gradient(model, X, Y)
    fd = _fd_grad(model, X, Y)
    assert np.max(np.abs(g - fd)) < 1e-9


def test_tiny_tanh_gradient_fd():
    model, X, Y = _model(workloads.tiny_tanh())
    g = mlp.gradient(model, X, Y)
    assert np.max(np.abs(g - _fd_grad(model, X, Y))) < 1e-9


@pytest.mark.parametrize("T,acts", [([4, 8, 3], ["tanh"]), ([3, 5, 4, 3], ["sigmoid", "tanh"]),
                                    ([3, 4, 5, 2], ["tanh", "sigmoid"]), ([4, 6, 3], ["relu"]),
                                    ([3, 4, 5, 3], ["relu", "relu"])])
def test_hessian_matches_complex_step(T, acts):
    model, X, Y = _small(T, acts, 12, 11)
    H = mlp.hessian(model, X, Y)
    Hcs = _complex_step_hessian(model, X, Y)
    assert _relf(H, Hcs) < 1e-13


def test_tiny_tanh_hessian_complex_step_and_fd():
    model, X, Y = _model(workloads.tiny_tanh())
    H = mlp.hessian(model, X, Y)
    assert _relf(H, _complex_step_hessian(model, X, Y)) < 1e-13
    # central FD of the analytic gradient (a weaker, independent check)
    om = mlp.flatten(model.W, model.b)
    P, h = om.size, 1e-5
    Hfd = np.empty((P, P))
    for j in range(P):
        e = np.zeros(P)
        e[j] = h
        Hfd[:, j] = (mlp.gradient(mlp.with_omega(model, om + e), X, Y)
                     - mlp.gradient(mlp.with_omega(model, om - e), X, Y)) / (2 * h)
    assert _relf(H, Hfd) < 1e-8


# ---------------------------------------------------------------------------
# Closed forms.
# ---------------------------------------------------------------------------

def _closed_form_last_layer(p, a):
    """(1/N) sum_n S_n (x) [a_n; 1][a_n; 1]^T reordered to (W row-major, then b)."""
    N, C = p.shape
    D = a.shape[1]
    HWW = np.zeros((C * D, C * D))
    HWb = np.zeros((C * D, C))
    Hbb = np.zeros((C, C))
    for n in range(N):
        S = np.diag(p[n]) - np.outer(p[n], p[n])
        HWW += np.kron(S, np.outer(a[n], a[n]))
        HWb += np.kron(S, a[n][:, None])
        Hbb += S
    top = np.hstack([HWW, HWb])
    bot = np.hstack([HWb.T, Hbb])
    return np.vstack([top, bot]) / N


def test_no_hidden_layer_closed_form():
    model, X, Y = _small([5, 3], [], 40, 3)
    H = mlp.hessian(model, X, Y)
    p = mlp.forward(model, X)[1][2]
    Hc = _closed_form_last_layer(p, X)
    assert _relf(H, Hc) < 1e-14


def test_no_hidden_layer_expected_opg_equals_hessian():
    """At L = 2, E_{y ~ p}[OPG] = H exactly (H does not depend on y there)."""
    model, X, Y = _small([5, 3], [], 30, 5)
    H = mlp.hessian(model, X, Y)
    p = mlp.forward(model, X)[1][2]
    N, C = p.shape
    EG = np.zeros_like(H)
    for c in range(C):
        Yc = np.zeros_like(Y)
        Yc[:, c] = 1.0
        J = mlp.jacobian(model, X, Yc)
        EG += (J * p[:, c:c + 1]).T @ J / N
    assert _relf(EG, H) < 1e-13


@pytest.mark.parametrize("T,acts", [([4, 6, 3], ["tanh"]), ([3, 5, 4, 3], ["sigmoid", "relu"])])
def test_last_layer_block_closed_form(T, acts):
    model, X, Y = _small(T, acts, 25, 9)
    H = mlp.hessian(model, X, Y)
    _, A = mlp.forward(model, X)
    L = model.L
    ow, _ = mlp.layer_offsets(T)[L - 2]
    Hc = _closed_form_last_layer(A[L], A[L - 1])
    assert _relf(H[ow:, ow:], Hc) < 1e-13


def test_relu_within_layer_blocks_equal_gauss_newton():
    """ReLU nets: sigma'' = 0 and the net is linear in each single layer's parameters,
    so every within-layer block of H equals the Gauss-Newton block (1/N) sum J_f^T S J_f,
    while the cross-layer blocks differ."""
    T = [4, 6, 5, 3]
    model, X, Y = _small(T, ["relu", "relu"], 20, 13)
    H = mlp.hessian(model, X, Y)
    N, C = X.shape[0], T[-1]
    p = mlp.forward(model, X)[1][model.L]
    Jf = np.stack([predvar.logit_grad(model, X, np.full(N, c)) for c in range(C)], axis=1)
    GN = np.zeros_like(H)
    for n in range(N):
        S = np.diag(p[n]) - np.outer(p[n], p[n])
        GN += Jf[n].T @ S @ Jf[n]
    GN /= N
    offs = mlp.layer_offsets(T)
    bounds = [(ow, ob + T[k + 1]) for k, (ow, ob) in enumerate(offs)]
    for (s, e) in bounds:
        assert _relf(H[s:e, s:e], GN[s:e, s:e]) < 1e-13
    s0, e0 = bounds[0]
    s1, e1 = bounds[1]
    assert _relf(H[s1:e1, s0:e0], GN[s1:e1, s0:e0]) > 1e-3


# ---------------------------------------------------------------------------
# Invariants.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("T,acts", [([4, 8, 3], ["tanh"]), ([3, 5, 4, 4], ["sigmoid", "relu"])])
def test_softmax_shift_null_space(T, acts):
    """Adding a constant to every logit leaves the cost unchanged, so H v = OPG v = 0 for
    v = ones on b^(L) and for v = 1 (x) r on W^(L-1) (same r added to every row)."""
    model, X, Y = _small(T, acts, 20, 17)
    P = mlp.num_params(T)
    ow, ob = mlp.layer_offsets(T)[-1]
    v1 = np.zeros(P)
    v1[ob:] = 1.0
    r = np.random.default_rng(1).standard_normal(T[-2])
    v2 = np.zeros(P)
    v2[ow:ob] = np.tile(r, T[-1])
    H = mlp.hessian(model, X, Y)
    G = mlp.opg(model, X, Y)
    for v in (v1, v2):
        assert np.linalg.norm(H @ v) < 1e-13 * np.linalg.norm(H) * np.linalg.norm(v)
        assert np.linalg.norm(G @ v) < 1e-13 * np.linalg.norm(G) * np.linalg.norm(v)
        assert np.linalg.norm(mlp.hvp(model, X, Y, v[None, :])) < 1e-13 * np.linalg.norm(H)


def test_symmetry_and_hvp_bilinearity():
    model, X, Y = _small([3, 5, 4, 3], ["tanh", "sigmoid"], 15, 19)
    H = mlp.hessian(model, X, Y)
    assert np.linalg.norm(H - H.T) < 1e-14 * np.linalg.norm(H)
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal((2, H.shape[0]))
    Hu, Hv = mlp.hvp(model, X, Y, np.stack([u, v]))
    assert abs(u @ Hv - v @ Hu) < 1e-13 * np.linalg.norm(H) * np.linalg.norm(u) * np.linalg.norm(v)


def test_opg_psd_and_trace():
    model, X, Y = _small([4, 8, 3], ["tanh"], 30, 23)
    G = mlp.opg(model, X, Y)
    w = np.linalg.eigvalsh(G)
    assert w.min() >= -10 * np.finfo(float).eps * np.abs(w).max()
    J = mlp.jacobian(model, X, Y)
    assert abs(np.trace(G) - np.mean(np.sum(J * J, axis=1))) < 1e-14 * np.trace(G)
    # OPG is not the outer product of the mean gradient (Sec. 3, the inequality)
    g = mlp.gradient(model, X, Y)
    assert _relf(np.outer(g, g), G) > 0.1


def test_sampled_helpers_match_full_matrices():
    model, X, Y = _small([5, 7, 4], ["sigmoid"], 20, 29)
    H = mlp.hessian(model, X, Y)
    G = mlp.opg(model, X, Y)
    P = H.shape[0]
    np.testing.assert_allclose(mlp.hessian_cols(model, X, Y, 10, 30, block=7), H[:, 10:30],
                               rtol=0, atol=1e-15 * np.abs(H).max())
    rows, cols = [0, 3, 34, 35, P - 1], [1, 2, 40, P - 4]
    np.testing.assert_allclose(mlp.opg_tile(model, X, Y, rows, cols), G[np.ix_(rows, cols)],
                               rtol=1e-13, atol=1e-16)
    # OPG columns from delta-weighted sums, against J^T J / N (two hidden layers)
    model2, X2, Y2 = _small([6, 9, 7, 4], ["tanh", "sigmoid"], 25, 31)
    G2 = mlp.opg(model2, X2, Y2)
    cols2 = [0, 5, 53, 62, 63, 64, 120, G2.shape[0] - 1]
    np.testing.assert_allclose(mlp.opg_cols(model2, X2, Y2, cols2), G2[:, cols2],
                               rtol=0, atol=1e-14 * np.abs(G2).max())


# ---------------------------------------------------------------------------
# Eigenpairs.
# ---------------------------------------------------------------------------

def test_curvature_operators_against_formed_matrices():
    # Sec. 5.5-5.6 and App. A.2: implicit forms against the explicit P x P matrices
    rng = np.random.default_rng(13)
    P, K = 40, 6
    Qf, _ = np.linalg.qr(rng.standard_normal((P, K)))
    Q = Qf.T                                   # K x P, orthonormal rows
    lam = np.sort(rng.uniform(0.5, 3.0, K))[::-1]
    lt = 0.2
    Hl = Q.T @ np.diag(lam) @ Q
    Hf = Hl + lt * (np.eye(P) - Q.T @ Q)
    x = rng.standard_normal(P)
    np.testing.assert_allclose(eig.low_rank_apply(lam, Q, x), Hl @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(eig.full_rank_apply(lam, Q, x, lt), Hf @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(eig.full_rank_inverse_apply(lam, Q, x, lt), np.linalg.solve(Hf, x), rtol=1e-12)
    # default lam~ = lam_K, and the quadratic forms are x . (operator x)
    np.testing.assert_allclose(eig.full_rank_apply(lam, Q, x), (Hl + lam[-1] * (np.eye(P) - Q.T @ Q)) @ x,
                               rtol=1e-13, atol=1e-13)
    assert abs(eig.low_rank_quadratic(lam, Q, x) - x @ Hl @ x) < 1e-12
    assert abs(eig.full_rank_quadratic(lam, Q, x, lt) - x @ Hf @ x) < 1e-12
    # H~~ is full rank: eigenvalues are lam_k and lam~ (P - K times)
    w = np.linalg.eigvalsh(Hf)
    np.testing.assert_allclose(np.sort(w), np.sort(np.concatenate([lam, np.full(P - K, lt)])), rtol=1e-12)


def test_topk_eigh_known_spectrum_and_sign():
    rng = np.random.default_rng(4)
    P = 30
    Qf, _ = np.linalg.qr(rng.standard_normal((P, P)))
    lam = np.linspace(3.0, -2.0, P)
    M = (Qf * lam) @ Qf.T
    w, Q = eig.topk_eigh(M, 5)
    np.testing.assert_allclose(w, lam[:5], atol=1e-13)
    for k in range(5):
        q = Q[k]
        assert abs(abs(q @ Qf[:, k]) - 1) < 1e-12
        i = np.argmax(np.abs(q))
        assert q[i] > 0


def test_lanczos_la_matches_eigh_on_oracle_hessian():
    """The paper's Sec. 5.3 procedure (eigsh which='LA' on the HVP operator)."""
    model, X, Y = _model(workloads.tiny_tanh())
    H = mlp.hessian(model, X, Y)
    Hs = 0.5 * (H + H.T)
    w1, Q1 = eig.topk_eigh(Hs, 10)
    w2, Q2 = eig.topk_lanczos(lambda v: mlp.hvp(model, X, Y, v[None, :])[0], H.shape[0], 10)
    np.testing.assert_allclose(w2, w1, atol=1e-10 * np.abs(w1).max())
    res = eig.residuals(lambda V: Hs @ V, w1, Q1)
    assert res.max() < 1e-12 * np.abs(w1).max()


def test_low_and_full_rank_forms():
    """Sec. 5.5/5.6: the implicit quadratic forms equal the explicitly formed matrices."""
    rng = np.random.default_rng(5)
    P, K = 25, 4
    Q, _ = np.linalg.qr(rng.standard_normal((P, K)))
    Q = Q.T
    lam = np.array([5.0, 3.0, 2.0, 1.5])
    x = rng.standard_normal(P)
    Hlow = Q.T @ np.diag(lam) @ Q
    Hfull = Hlow + lam[-1] * (np.eye(P) - Q.T @ Q)
    assert abs(eig.low_rank_quadratic(lam, Q, x) - x @ Hlow @ x) < 1e-12
    assert abs(eig.full_rank_quadratic(lam, Q, x) - x @ Hfull @ x) < 1e-12
    wf = np.linalg.eigvalsh(Hfull)
    assert wf.min() > 0  # full rank (Appendix A.2)


# ---------------------------------------------------------------------------
# Predictive variance.
# ---------------------------------------------------------------------------

def test_logit_grad_matches_fd():
    model, X, Y = _small([4, 6, 5, 3], ["tanh", "sigmoid"], 5, 31)
    cls = np.array([0, 2, 1, 1, 0])
    G = predvar.logit_grad(model, X, cls)
    om = mlp.flatten(model.W, model.b)
    h = 1e-6
    for p in range(om.size):
        e = np.zeros_like(om)
        e[p] = h
        zp = mlp.logits_forward(mlp.with_omega(model, om + e), X)[np.arange(5), cls]
        zm = mlp.logits_forward(mlp.with_omega(model, om - e), X)[np.arange(5), cls]
        np.testing.assert_allclose(G[:, p], (zp - zm) / (2 * h), atol=1e-8)


def test_predvar_identity_equals_dense_solve():
    model, X, Y = _model(workloads.tiny_tanh())
    H = mlp.hessian(model, X, Y)
    lam, Q = eig.topk_eigh(0.5 * (H + H.T), 10)
    Xq = X[:7]
    G = predvar.logit_grad(model, Xq, predvar.default_classes(model, Xq))
    for delta in (1e-3, 0.5):
        if np.min(lam) + delta <= 0:
            continue
        s1 = predvar.predvar_identity(lam, Q, delta, G)
        s2 = predvar.predvar_dense(lam, Q, delta, G)
        np.testing.assert_allclose(s1, s2, rtol=1e-9)
