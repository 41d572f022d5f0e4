"""Leading eigenpairs at the benchmarked sizes against FP64 oracle references.

The references (tests/golden/eig_sigmoid64_mnist.npz, written by
tests/golden/make_eig_golden.py from oracle/ only) are the algebraically largest
eigenvalues, sorted descending (Sec. 4.1, Sec. 5.3 which='LA'):

* sigmoid-64 at full N = 10000: LAPACK eigh of the oracle H and OPG;
* MNIST-shaped at full N = 60000: ARPACK Lanczos on the oracle Hessian-vector
  product, the paper's own procedure (Sec. 5.3).

Bounds.  The device solves to max_k ||M q_k - theta_k q_k|| <= tol |theta_1| on its
FP32 operator M, whose distance from the exact matrix is at most the FP32 tolerance
times its Frobenius norm.  Against the exact operator a Ritz pair's residual is then
at most tol |lambda_1| + 1e-5 ||M||_F, and each Ritz value lies within that residual
of an eigenvalue.  Residuals are taken with the oracle's own operator (Hessian-vector
products, or J^T (J q) / N for the OPG).
"""
import os

import numpy as np
import pytest
import torch

from oracle import mlp
from paper_1905_05559_amd import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "eig_sigmoid64_mnist.npz")
TOL_OP = 1e-5   # FP32 operator, relative Frobenius


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05559_amd import api as A
    return A


@pytest.fixture(scope="module")
def golden():
    return np.load(GOLDEN)


@pytest.fixture(scope="module")
def sig(api):
    w = workloads.sigmoid_64()
    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    Xo, Yo = w.X.astype(np.float64), w.Y.astype(np.float64)
    J = mlp.jacobian(om, Xo, Yo)
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).cuda()
    Y = torch.from_numpy(w.Y).cuda()
    ctx = api.Context(0)
    H = api.hess_exact(model, X, Y, "f32", ctx=ctx)
    G = api.hess_opg(model, X, Y, "f32", ctx=ctx)
    return w, om, Xo, Yo, J, model, X, Y, H, G, ctx


def _oracle_apply(which, om, Xo, Yo, J, Q):
    """M q for the rows q of Q with the oracle operator."""
    if which == "H":
        return mlp.hvp(om, Xo, Yo, Q)
    return ((J @ Q.T).T @ J) / J.shape[0]


def _check_pairs(tag, lam, Q, lam_ref, fro, apply_ref, tol, Qref=None):
    K = lam.shape[0]
    bound = tol * abs(lam_ref[0]) + TOL_OP * fro
    dl = np.abs(lam - lam_ref[:K])
    R = apply_ref(Q) - lam[:, None] * Q
    res = np.linalg.norm(R, axis=1)
    orth = np.abs(Q @ Q.T - np.eye(K)).max()
    print("%-44s max|dl| %.2e  max res %.2e  bound %.2e  (|l1| %.3e, ||M||F %.3e)  orth %.1e"
          % (tag, dl.max(), res.max(), bound, abs(lam_ref[0]), fro, orth), flush=True)
    assert np.all(np.diff(lam) <= 0)
    assert dl.max() <= bound
    assert res.max() <= bound
    assert orth <= 1e-10
    if Qref is not None:
        # vectors of well-separated eigenvalues: sin of the angle <= residual / gap
        for k in range(Qref.shape[0]):
            gap = min(abs(lam_ref[k] - lam_ref[k - 1]) if k > 0 else np.inf, abs(lam_ref[k] - lam_ref[k + 1]))
            if gap > 100 * bound:
                c = abs(float(Q[k] @ Qref[k]))
                s = np.sqrt(max(0.0, 1.0 - c * c))
                assert s <= 2 * res[k] / gap + 1e-7, (k, s, res[k], gap)
                assert Q[k] @ Qref[k] > 0  # same sign rule


@pytest.mark.parametrize("K", [32, 100])
@pytest.mark.parametrize("method", ["subspace", "lanczos"])
@pytest.mark.parametrize("source", ["dense", "matrix_free"])
@pytest.mark.parametrize("which", ["H", "OPG"])
def test_sigmoid64_full_n_topk(api, golden, sig, which, source, method, K):
    w, om, Xo, Yo, J, model, X, Y, H, G, ctx = sig
    print("case sigmoid-64 N=10000 top-%d of %s, %s operator, %s" % (K, which, source, method), flush=True)
    tol = 1e-5
    kw = dict(tol=tol, seed=11, max_iter=200, method=method)
    if method == "subspace":
        kw["oversample"] = 12 if K == 100 else 10
    else:
        kw["block"] = 16
    if source == "dense":
        o = api.eig_opts(which=which, source="dense", M=H if which == "H" else G, **kw)
        lam, Q, info, st = api.hess_topk_eig(None, None, None, K, o, ctx=ctx)
    else:
        o = api.eig_opts(which=which, source="matrix_free", prec="f32", **kw)
        lam, Q, info, st = api.hess_topk_eig(model, X, Y, K, o, ctx=ctx)
    assert st == "HESS_OK", (st, info)
    tag = "H" if which == "H" else "G"
    _check_pairs("sig64 %s %s %s top-%d" % (which, source, method, K), lam.cpu().numpy(), Q.cpu().numpy(),
                 golden["sig_%s_lam" % tag], float(golden["sig_%s_fro" % tag]),
                 lambda V: _oracle_apply(which, om, Xo, Yo, J, V), tol, golden["sig_%s_Q8" % tag])


def test_mnist_shaped_top100_against_lanczos_reference(api, golden):
    # the bench's eigen step: dense FP32 H (split-BF16 products), block Lanczos with
    # blocks of 16, tol 1e-5; eigenvalues against ARPACK on the oracle HVP, residuals of
    # 8 seeded Ritz pairs with the oracle HVP
    w = workloads.mnist_relu()
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).cuda()
    Y = torch.from_numpy(w.Y).cuda()
    ctx = api.Context(0)
    H = api.hess_exact(model, X, Y, "f32_split", ctx=ctx)
    o = api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=1, max_iter=200, method="lanczos", block=16)
    lam, Q, info, st = api.hess_topk_eig(None, None, None, 100, o, ctx=ctx)
    assert st == "HESS_OK", (st, info)
    del H
    ctx.release_workspace()
    torch.cuda.empty_cache()
    lam = lam.cpu().numpy()
    lref = golden["mnist_H_lam"][:100]
    dl = np.abs(lam - lref)
    print("MNIST-shaped top-100: max|dl|/|l1| %.2e (lambda_1 %.6e ref %.6e, lambda_100 %.6e ref %.6e), info %s"
          % (dl.max() / abs(lref[0]), lam[0], lref[0], lam[99], lref[99], info), flush=True)
    assert np.all(np.diff(lam) <= 0)
    assert dl.max() <= 1e-5 * abs(lref[0])
    rng = np.random.Generator(np.random.PCG64(8))
    ks = np.sort(rng.choice(100, size=8, replace=False))
    Qs = Q[ks].cpu().numpy()
    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    HQ = mlp.hvp(om, w.X.astype(np.float64), w.Y.astype(np.float64), Qs)
    res = np.linalg.norm(HQ - lam[ks][:, None] * Qs, axis=1) / abs(lref[0])
    print("oracle-HVP residuals / |l1| of pairs %s: %s" % (ks.tolist(), np.array2string(res, precision=2)),
          flush=True)
    assert res.max() <= 3e-5
    ctx.close()
