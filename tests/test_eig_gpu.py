"""GPU parity of hess_topk_eig against LAPACK eigh of the FP64 oracle matrices.

Eigenvalues: |lambda - lambda_ref| <= tol_op * ||M||_F (Weyl, with the operator's own
precision) and residuals ||M q - lambda q|| <= tol * |lambda_1| on the oracle matrix.
Eigenvectors are compared only where the spectral gap is large (|q . q_ref| close to
1, sign fixed by the largest-|.| component rule); bases of clustered eigenvalues are
not unique.
"""
import numpy as np
import pytest
import torch

from oracle import eig, mlp
from paper_1905_05559_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05559_amd import api as A
    return A


def _check(tag, lam, Q, Mref, K, tol_val, tol_res):
    lam = lam.cpu().numpy()
    Q = Q.cpu().numpy()
    Ms = 0.5 * (Mref + Mref.T)
    w_ref, Q_ref = eig.topk_eigh(Ms, K)
    nrm = np.linalg.norm(Ms)
    dl = np.abs(lam - w_ref).max()
    res = eig.residuals(lambda V: Ms @ V, lam, Q).max() / abs(w_ref[0])
    orth = np.abs(Q @ Q.T - np.eye(K)).max()
    print("%-34s max|dl|/||M||F %.2e  max res/|l1| %.2e  orth %.1e" % (tag, dl / nrm, res, orth), flush=True)
    assert dl <= tol_val * nrm
    assert res <= tol_res
    assert orth <= 1e-10
    # sign rule
    for k in range(K):
        i = int(np.argmax(np.abs(Q[k])))
        assert Q[k, i] > 0
    # vectors where the gap to the rest of the spectrum is large
    w_all = np.linalg.eigvalsh(Ms)[::-1]
    for k in range(K):
        gap = min(abs(w_all[k] - w_all[k - 1]) if k > 0 else np.inf, abs(w_all[k] - w_all[k + 1]))
        if gap > 1e3 * tol_val * nrm:
            assert abs(abs(Q[k] @ Q_ref[k]) - 1) < 1e-6


def _tiny(api, dtype="float64"):
    w = workloads.tiny_tanh()
    td = torch.float64 if dtype == "float64" else torch.float32
    model = api.MLP.from_workload(w, dtype=td)
    X = torch.from_numpy(w.X).to("cuda", td)
    Y = torch.from_numpy(w.Y).to("cuda", td)
    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    return w, model, X, Y, om


def test_dense_f64_hessian_tiny(api):
    w, model, X, Y, om = _tiny(api)
    Href = mlp.hessian(om, w.X, w.Y)
    H = api.hess_exact(model, X, Y, "f64")
    o = api.eig_opts(which="H", source="dense", M=H, tol=1e-11, seed=1)
    lam, Q, info, st = api.hess_topk_eig(None, None, None, 10, o)
    print("info", info, st)
    _check("tiny dense H f64", lam, Q, Href, 10, 1e-10, 1e-10)


def test_matrix_free_f64_hessian_tiny(api):
    w, model, X, Y, om = _tiny(api)
    Href = mlp.hessian(om, w.X, w.Y)
    o = api.eig_opts(which="H", source="matrix_free", prec="f64", tol=1e-11, seed=2)
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 10, o)
    print("info", info, st)
    _check("tiny matrix-free H f64", lam, Q, Href, 10, 1e-10, 1e-10)


def test_matrix_free_f64_opg_tiny(api):
    w, model, X, Y, om = _tiny(api)
    Gref = mlp.opg(om, w.X, w.Y)
    o = api.eig_opts(which="OPG", source="matrix_free", prec="f64", tol=1e-11, seed=3)
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 10, o)
    print("info", info, st)
    _check("tiny matrix-free OPG f64", lam, Q, Gref, 10, 1e-10, 1e-10)


@pytest.fixture(scope="module")
def sig600():
    w = workloads.sigmoid_64(N=600)
    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    Href = mlp.hessian(om, w.X.astype(np.float64), w.Y.astype(np.float64), block=256)
    return w, Href


@pytest.mark.parametrize("source", ["dense", "matrix_free"])
def test_sigmoid64_f32_top32(api, sig600, source):
    w, Href = sig600
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).cuda()
    Y = torch.from_numpy(w.Y).cuda()
    if source == "dense":
        H = api.hess_exact(model, X, Y, "f32")
        o = api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=4)
        lam, Q, info, st = api.hess_topk_eig(None, None, None, 32, o)
    else:
        o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=4)
        lam, Q, info, st = api.hess_topk_eig(model, X, Y, 32, o)
    print("info", info, st)
    _check("sigmoid64 N=600 %s H f32 top-32" % source, lam, Q, Href, 32, 1e-5, 3e-5)


def test_bitwise_repeatable_and_noconv(api):
    w, model, X, Y, om = _tiny(api)
    o = api.eig_opts(which="H", source="matrix_free", prec="f64", tol=1e-11, seed=9)
    a = api.hess_topk_eig(model, X, Y, 6, o)
    b = api.hess_topk_eig(model, X, Y, 6, o)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    o2 = api.eig_opts(which="H", source="matrix_free", prec="f64", tol=1e-30, max_iter=1, seed=9)
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 6, o2, raise_on_noconv=False)
    assert st == "HESS_E_NOCONV" and info["iters"] == 1


@pytest.mark.parametrize("source", ["matrix_free", "dense"])
def test_graph_replays_equal_eager(api, source):
    # the operator applications replay captured HIP graphs (default) with eager orthogonalisation
    # and Rayleigh-Ritz work in between; every result must equal the eager run bitwise
    w = workloads.sigmoid_64(N=600)
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to("cuda", torch.float32)
    Y = torch.from_numpy(w.Y).to("cuda", torch.float32)
    M = api.hess_exact(model, X, Y, "f32") if source == "dense" else None
    out = {}
    for graphs in (1, 0):
        ctx = api.Context(0)
        ctx.set_option("graphs", graphs)
        o = api.eig_opts(which="H", source=source, M=M, prec="f32", tol=1e-6, seed=11, max_iter=40)
        lam, Q, info, st = api.hess_topk_eig(model, X, Y, 16, o, ctx=ctx, raise_on_noconv=False)
        torch.cuda.synchronize()
        out[graphs] = (lam.clone(), Q.clone(), info, st)
        print("case graphs=%d source=%s: %s %s" % (graphs, source, info, st), flush=True)
    assert out[1][2]["applies"] > 6  # several replays of each captured pair
    assert torch.equal(out[1][0], out[0][0]) and torch.equal(out[1][1], out[0][1])
    assert out[1][2] == out[0][2] and out[1][3] == out[0][3]
