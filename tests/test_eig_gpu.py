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


# ---------------------------------------------------------------------------
# Dense symmetric eigen-decomposition (the Lanczos projected problem)
# ---------------------------------------------------------------------------

def _syev_cases():
    rng = np.random.default_rng(31)
    cases = []
    for n in (1, 2, 3, 17, 100, 257, 512):
        B = rng.standard_normal((n, n))
        cases.append(("random n=%d" % n, 0.5 * (B + B.T)))
    cases.append(("diagonal n=40", np.diag(rng.standard_normal(40))))
    A = 2.0 * np.eye(64)
    A[3, 5] = A[5, 3] = 1e-3
    cases.append(("near-identity n=64", A))
    u = rng.standard_normal(90)
    cases.append(("rank one n=90", np.outer(u, u)))
    cases.append(("zero n=8", np.zeros((8, 8))))
    Qr, _ = np.linalg.qr(rng.standard_normal((200, 200)))
    d = np.repeat([3.0, 1.0, -2.0, 0.5], 50) + 1e-9 * rng.standard_normal(200)
    cases.append(("clustered n=200", (Qr * d) @ Qr.T))
    B = rng.standard_normal((416, 416))
    cases.append(("graded n=416", np.diag(np.logspace(-8, 2, 416)) + 1e-3 * (B + B.T)))
    return cases


def test_syev_matches_oracle(api):
    for tag, A in _syev_cases():
        n = A.shape[0]
        print("case syev %s" % tag, flush=True)
        # rows with a stride (lda > n) on the device
        big = torch.zeros((n, n + 7), dtype=torch.float64, device="cuda")
        big[:, :n] = torch.from_numpy(A).cuda()
        w, U = api.syev(big[:, :n])
        w, U = w.cpu().numpy(), U.cpu().numpy()
        w_ref, U_ref = eig.topk_eigh(A, n)
        nrm = max(np.linalg.norm(A), 1e-300)
        dl = np.abs(w - w_ref).max() / nrm
        res = np.linalg.norm(A @ U.T - U.T * w) / nrm
        orth = np.abs(U @ U.T - np.eye(n)).max()
        print("  max|dl|/||A|| %.1e  resid %.1e  orth %.1e" % (dl, res, orth), flush=True)
        assert dl <= 1e-12 * max(1.0, n / 64)
        assert res <= 1e-12 * max(1.0, n / 64)
        assert orth <= 1e-12 * max(1.0, n / 64)
        assert np.all(np.diff(w) <= 0)
        for k in range(n):
            i = int(np.argmax(np.abs(U[k])))
            assert U[k, i] > 0
            gap = min(abs(w_ref[k] - w_ref[k - 1]) if k > 0 else np.inf,
                      abs(w_ref[k] - w_ref[k + 1]) if k < n - 1 else np.inf)
            if gap > 1e-6 * nrm:
                assert np.abs(U[k] - U_ref[k]).max() < 1e-8, (tag, k)


def test_syev_errors(api):
    for n in (0, 513):
        A = torch.zeros((max(n, 1), max(n, 1)), dtype=torch.float64, device="cuda")
        with pytest.raises(api.HessError) as e:
            w = torch.empty(1, dtype=torch.float64, device="cuda")
            api.default_context()._check(api.default_context().lib.hess_syev(
                api.default_context().h, n, A.data_ptr(), max(n, 1), w.data_ptr(), w.data_ptr(), None, 0))
        assert e.value.name == "HESS_E_SHAPE"
    A = torch.full((5, 5), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(api.HessError) as e:
        api.syev(A)
    assert e.value.name == "HESS_E_NOCONV"


# ---------------------------------------------------------------------------
# Block Lanczos (method 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["H", "OPG"])
def test_lanczos_matrix_free_f64_tiny(api, which):
    w, model, X, Y, om = _tiny(api)
    Mref = mlp.hessian(om, w.X, w.Y) if which == "H" else mlp.opg(om, w.X, w.Y)
    o = api.eig_opts(which=which, source="matrix_free", prec="f64", tol=1e-11, seed=2, method="lanczos")
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 10, o)
    print("info", info, st)
    _check("tiny matrix-free %s f64 lanczos" % which, lam, Q, Mref, 10, 1e-10, 1e-10)


@pytest.mark.parametrize("source", ["dense", "matrix_free"])
def test_lanczos_sigmoid64_f32_top32(api, sig600, source):
    w, Href = sig600
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).cuda()
    Y = torch.from_numpy(w.Y).cuda()
    if source == "dense":
        H = api.hess_exact(model, X, Y, "f32")
        o = api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=4, method="lanczos")
        lam, Q, info, st = api.hess_topk_eig(None, None, None, 32, o)
    else:
        o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=4, method="lanczos")
        lam, Q, info, st = api.hess_topk_eig(model, X, Y, 32, o)
    print("info", info, st)
    _check("sigmoid64 N=600 %s H f32 top-32 lanczos" % source, lam, Q, Href, 32, 1e-5, 3e-5)


@pytest.mark.parametrize("K,block", [(100, 32), (100, 16), (1, 32), (150, 48)])
def test_lanczos_dense_f64_prescribed_spectrum(api, K, block):
    # M = V diag(s) V^T with an indefinite spectrum: a few outliers, a decaying bulk and
    # a negative tail, so 'LA' differs from largest-magnitude
    rng = np.random.default_rng(7 + K)
    P = 1500
    V, _ = np.linalg.qr(rng.standard_normal((P, P)))
    s = np.concatenate([[40.0, 25.0, 12.0], 5.0 * np.exp(-np.arange(P - 203) / 60.0), -np.linspace(0.5, 60.0, 200)])
    M = (V * s) @ V.T
    Md = torch.from_numpy(M).cuda()
    o = api.eig_opts(which="H", source="dense", M=Md, tol=1e-9, seed=5, method="lanczos", block=block)
    lam, Q, info, st = api.hess_topk_eig(None, None, None, K, o)
    print("case K=%d block=%d info %s %s" % (K, block, info, st), flush=True)
    _check("prescribed spectrum K=%d block=%d lanczos" % (K, block), lam, Q, M, K, 1e-9, 1e-9)


def test_lanczos_repeatable_graphs_noconv_and_shapes(api):
    w = workloads.sigmoid_64(N=600)
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to("cuda", torch.float32)
    Y = torch.from_numpy(w.Y).to("cuda", torch.float32)
    out = {}
    for graphs in (1, 0):
        ctx = api.Context(0)
        ctx.set_option("graphs", graphs)
        o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-6, seed=11, method="lanczos")
        lam, Q, info, st = api.hess_topk_eig(model, X, Y, 16, o, ctx=ctx, raise_on_noconv=False)
        torch.cuda.synchronize()
        out[graphs] = (lam.clone(), Q.clone(), info, st)
        print("case lanczos graphs=%d: %s %s" % (graphs, info, st), flush=True)
    assert torch.equal(out[1][0], out[0][0]) and torch.equal(out[1][1], out[0][1]) and out[1][2] == out[0][2]
    again = api.hess_topk_eig(model, X, Y, 16, api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-6,
                                                          seed=11, method="lanczos"))
    assert torch.equal(again[0], out[1][0]) and torch.equal(again[1], out[1][1])
    o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-30, max_iter=1, seed=11, method="lanczos")
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 16, o, raise_on_noconv=False)
    assert st == "HESS_E_NOCONV" and info["iters"] == 1
    assert np.all(np.isfinite(lam.cpu().numpy()))
    # the window must hold K + 2 blocks (at most 512 rows)
    with pytest.raises(api.HessError) as e:
        api.hess_topk_eig(model, X, Y, 460, api.eig_opts(which="H", source="matrix_free", prec="f32",
                                                           method="lanczos"))
    assert e.value.name == "HESS_E_SHAPE"


def test_lanczos_matrix_free_split_products(api, sig600):
    # the matrix-free H operator with split-BF16 products in its FP32 GEMMs: same eigenpairs to the
    # FP32 tolerance
    w, Href = sig600
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).cuda()
    Y = torch.from_numpy(w.Y).cuda()
    o = api.eig_opts(which="H", source="matrix_free", prec="f32_split", tol=1e-5, seed=4, method="lanczos")
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 32, o)
    print("info", info, st)
    _check("sigmoid64 N=600 matrix-free H split products top-32 lanczos", lam, Q, Href, 32, 1e-5, 3e-5)
