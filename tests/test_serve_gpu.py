"""GPU tests of the serving core: every result is the same alone and in the mix, and
every served result agrees with the FP64 oracle at its path's tolerance (FP64 damped
queries and curvature operators 1e-10; FP32 H and OPG 1e-5; FP32 top-k eigenpairs within
the solver tolerance plus the FP32 operator error, Sec. 4.1 / 5.3)."""
import numpy as np
import pytest
import torch

from oracle import eig as oeig
from oracle import mlp
from oracle import predvar as opv
from paper_1905_05559_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05559_amd import api as A
    return A


def _dev(api, w):
    return (api.MLP.from_workload(w, dtype=torch.float32), torch.from_numpy(w.X).cuda(),
            torch.from_numpy(w.Y).cuda())


def test_mix_equals_alone(api):
    rng = np.random.default_rng(0)
    # resident network and its leading eigenpairs
    wr = workloads.mlp_gaussian([33, 40, 10], ["tanh"], 400, 21, dtype="float32")
    model, X, Y = _dev(api, wr)
    o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=3)
    lam, Q, info, st = api.hess_topk_eig(model, X, Y, 12, o)
    delta = max(1e-3, 1e-3 - float(lam.min()))
    # other networks for full / top-k requests
    others = [workloads.mlp_gaussian(T, a, N, s, dtype="float32")
              for T, a, N, s in [([12, 17, 9, 3], ["tanh", "tanh"], 300, 6), ([7, 20, 13, 5], ["sigmoid", "relu"], 100, 4)]]
    odev = [_dev(api, w) for w in others]
    # requests
    preds = []
    for k in range(64):
        nq = int(rng.integers(1, 60))
        Xq = torch.from_numpy(rng.standard_normal((nq, 33)).astype(np.float32)).cuda()
        cls = torch.from_numpy(rng.integers(0, 10, nq).astype(np.int32)).cuda() if k % 3 == 0 else None
        preds.append((Xq, cls))
    alone = [api.hess_predvar(model, lam, Q, delta, Xq, cls).clone() for Xq, cls in preds]
    full_alone = [(api.hess_exact(m, x, y, "f32").clone(), api.hess_opg(m, x, y, "f32").clone()) for m, x, y in odev]
    topk_alone = []
    for m, x, y in odev:
        oo = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=7)
        l2, q2, _, _ = api.hess_topk_eig(m, x, y, 4, oo, raise_on_noconv=False)
        topk_alone.append((l2.clone(), q2.clone()))
    # curvature-operator queries against the resident pairs (one per mode, two levels)
    lam_pd = lam.abs() + 1e-2
    curv = []
    for k, mode in enumerate(sorted(api.CURV_MODES)):
        V = torch.from_numpy(rng.standard_normal((int(rng.integers(1, 9)), model.P))).cuda()
        lt = 0.03 * (k + 1)
        curv.append((mode, V, lt, api.curvature(mode, lam_pd, Q, V, lam_tilde=lt).clone()))
    torch.cuda.synchronize()

    srv = api.Server(pool_bytes=2 << 30, n_slots=4, coalesce=True)
    ids, outs = [], []
    for i, (Xq, cls) in enumerate(preds):
        s = torch.empty(Xq.shape[0], dtype=torch.float64, device="cuda")
        outs.append(("predvar", i, s))
        ids.append(srv.submit("predvar", model, K=12, lam=lam, Q=Q, delta=delta, Xq=Xq, cls=cls, s=s))
        if i % 12 == 5 and i // 12 < len(curv):
            j = i // 12
            mode, V, lt, ref = curv[j]
            o = torch.empty_like(ref)
            outs.append(("curvature", j, o))
            ids.append(srv.submit("curvature", model, K=12, lam=lam_pd, Q=Q, Xq=V, s=o, curv_mode=mode, lam_tilde=lt))
        if i in (10, 40):
            for j, (m, x, y) in enumerate(odev):
                H = torch.empty((m.P, m.P), dtype=torch.float32, device="cuda")
                G = torch.empty_like(H)
                outs.append(("full", j, (H, G)))
                ids.append(srv.submit("full", m, X=x, Y=y, H=H, G=G))
                l2 = torch.empty(4, dtype=torch.float64, device="cuda")
                q2 = torch.empty((4, m.P), dtype=torch.float64, device="cuda")
                outs.append(("topk", j, (l2, q2)))
                ids.append(srv.submit("topk", m, X=x, Y=y, K=4, lam=l2, Q=q2, tol=1e-5, seed=7))
    lats = []
    for rid, (kind, j, out) in zip(ids, outs):
        st, lat = srv.wait(rid)
        assert st == "HESS_OK", (kind, j, st)
        lats.append(lat)
        if kind == "predvar":
            assert torch.equal(out, alone[j]), j
        elif kind == "curvature":
            assert torch.equal(out, curv[j][3]), curv[j][0]
        elif kind == "full":
            assert torch.equal(out[0], full_alone[j][0]) and torch.equal(out[1], full_alone[j][1])
        else:
            assert torch.equal(out[0], topk_alone[j][0]) and torch.equal(out[1], topk_alone[j][1])
    stats = srv.stats()
    print("served %d requests, stats %s, p50 %.2f ms" % (len(ids), stats, float(np.median(lats))), flush=True)
    assert stats["completed"] == len(ids) and stats["failed"] == 0
    assert sum(1 for o in outs if o[0] == "curvature") == len(curv)
    srv.close()

    # ---- every served result against the FP64 oracle ----
    om = mlp.model_from(wr.T, wr.acts, wr.W, wr.b)
    lam_h, Q_h = lam.cpu().numpy(), Q.cpu().numpy()
    lpd_h = lam_pd.cpu().numpy()
    worst = {}
    for kind, j, out in outs:
        if kind == "predvar":
            Xq, cls = preds[j]
            Xn = Xq.cpu().numpy().astype(np.float64)
            c = cls.cpu().numpy() if cls is not None else opv.default_classes(om, Xn)
            ref = opv.predvar_dense(lam_h, Q_h, delta, opv.logit_grad(om, Xn, c))
            e = relf(out.cpu().numpy(), ref)
            tol = 1e-10
        elif kind == "curvature":
            mode, V, lt, _ = curv[j]
            Vn = V.cpu().numpy()
            f = {"low_quad": lambda x: oeig.low_rank_quadratic(lpd_h, Q_h, x),
                 "full_quad": lambda x: oeig.full_rank_quadratic(lpd_h, Q_h, x, lt),
                 "low_apply": lambda x: oeig.low_rank_apply(lpd_h, Q_h, x),
                 "full_apply": lambda x: oeig.full_rank_apply(lpd_h, Q_h, x, lt),
                 "full_inverse": lambda x: oeig.full_rank_inverse_apply(lpd_h, Q_h, x, lt)}[mode]
            ref = np.array([f(x) for x in Vn])
            e = relf(out.cpu().numpy(), ref)
            tol = 1e-10
            kind = "curvature_" + mode
        elif kind == "full":
            w = others[j]
            o2 = mlp.model_from(w.T, w.acts, w.W, w.b)
            Xo, Yo = w.X.astype(np.float64), w.Y.astype(np.float64)
            eH = relf(out[0].double().cpu().numpy(), mlp.hessian(o2, Xo, Yo))
            eG = relf(out[1].double().cpu().numpy(), mlp.opg(o2, Xo, Yo))
            e, tol = max(eH, eG), 1e-5
        else:
            w = others[j]
            o2 = mlp.model_from(w.T, w.acts, w.W, w.b)
            Href = mlp.hessian(o2, w.X.astype(np.float64), w.Y.astype(np.float64))
            lref, _ = oeig.topk_eigh(Href, 4)
            l2, q2 = out[0].cpu().numpy(), out[1].cpu().numpy()
            # residual against the exact H: solver tolerance plus the FP32 operator error
            bound = 1e-5 * abs(lref[0]) + 1e-5 * np.linalg.norm(Href)
            res = oeig.residuals(lambda B: Href @ B, l2, q2)
            assert res.max() <= bound, (j, res, bound)
            e, tol = float(np.abs(l2 - lref).max()), bound
        worst[kind] = max(worst.get(kind, 0.0), e)
        assert e <= tol, (kind, j, e, tol)
    print("served results vs the FP64 oracle (worst error per kind): %s"
          % {k: "%.2e" % v for k, v in worst.items()}, flush=True)


def relf(A, R):
    return float(np.linalg.norm(np.asarray(A) - R) / np.linalg.norm(R))


def test_budget_rejection(api):
    w = workloads.mlp_gaussian([33, 40, 10], ["tanh"], 400, 21, dtype="float32")
    model, X, Y = _dev(api, w)
    srv = api.Server(pool_bytes=1 << 20, n_slots=1, coalesce=False)
    H = torch.empty((model.P, model.P), dtype=torch.float32, device="cuda")
    with pytest.raises(api.HessError) as e:
        srv.submit("full", model, X=X, Y=Y, H=H)
    assert e.value.name == "HESS_E_BUDGET"
    # curvature requests are checked at submission (mode, K and buffers)
    lam = torch.ones(4, dtype=torch.float64, device="cuda")
    Q = torch.zeros((4, model.P), dtype=torch.float64, device="cuda")
    V = torch.zeros((2, model.P), dtype=torch.float64, device="cuda")
    o = torch.empty(2, dtype=torch.float64, device="cuda")
    for kw in ({"curv_mode": 7}, {"curv_mode": 0, "K": model.P + 1}):
        args = dict(K=4, lam=lam, Q=Q, Xq=V, s=o, lam_tilde=0.5)
        args.update(kw)
        with pytest.raises(api.HessError) as e:
            srv.submit("curvature", model, **args)
        assert e.value.name == "HESS_E_ARG"
    srv.close()
