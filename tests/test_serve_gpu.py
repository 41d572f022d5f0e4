"""GPU tests of the serving core: every result is the same alone and in the mix."""
import numpy as np
import pytest
import torch

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
    torch.cuda.synchronize()

    srv = api.Server(pool_bytes=2 << 30, n_slots=4, coalesce=True)
    ids, outs = [], []
    for i, (Xq, cls) in enumerate(preds):
        s = torch.empty(Xq.shape[0], dtype=torch.float64, device="cuda")
        outs.append(("predvar", i, s))
        ids.append(srv.submit("predvar", model, K=12, lam=lam, Q=Q, delta=delta, Xq=Xq, cls=cls, s=s))
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
        elif kind == "full":
            assert torch.equal(out[0], full_alone[j][0]) and torch.equal(out[1], full_alone[j][1])
        else:
            assert torch.equal(out[0], topk_alone[j][0]) and torch.equal(out[1], topk_alone[j][1])
    stats = srv.stats()
    print("served %d requests, stats %s, p50 %.2f ms" % (len(ids), stats, float(np.median(lats))), flush=True)
    assert stats["completed"] == len(ids) and stats["failed"] == 0
    srv.close()


def test_budget_rejection(api):
    w = workloads.mlp_gaussian([33, 40, 10], ["tanh"], 400, 21, dtype="float32")
    model, X, Y = _dev(api, w)
    srv = api.Server(pool_bytes=1 << 20, n_slots=1, coalesce=False)
    H = torch.empty((model.P, model.P), dtype=torch.float32, device="cuda")
    with pytest.raises(api.HessError) as e:
        srv.submit("full", model, X=X, Y=Y, H=H)
    assert e.value.name == "HESS_E_BUDGET"
    srv.close()
