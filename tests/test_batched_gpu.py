"""GPU tests of hess_batched: many networks of uneven shapes in one call.

Each network's H and OPG must equal the single-network entry points bitwise (same
tile arithmetic, different schedule) and the FP64 oracle within the FP32 tolerance.
"""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_1905_05559_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05559_amd import api as A
    return A


def _dev(api, w):
    model = api.MLP.from_workload(w, dtype=torch.float32)
    return model, torch.from_numpy(w.X).cuda(), torch.from_numpy(w.Y).cuda()


def _relf(a, r):
    return float(np.linalg.norm(a - r) / np.linalg.norm(r))


NETS = [([5, 3], [], 37, 1), ([4, 8, 3], ["tanh"], 64, 2), ([33, 40, 10], ["tanh"], 129, 3),
        ([7, 20, 13, 5], ["sigmoid", "relu"], 100, 4), ([150, 30, 4], ["sigmoid"], 50, 5),
        ([12, 17, 9, 3], ["tanh", "tanh"], 333, 6)]


def test_batched_matches_single_and_oracle(api):
    ws = [workloads.mlp_gaussian(T, a, N, s, dtype="float32") for T, a, N, s in NETS]
    devs = [_dev(api, w) for w in ws]
    Hs, Gs = api.hess_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    for w, (model, X, Y), Hb, Gb in zip(ws, devs, Hs, Gs):
        Hs1 = api.hess_exact(model, X, Y, "f32")
        Gs1 = api.hess_opg(model, X, Y, "f32")
        assert torch.equal(Hb, Hs1) and torch.equal(Gb, Gs1), w.T
        om = mlp.model_from(w.T, w.acts, w.W, w.b)
        Xo, Yo = w.X.astype(np.float64), w.Y.astype(np.float64)
        eh = _relf(Hb.double().cpu().numpy(), mlp.hessian(om, Xo, Yo))
        eg = _relf(Gb.double().cpu().numpy(), mlp.opg(om, Xo, Yo))
        print("batched %-16s H relF %.2e  OPG relF %.2e" % (w.T, eh, eg), flush=True)
        assert eh <= 1e-5 and eg <= 1e-5


def test_batched_partial_outputs(api):
    ws = [workloads.mlp_gaussian(T, a, N, s, dtype="float32") for T, a, N, s in NETS[:3]]
    devs = [_dev(api, w) for w in ws]
    Hs, Gs = api.hess_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], with_G=False)
    assert Gs is None
    for (model, X, Y), Hb in zip(devs, Hs):
        assert torch.equal(Hb, api.hess_exact(model, X, Y, "f32"))


def test_batched_model_distribution_subset(api):
    """Networks drawn from the 256-network distribution (the smallest 6 of the first 40)."""
    cand = []
    for m in range(40):
        w = workloads.batched_model(m)
        cand.append((w.P, m, w))
    cand.sort()
    ws = [w for _, _, w in cand[:6]]
    devs = [_dev(api, w) for w in ws]
    Hs, Gs = api.hess_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    for w, (model, X, Y), Hb, Gb in zip(ws, devs, Hs, Gs):
        assert torch.equal(Hb, api.hess_exact(model, X, Y, "f32"))
        assert torch.equal(Gb, api.hess_opg(model, X, Y, "f32"))
        om = mlp.model_from(w.T, w.acts, w.W, w.b)
        Xo, Yo = w.X.astype(np.float64), w.Y.astype(np.float64)
        cols = list(range(0, w.P, max(1, w.P // 24)))[:24]
        ref = mlp.hessian_cols(om, Xo, Yo, 0, w.P, block=256)[:, cols] if w.P <= 3000 else None
        if ref is not None:
            e = _relf(Hb.double().cpu().numpy()[:, cols], ref)
            print("batch model %s P=%d N=%d: sampled H relF %.2e" % (w.T, w.P, w.N, e), flush=True)
            assert e <= 1e-5


# ---------------------------------------------------------------------------
# Verification subset of the 256-network distribution: the 4 smallest and the 4
# largest networks by P plus 8 seeded others, checked against FP64 oracle references
# written by tests/golden/make_batched_golden.py (diagonal 64 x 64 blocks exactly,
# whole 64-column blocks through a 32-row Gaussian sketch).
# ---------------------------------------------------------------------------

import os  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_cfg4_subset.npz")


def _sketch(P, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((32, P))


def test_batched_distribution_verification_subset(api):
    g = np.load(GOLDEN)
    models = [int(m) for m in g["models"]]
    ws = {m: workloads.batched_model(m) for m in models}
    Ps = sorted(ws[m].P for m in ws)
    assert len(models) == 16 and max(Ps) > 80000
    # waves whose outputs (H and OPG, FP32) stay within about 120 GB of HBM
    waves, cur, used = [], [], 0
    for m in sorted(models, key=lambda m: ws[m].P):
        b = 2 * 4 * ws[m].P ** 2
        if cur and used + b > 120e9:
            waves.append(cur)
            cur, used = [], 0
        cur.append(m)
        used += b
    waves.append(cur)
    worst = 0.0
    for wave in waves:
        devs = [_dev(api, ws[m]) for m in wave]
        print("wave of %d networks, P = %s" % (len(wave), [ws[m].P for m in wave]), flush=True)
        Hs, Gs = api.hess_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
        torch.cuda.synchronize()
        for m, (model, X, Y), Hb, Gb in zip(wave, devs, Hs, Gs):
            w = ws[m]
            S = _sketch(w.P, 9000 + m)
            for bi in range(2):
                key = "m%d_b%d" % (m, bi)
                c0, c1 = (int(c) for c in g[key + "_cols"])
                for tag, M in (("H", Hb), ("G", Gb)):
                    cols = M[:, c0:c1].double().cpu().numpy()
                    ed = _relf(cols[c0:c1, :], g[key + "_%s_diag" % tag])
                    es = _relf(S @ cols, g[key + "_%s_sketch" % tag])
                    worst = max(worst, ed, es)
                    print("  model %3d P=%6d N=%4d %s[:, %d:%d]  diag relF %.2e  sketch relF %.2e"
                          % (m, w.P, w.N, tag, c0, c1, ed, es), flush=True)
                    assert ed <= 1e-5 and es <= 1e-5, (m, tag, bi, ed, es)
        # the largest network of the wave also through the single-network calls: bitwise equal
        model, X, Y = devs[-1]
        Hs1 = api.hess_exact(model, X, Y, "f32")
        assert torch.equal(Hs[-1], Hs1)
        del Hs1
        Gs1 = api.hess_opg(model, X, Y, "f32")
        assert torch.equal(Gs[-1], Gs1)
        del Hs, Gs, Gs1, devs
        torch.cuda.empty_cache()
    print("verification subset: worst relF %.2e over %d networks" % (worst, len(models)), flush=True)


def test_batched_split_products_and_autotune(api):
    # split-BF16 products in the persistent launches: against the oracle at the FP32
    # tolerance and against the single-network split calls; autotuned FP32 configuration:
    # bitwise equal to the default
    ws = [workloads.mlp_gaussian(T, a, N, s, dtype="float32") for T, a, N, s in NETS]
    ws += [workloads.batched_model(m) for m in (58, 76, 148)]
    devs = [_dev(api, w) for w in ws]
    args = ([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    Hs, Gs = api.hess_batched(*args, prec="f32_split")
    for w, (model, X, Y), Hb, Gb in zip(ws, devs, Hs, Gs):
        om = mlp.model_from(w.T, w.acts, w.W, w.b)
        Xo, Yo = w.X.astype(np.float64), w.Y.astype(np.float64)
        eh = _relf(Hb.double().cpu().numpy(), mlp.hessian(om, Xo, Yo, block=256))
        eg = _relf(Gb.double().cpu().numpy(), mlp.opg(om, Xo, Yo))
        H1 = api.hess_exact(model, X, Y, "f32_split")
        G1 = api.hess_opg(model, X, Y, "f32_split")
        same = torch.equal(Hb, H1) and torch.equal(Gb, G1)
        d1 = max(_relf(Hb.double().cpu().numpy(), H1.double().cpu().numpy()),
                 _relf(Gb.double().cpu().numpy(), G1.double().cpu().numpy()))
        print("batched split %-20s H relF %.2e  OPG relF %.2e  vs single split: bitwise %s (relF %.1e)"
              % (w.T, eh, eg, same, d1), flush=True)
        assert eh <= 1e-5 and eg <= 1e-5 and d1 <= 1e-5
        assert np.array_equal(Hb.cpu().numpy(), Hb.cpu().numpy().T)
    ref = api.hess_batched(*args)
    ctx = api.Context(0)
    ctx.set_option("autotune", 1)
    tuned = api.hess_batched(*args, ctx=ctx)
    rep = ctx.autotune_report()
    print("autotune report:\n" + rep, flush=True)
    assert "krg_f32_persistent" in rep
    for a, b in zip(ref[0] + ref[1], tuned[0] + tuned[1]):
        assert torch.equal(a, b)
    ctx.close()
