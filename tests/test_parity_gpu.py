"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative Frobenius error over the compared entries): FP64 paths
1e-10, FP32 paths 1e-5, BF16 OPG 2e-2.  Every result is also reported with its
max-abs error.  Outputs must be exactly symmetric.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mlp
from paper_1905_05559_amd import workloads

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-2, "f32_split": 1e-5}


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05559_amd import api as A
    return A


def relf(A, R):
    return float(np.linalg.norm(A - R) / np.linalg.norm(R))


def report(tag, A, R):
    e = relf(A, R)
    print("%-48s relF %.3e  maxabs %.3e" % (tag, e, float(np.abs(A - R).max())), flush=True)
    sys.stdout.flush()
    return e


def to_dev(api, w, dtype):
    td = {"float64": torch.float64, "float32": torch.float32}[dtype]
    model = api.MLP.from_workload(w, dtype=td)
    X = torch.from_numpy(w.X).to("cuda", td)
    Y = torch.from_numpy(w.Y).to("cuda", td)
    return model, X, Y


def oracle_of(w):
    return mlp.model_from(w.T, w.acts, w.W, w.b), w.X.astype(np.float64), w.Y.astype(np.float64)


SMALL = [
    ([4, 8, 3], ["tanh"], 64, 1),
    ([5, 3], [], 37, 2),
    ([7, 20, 13, 5], ["sigmoid", "relu"], 100, 3),
    ([3, 17, 2], ["relu"], 1, 4),
    ([33, 40, 10], ["tanh"], 129, 5),
    ([150, 30, 4], ["sigmoid"], 50, 6),
    ([6, 9, 7, 8, 4], ["tanh", "sigmoid", "tanh"], 70, 7),
]


@pytest.mark.parametrize("T,acts,N,seed", SMALL)
@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_small_exact_and_opg(api, T, acts, N, seed, prec):
    print("case T=%s acts=%s N=%d seed=%d prec=%s" % (T, acts, N, seed, prec), flush=True)
    w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float64" if prec == "f64" else "float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    Href = mlp.hessian(om, Xo, Yo)
    Gref = mlp.opg(om, Xo, Yo)
    H = api.hess_exact(model, X, Y, prec).double().cpu().numpy()
    G = api.hess_opg(model, X, Y, prec).double().cpu().numpy()
    assert np.array_equal(H, H.T) and np.array_equal(G, G.T)
    assert report("H   %s %s" % (T, prec), H, Href) <= TOL[prec]
    assert report("OPG %s %s" % (T, prec), G, Gref) <= TOL[prec]


@pytest.mark.parametrize("T,acts,N,seed", SMALL[:5])
def test_small_opg_bf16(api, T, acts, N, seed):
    w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float32")
    model, X, Y = to_dev(api, w, "float32")
    om, Xo, Yo = oracle_of(w)
    G = api.hess_opg(model, X, Y, "bf16").double().cpu().numpy()
    assert np.array_equal(G, G.T)
    assert report("OPG %s bf16" % T, G, mlp.opg(om, Xo, Yo)) <= TOL["bf16"]


@pytest.fixture(scope="module")
def sig64():
    w = workloads.sigmoid_64()
    om, Xo, Yo = oracle_of(w)
    return w, om, Xo, Yo, mlp.opg(om, Xo, Yo)


SIG64_BLOCKS = [(0, 64), (4032, 4096), (4096, 4170), (4746, 4810)]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32_split"])
def test_sigmoid64_opg_full(api, sig64, prec):
    w, om, Xo, Yo, Gref = sig64
    model, X, Y = to_dev(api, w, "float64" if prec == "f64" else "float32")
    if prec == "f64":
        model = api.MLP.from_workload(w, dtype=torch.float64)
        X, Y = X.double(), Y.double()
    G = api.hess_opg(model, X, Y, prec).double().cpu().numpy()
    assert np.array_equal(G, G.T)
    assert report("sigmoid64 OPG %s" % prec, G, Gref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_sigmoid64_exact_sampled_blocks(api, sig64, prec):
    w, om, Xo, Yo, _ = sig64
    td = torch.float64 if prec == "f64" else torch.float32
    model = api.MLP.from_workload(w, dtype=td)
    X = torch.from_numpy(w.X).to("cuda", td)
    Y = torch.from_numpy(w.Y).to("cuda", td)
    H = api.hess_exact(model, X, Y, prec)
    Hn = H.double().cpu().numpy()
    del H
    assert np.array_equal(Hn, Hn.T)
    for c0, c1 in SIG64_BLOCKS:
        ref = mlp.hessian_cols(om, Xo, Yo, c0, c1)
        assert report("sigmoid64 H[:, %d:%d] %s" % (c0, c1, prec), Hn[:, c0:c1], ref) <= TOL[prec]


def test_sigmoid64_reduced_n_exact_full(api):
    w = workloads.sigmoid_64(N=600)
    om, Xo, Yo = oracle_of(w)
    Href = mlp.hessian(om, Xo, Yo, block=256)
    for prec in ("f64", "f32"):
        td = torch.float64 if prec == "f64" else torch.float32
        model = api.MLP.from_workload(w, dtype=td)
        X = torch.from_numpy(w.X).to("cuda", td)
        Y = torch.from_numpy(w.Y).to("cuda", td)
        H = api.hess_exact(model, X, Y, prec).double().cpu().numpy()
        assert report("sigmoid64 N=600 H %s" % prec, H, Href) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_wide_units_exact_and_opg(api, prec):
    # 301 inputs per hidden unit: tiles touch at most two units per side; N = 300 leaves a
    # ragged last chunk of examples
    print("case wide units [300, 20, 6] tanh N=300 prec=%s" % prec, flush=True)
    w = workloads.mlp_gaussian([300, 20, 6], ["tanh"], 300, 8, dtype="float64" if prec == "f64" else "float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    Href = mlp.hessian(om, Xo, Yo, block=256)
    Gref = mlp.opg(om, Xo, Yo)
    H = api.hess_exact(model, X, Y, prec).double().cpu().numpy()
    G = api.hess_opg(model, X, Y, prec).double().cpu().numpy()
    assert np.array_equal(H, H.T) and np.array_equal(G, G.T)
    assert report("H   wide %s" % prec, H, Href) <= TOL[prec]
    assert report("OPG wide %s" % prec, G, Gref) <= TOL[prec]


@pytest.mark.parametrize("T,acts,N,seed", [
    ([127, 24, 10], ["relu"], 300, 11),   # 128 slots per unit: wavefronts never straddle units
    ([223, 12, 5], ["tanh"], 97, 12),     # 224 slots: every other unit boundary splits a wavefront
])
def test_presplit_columns_exact(api, T, acts, N, seed):
    # split products read the first layer's column source pre-split (unit slots padded to a
    # multiple of 32, at least 128); ragged last chunk of examples in both cases
    print("case presplit columns T=%s acts=%s N=%d seed=%d" % (T, acts, N, seed), flush=True)
    w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    Href = mlp.hessian(om, Xo, Yo, block=256)
    H = api.hess_exact(model, X, Y, "f32_split").double().cpu().numpy()
    assert np.array_equal(H, H.T)
    assert report("H   %s f32_split (pre-split columns)" % T, H, Href) <= TOL["f32_split"]


@pytest.mark.parametrize("T,N,seed,dead", [
    ([127, 24, 10], 300, 31, 12),   # 128 slots per unit: one unit per column tile
    ([223, 12, 5], 97, 32, 4),      # 224 slots: column tiles that straddle two units
])
def test_relu_example_lists_with_dead_units(api, T, N, seed, dead):
    # Split products on a ReLU column layer sum each column tile over the examples where one of
    # its units has a nonzero weight.  The first `dead` hidden units never fire (bias -1e3), so
    # the tiles of their columns have empty lists: those rows of H must come out exactly zero,
    # and the rest must match the oracle.
    print("case relu example lists, dead units T=%s N=%d dead=%d" % (T, N, dead), flush=True)
    w = workloads.mlp_gaussian(T, ["relu"], N, seed, dtype="float32")
    w.b[0][:dead] = -1e3
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    Href = mlp.hessian(om, Xo, Yo, block=256)
    H = api.hess_exact(model, X, Y, "f32_split").double().cpu().numpy()
    T0, T1 = T[0], T[1]
    rows = [j * T0 + i for j in range(dead) for i in range(T0)] + [T1 * T0 + j for j in range(dead)]
    assert not np.any(H[rows, :]) and not np.any(Href[rows, :])
    assert np.array_equal(H, H.T)
    assert report("H   %s f32_split (example lists, %d dead units)" % (T, dead), H, Href) <= TOL["f32_split"]


@pytest.mark.parametrize("T,acts,N,seed", [
    ([127, 24, 10], ["relu"], 97, 13),
    ([150, 20, 5], ["tanh"], 300, 14),
])
def test_presplit_ragged_n_ignores_stale_workspace(api, T, acts, N, seed):
    # Regression: the last (partial) chunk of examples of the pre-split tile must not read
    # source rows past N.  The workspace is filled with NaN first (all bits set), so any such
    # read would reach H through a zero weight as NaN.
    print("case presplit ragged N, NaN-filled workspace T=%s N=%d" % (T, N), flush=True)
    w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    ctx = api.Context(0)
    nb = api.workspace_size("exact", model, X, Y, "f32_split", ctx=ctx)
    ctx.workspace(nb).fill_(255)
    H = api.hess_exact(model, X, Y, "f32_split", ctx=ctx).double().cpu().numpy()
    assert np.isfinite(H).all()
    assert np.array_equal(H, H.T)
    assert report("H   %s N=%d f32_split (NaN workspace)" % (T, N), H,
                  mlp.hessian(om, Xo, Yo, block=256)) <= TOL["f32_split"]
    ctx.close()


# Column blocks of the MNIST-shaped network (P = 79510): the first inputs of unit 0, the
# boundary between hidden units 37 and 38, the last hidden biases and first output
# weights, and the output layer's tail with its biases.
MNIST_BLOCKS = [(0, 16), (29784, 29800), (78490, 78506), (79494, 79510)]


@pytest.fixture(scope="module")
def mnist_refs():
    w = workloads.mnist_relu()
    om, Xo, Yo = oracle_of(w)
    return w, om, Xo, Yo, {b: mlp.hessian_cols(om, Xo, Yo, b[0], b[1]) for b in MNIST_BLOCKS}


def test_mnist_shaped_full_size_sampled_columns(api, mnist_refs):
    # the configuration the bench times: full N = 60000, FP32 H and OPG, BF16 OPG
    print("case mnist-shaped [784, 100, 10] relu N=60000, column blocks %s" % MNIST_BLOCKS, flush=True)
    w, om, Xo, Yo, refs = mnist_refs
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to("cuda")
    Y = torch.from_numpy(w.Y).to("cuda")
    for prec in ("f32", "f32_split"):
        H = api.hess_exact(model, X, Y, prec)
        rowsH = {b: H[b[0]:b[1], :].double().cpu().numpy() for b in MNIST_BLOCKS}
        colsH = {b: H[:, b[0]:b[1]].double().cpu().numpy() for b in MNIST_BLOCKS[:2]}
        del H
        torch.cuda.empty_cache()
        for b in MNIST_BLOCKS[:2]:
            assert np.array_equal(rowsH[b], colsH[b].T)
        for b in MNIST_BLOCKS:
            assert report("mnist H[:, %d:%d] %s" % (b + (prec,)), rowsH[b].T, refs[b]) <= TOL[prec]
    cols = [c for b in MNIST_BLOCKS for c in range(b[0], b[1])]
    Gref = mlp.opg_cols(om, Xo, Yo, cols)
    for prec in ("f32", "bf16", "f32_split"):
        G = api.hess_opg(model, X, Y, prec)
        Gc = G[:, cols].double().cpu().numpy()
        del G
        torch.cuda.empty_cache()
        assert report("mnist OPG[:, blocks] %s" % prec, Gc, Gref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f32_split"])
def test_mnist_shaped_full_size_hvp_block(api, mnist_refs, prec):
    # 64 directions at full N = 60000 (the bench's HVP configuration in width, in chunks of
    # examples): the basis vectors of the four column blocks, so that H V^T holds those
    # columns of H; with split products the R-backward step of the hidden layer is formed,
    # split and transposed in one pass (a block of 64 directions fills the device)
    w, om, Xo, Yo, refs = mnist_refs
    print("case mnist-shaped HVP, 64 basis directions, full N, %s" % prec, flush=True)
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to("cuda")
    Y = torch.from_numpy(w.Y).to("cuda")
    cols = [c for b in MNIST_BLOCKS for c in range(b[0], b[1])]
    V = torch.zeros((len(cols), model.P), dtype=torch.float32, device="cuda")
    for k, c in enumerate(cols):
        V[k, c] = 1.0
    HV = api.hess_hvp(model, X, Y, V, prec).double().cpu().numpy()
    ref = np.concatenate([refs[b] for b in MNIST_BLOCKS], axis=1).T
    assert report("mnist HV (64 basis directions) %s" % prec, HV, ref) <= TOL[prec]


@pytest.mark.parametrize("N", [2000, 333])
@pytest.mark.parametrize("prec", ["f32", "f32_split"])
def test_wide_direction_block_hvp(api, N, prec):
    # MNIST-shaped layers at a small N: 64 random directions against the oracle (the
    # one-pass R-backward step with split products); both example counts end in a partial
    # 64-example tile and a zero-padded 32-example chunk of the contraction
    print("case wide-block HVP [784, 100, 10] relu N=%d B=64 %s" % (N, prec), flush=True)
    w = workloads.mlp_gaussian([784, 100, 10], ["relu"], N, 21, dtype="float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    V = workloads.gaussian_directions(64, model.P, 5, dtype="float32")
    ref = mlp.hvp(om, Xo, Yo, V.astype(np.float64))
    HV = api.hess_hvp(model, X, Y, torch.from_numpy(V).cuda(), prec).double().cpu().numpy()
    assert report("wide-block HV N=%d %s" % (N, prec), HV, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_exact_cols_match_oracle(api, prec):
    for T, acts, N, seed in (SMALL[2], SMALL[4]):
        print("case exact_cols T=%s N=%d prec=%s" % (T, N, prec), flush=True)
        w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float64" if prec == "f64" else "float32")
        model, X, Y = to_dev(api, w, w.dtype)
        om, Xo, Yo = oracle_of(w)
        P = model.P
        for c0, nc in ((0, P), (P // 3, 37), (P - 5, 5)):
            ref = mlp.hessian_cols(om, Xo, Yo, c0, c0 + nc)
            Hc = api.hess_exact_cols(model, X, Y, c0, nc, prec).double().cpu().numpy()
            assert report("H cols %d..%d of %s %s" % (c0, c0 + nc, T, prec), Hc, ref) <= TOL[prec]


def test_exact_cols_several_blocks(api):
    # 600 columns: two blocks of basis HVPs (512 + 88); against the oracle and hess_exact
    w = workloads.sigmoid_64(N=600)
    om, Xo, Yo = oracle_of(w)
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to("cuda", torch.float32)
    Y = torch.from_numpy(w.Y).to("cuda", torch.float32)
    print("case exact_cols sigmoid64 N=600 columns 1000..1600", flush=True)
    Hc = api.hess_exact_cols(model, X, Y, 1000, 600, "f32").double().cpu().numpy()
    ref = mlp.hessian_cols(om, Xo, Yo, 1000, 1600, block=256)
    assert report("sigmoid64 N=600 H[:, 1000:1600] via columns", Hc, ref) <= TOL["f32"]
    H = api.hess_exact(model, X, Y, "f32")[:, 1000:1600].double().cpu().numpy()
    assert report("columns vs hess_exact", Hc, H) <= 2 * TOL["f32"]
    with pytest.raises(api.HessError) as e:
        api.hess_exact_cols(model, X, Y, model.P - 3, 4, "f32")
    assert e.value.name == "HESS_E_SHAPE"


def test_autotune_keeps_results_bitwise(api):
    # every tile configuration the tuner may pick gives the same bits as the default
    w = workloads.sigmoid_64(N=600)
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to("cuda", torch.float32)
    Y = torch.from_numpy(w.Y).to("cuda", torch.float32)
    ref = {}
    for tune in (0, 1):
        ctx = api.Context(0)
        ctx.set_option("autotune", tune)
        H = api.hess_exact(model, X, Y, "f32", ctx=ctx).clone()
        G = api.hess_opg(model, X, Y, "f32", ctx=ctx).clone()
        Gb = api.hess_opg(model, X, Y, "bf16", ctx=ctx).clone()
        torch.cuda.synchronize()
        ref[tune] = (H, G, Gb)
        rep = ctx.autotune_report()
        print("case autotune=%d report:\n%s" % (tune, rep), flush=True)
        if tune:
            assert "krg_f32" in rep and "gram_bf16" in rep and "->" in rep
        else:
            assert rep == ""
    for a, b in zip(ref[0], ref[1]):
        assert torch.equal(a, b)


def test_run_twice_bitwise(api):
    """No atomics in any reduction: two runs give bitwise-identical results."""
    w = workloads.mlp_gaussian([33, 40, 10], ["tanh"], 300, 9, dtype="float32")
    model, X, Y = to_dev(api, w, "float32")
    for prec in ("f32", "bf16"):
        a = api.hess_opg(model, X, Y, prec).cpu()
        b = api.hess_opg(model, X, Y, prec).cpu()
        assert torch.equal(a, b)
    a = api.hess_exact(model, X, Y, "f32").cpu()
    b = api.hess_exact(model, X, Y, "f32").cpu()
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------
# Dense Hessian-vector products (R-operator, Appendix A.1).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("T,acts,N,seed", SMALL)
@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_small_hvp(api, T, acts, N, seed, prec):
    print("hvp case T=%s N=%d prec=%s" % (T, N, prec), flush=True)
    w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float64" if prec == "f64" else "float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    P = mlp.num_params(T)
    for B in (1, 5):
        V = workloads.gaussian_directions(B, P, seed + B, dtype=w.dtype)
        ref = mlp.hvp(om, Xo, Yo, V.astype(np.float64))
        HV = api.hess_hvp(model, X, Y, torch.from_numpy(V).cuda(), prec).double().cpu().numpy()
        assert report("HV %s B=%d %s" % (T, B, prec), HV, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_prepared_hvp_operator(api, prec):
    # one preparation, several blocks of different sizes; against the oracle and hess_hvp
    T, acts, N, seed = SMALL[4]
    w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float64" if prec == "f64" else "float32")
    model, X, Y = to_dev(api, w, w.dtype)
    om, Xo, Yo = oracle_of(w)
    op = api.HvpOperator(model, X, Y, prec, max_B=64)
    rng = np.random.default_rng(9)
    for B in (1, 7, 64):
        print("case prepared HVP T=%s B=%d prec=%s" % (T, B, prec), flush=True)
        Vn = rng.standard_normal((B, model.P))
        V = torch.from_numpy(Vn).to("cuda", X.dtype)
        HV = op.apply(V).double().cpu().numpy()
        ref = mlp.hvp(om, Xo, Yo, Vn if prec == "f64" else Vn.astype(np.float32).astype(np.float64))
        assert report("prepared HVP B=%d %s" % (B, prec), HV, ref) <= TOL[prec]
        HV2 = api.hess_hvp(model, X, Y, V, prec).double().cpu().numpy()
        assert report("prepared vs per-call HVP B=%d %s" % (B, prec), HV, HV2) <= TOL[prec]
    with pytest.raises(api.HessError) as e:
        op.apply(torch.zeros((65, model.P), dtype=X.dtype, device="cuda"))
    assert e.value.name == "HESS_E_SHAPE"
    op.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_sigmoid64_hvp(api, sig64, prec):
    w, om, Xo, Yo, _ = sig64
    td = torch.float64 if prec == "f64" else torch.float32
    model = api.MLP.from_workload(w, dtype=td)
    X = torch.from_numpy(w.X).to("cuda", td)
    Y = torch.from_numpy(w.Y).to("cuda", td)
    V = workloads.gaussian_directions(8, w.P, 77, dtype="float64")
    ref = mlp.hvp(om, Xo, Yo, V)
    HV = api.hess_hvp(model, X, Y, torch.from_numpy(V).to("cuda", td), prec).double().cpu().numpy()
    assert report("sigmoid64 HV B=8 %s" % prec, HV, ref) <= TOL[prec]


def test_hvp_basis_equals_exact_columns(api):
    """H e_j from the dense R-operator path equals column j of the assembled H."""
    w = workloads.mlp_gaussian([6, 9, 7, 8, 4], ["tanh", "sigmoid", "tanh"], 70, 7, dtype="float64")
    model, X, Y = to_dev(api, w, "float64")
    P = w.P
    H = api.hess_exact(model, X, Y, "f64")
    cols = [0, 5, 53, 54, 60, P - 1]
    V = torch.zeros((len(cols), P), dtype=torch.float64, device="cuda")
    for k, c in enumerate(cols):
        V[k, c] = 1.0
    HV = api.hess_hvp(model, X, Y, V, "f64")
    err = (HV - H[:, cols].T).abs().max().item() / H.abs().max().item()
    print("basis HVP vs exact columns: rel max err %.3e" % err, flush=True)
    assert err < 1e-12


# ---------------------------------------------------------------------------
# Mini-batch and per-example modes (Sec. 3: H and the OPG of a mini-batch or of one
# example are the same means over N' examples; the paper's listings average mini-batch
# matrices over floor(N / bs) batches and drop the remainder)
# ---------------------------------------------------------------------------

def test_minibatch_mean_equals_full_n(api):
    w = workloads.mlp_gaussian([12, 17, 9, 4], ["tanh", "sigmoid"], 300, 21, dtype="float64")
    model, X, Y = to_dev(api, w, "float64")
    om, Xo, Yo = oracle_of(w)
    bs = 60
    Hb = [api.hess_exact(model, X[i:i + bs].contiguous(), Y[i:i + bs].contiguous(), "f64").clone()
          for i in range(0, 300, bs)]
    Gb = [api.hess_opg(model, X[i:i + bs].contiguous(), Y[i:i + bs].contiguous(), "f64").clone()
          for i in range(0, 300, bs)]
    Hm = (sum(Hb) / len(Hb)).cpu().numpy()
    Gm = (sum(Gb) / len(Gb)).cpu().numpy()
    print("case mini-batch mean, bs=%d, %d batches" % (bs, len(Hb)), flush=True)
    assert report("mean of mini-batch H vs oracle full-N H", Hm, mlp.hessian(om, Xo, Yo)) <= TOL["f64"]
    assert report("mean of mini-batch OPG vs oracle full-N OPG", Gm, mlp.opg(om, Xo, Yo)) <= TOL["f64"]
    # the listings' loop with a remainder: floor(N / bs) batches, the last N mod bs examples dropped
    bs2 = 70
    nb = 300 // bs2
    Hd = sum(api.hess_exact(model, X[i * bs2:(i + 1) * bs2].contiguous(), Y[i * bs2:(i + 1) * bs2].contiguous(),
                            "f64").clone() for i in range(nb)) / nb
    Hk = api.hess_exact(model, X[:nb * bs2].contiguous(), Y[:nb * bs2].contiguous(), "f64")
    assert report("dropped-remainder mean vs H of the kept examples", Hd.cpu().numpy(),
                  Hk.cpu().numpy()) <= TOL["f64"]


def test_per_example_hessians_batched(api):
    # one hess_batched call with N' = 1 per network: the per-example H_n and OPG_n
    w = workloads.mlp_gaussian([9, 14, 5], ["tanh"], 8, 22, dtype="float32")
    model, X, Y = to_dev(api, w, "float32")
    om, Xo, Yo = oracle_of(w)
    n = X.shape[0]
    Hs, Gs = api.hess_batched([model] * n, [X[i:i + 1].contiguous() for i in range(n)],
                              [Y[i:i + 1].contiguous() for i in range(n)])
    J = mlp.jacobian(om, Xo, Yo)
    print("case per-example H and OPG of %d examples in one batched call" % n, flush=True)
    for i in range(n):
        Hr = mlp.hessian(om, Xo[i:i + 1], Yo[i:i + 1])
        assert report("per-example H_%d" % i, Hs[i].cpu().numpy().astype(np.float64), Hr) <= TOL["f32"]
        assert report("per-example OPG_%d = g g^T" % i, Gs[i].cpu().numpy().astype(np.float64),
                      np.outer(J[i], J[i])) <= TOL["f32"]
    Hmean = sum(h.double() for h in Hs).cpu().numpy() / n
    assert report("mean of per-example H vs full H", Hmean, mlp.hessian(om, Xo, Yo)) <= TOL["f32"]


@pytest.mark.parametrize("T,acts,N,seed,cap", [
    ([64, 64, 10], ["sigmoid"], 1000, 2, 20_000_000),    # chunks of 288 examples, last one 136
    ([127, 24, 10], ["relu"], 700, 15, 4_000_000),       # pre-split columns, chunks of 288
])
def test_exact_chunked_over_examples(api, T, acts, N, seed, cap):
    # a small factor cap forces hess_exact to accumulate H over chunks of examples (the
    # mini-batch sum of Sec. 5.1); against the oracle and the one-pass H
    om_w = {}
    for prec in ("f64", "f32", "f32_split"):
        w = workloads.mlp_gaussian(T, acts, N, seed, dtype="float64" if prec == "f64" else "float32")
        model, X, Y = to_dev(api, w, w.dtype)
        if "H" not in om_w:
            om, Xo, Yo = oracle_of(w)
            om_w["H"] = mlp.hessian(om, Xo, Yo, block=256)
        ctx1 = api.Context(0)
        H1 = api.hess_exact(model, X, Y, prec, ctx=ctx1).double().cpu().numpy()
        ws1 = api.workspace_size("exact", model, X, Y, prec, ctx=ctx1)
        ctx = api.Context(0)
        ctx.set_option("factor_bytes", cap)
        wsc = api.workspace_size("exact", model, X, Y, prec, ctx=ctx)
        print("case chunked exact T=%s N=%d %s: workspace %.1f MB one pass, %.1f MB chunked"
              % (T, N, prec, ws1 / 1e6, wsc / 1e6), flush=True)
        assert wsc < ws1
        Hc = api.hess_exact(model, X, Y, prec, ctx=ctx).double().cpu().numpy()
        assert np.array_equal(Hc, Hc.T)
        assert report("H chunked %s %s" % (T, prec), Hc, om_w["H"]) <= TOL[prec]
        assert report("H chunked vs one pass %s %s" % (T, prec), Hc, H1) <= (1e-13 if prec == "f64" else 2e-6)
        ctx.close()
        ctx1.close()
