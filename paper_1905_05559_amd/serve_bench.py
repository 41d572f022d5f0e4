"""Served vs plain curvature requests under a Poisson load on one GPU.

Usage: python -m paper_1905_05559_amd.serve_bench [--seconds S] [--rate R] [--slots n]

Resident: the MNIST-shaped [784, 100, 10] ReLU network (N = 60000) with its 100
leading Hessian eigenpairs (computed once, FP32 operator and FP64 Rayleigh-Ritz).
Request mix (Poisson arrivals, seed 5): 97.25 % damped queries against the resident
eigenpairs (delta = 1e-3 shifted to keep lambda_k + delta > 0, batch size log-uniform
on 1..1024, inputs drawn like the MNIST-shaped X), 2.5 % top-32 eigenpairs of H and
0.25 % full H + OPG of networks from the 256-network distribution (a pool of the 16
smallest of the first 64, resident with their data).

served: hess_server with n slots and query coalescing; plain: one request at a time in
arrival order through the synchronous entry points on one context.  Latency = arrival
to result in device memory.  One JSON line per mode, then a consistency check: 64
seeded queries answered in the served mix equal their answers alone.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api, workloads


def build_world(n_pool_models: int = 16):
    dev = "cuda:0"
    w = workloads.mnist_relu()
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    ctx = api.Context(0)
    H = api.hess_exact(model, X, Y, "f32", ctx=ctx)
    o = api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=1, oversample=12)
    lam, Q, _, _ = api.hess_topk_eig(None, None, None, 100, o, ctx=ctx)
    del H
    ctx.release_workspace()
    torch.cuda.empty_cache()
    delta = max(1e-3, 1e-3 - float(lam.min()))
    cands = sorted(((workloads.batched_model(m).P, m) for m in range(64)))[:n_pool_models]
    pool = []
    for _, m in cands:
        wm = workloads.batched_model(m)
        mm = api.MLP.from_workload(wm, dtype=torch.float32)
        pool.append((mm, torch.from_numpy(wm.X).to(dev), torch.from_numpy(wm.Y).to(dev),
                     torch.empty((wm.P, wm.P), dtype=torch.float32, device=dev),
                     torch.empty((wm.P, wm.P), dtype=torch.float32, device=dev),
                     torch.empty(32, dtype=torch.float64, device=dev),
                     torch.empty((32, wm.P), dtype=torch.float64, device=dev)))
    Xq_all = torch.from_numpy(workloads.queries_like_mnist(1024, 11)).to(dev)
    return model, lam, Q, delta, pool, Xq_all


def make_stream(seconds: float, rate: float):
    n = max(1, int(seconds * rate))
    return workloads.serving_mix(n, seed=5, rate=rate)


def pct(v, p):
    return float(np.percentile(np.asarray(v), p)) if len(v) else float("nan")


def summarize(mode, stream, lat, t_total):
    out = {"mode": mode, "requests": len(stream), "seconds": t_total, "throughput_req_s": len(stream) / t_total}
    for kind in ("predvar", "topk", "full"):
        v = [l for (t, k, a), l in zip(stream, lat) if k == kind]
        out[kind] = {"n": len(v), "p50_ms": pct(v, 50), "p99_ms": pct(v, 99)}
    return out


def run_served(world, stream, slots, pool_gb):
    model, lam, Q, delta, pool, Xq_all = world
    srv = api.Server(pool_bytes=int(pool_gb * (1 << 30)), n_slots=slots, coalesce=True)
    outs = [torch.empty(1024, dtype=torch.float64, device="cuda") for _ in range(256)]
    ids = []
    t0 = time.perf_counter()
    for i, (ta, kind, arg) in enumerate(stream):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        if kind == "predvar":
            ids.append(srv.submit("predvar", model, K=100, lam=lam, Q=Q, delta=delta, Xq=Xq_all[:arg],
                                  s=outs[i % 256]))
        else:
            mm, X, Y, H, G, l2, q2 = pool[arg % len(pool)]
            if kind == "full":
                ids.append(srv.submit("full", mm, X=X, Y=Y, H=H, G=G))
            else:
                ids.append(srv.submit("topk", mm, X=X, Y=Y, K=32, lam=l2, Q=q2, tol=1e-5, seed=arg))
    # latency measured by the server from submission (= arrival, the loop submits on time)
    lat = []
    for rid in ids:
        st, l = srv.wait(rid)
        lat.append(l)
    t_total = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    res = summarize("served", stream, lat, t_total)
    res["server"] = stats
    return res


def run_plain(world, stream):
    model, lam, Q, delta, pool, Xq_all = world
    ctx = api.Context(0)
    s_out = torch.empty(1024, dtype=torch.float64, device="cuda")
    lat = []
    t0 = time.perf_counter()
    for ta, kind, arg in stream:
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        if kind == "predvar":
            api.hess_predvar(model, lam, Q, delta, Xq_all[:arg], ctx=ctx)
        else:
            mm, X, Y, H, G, l2, q2 = pool[arg % len(pool)]
            if kind == "full":
                api.hess_exact(mm, X, Y, "f32", out=H, ctx=ctx)
                api.hess_opg(mm, X, Y, "f32", out=G, ctx=ctx)
            else:
                o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=arg)
                api.hess_topk_eig(mm, X, Y, 32, o, ctx=ctx, raise_on_noconv=False)
        lat.append((time.perf_counter() - t0 - ta) * 1e3)
    t_total = time.perf_counter() - t0
    return summarize("plain", stream, lat, t_total)


def consistency(world, n=64):
    model, lam, Q, delta, pool, Xq_all = world
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(1, 200, n)]
    starts = [int(x) for x in rng.integers(0, 1024 - 200, n)]
    alone = [api.hess_predvar(model, lam, Q, delta, Xq_all[a:a + b].contiguous()).clone() for a, b in zip(starts, sizes)]
    srv = api.Server(pool_bytes=8 << 30, n_slots=4, coalesce=True)
    outs, ids = [], []
    for a, b in zip(starts, sizes):
        s = torch.empty(b, dtype=torch.float64, device="cuda")
        outs.append(s)
        ids.append(srv.submit("predvar", model, K=100, lam=lam, Q=Q, delta=delta, Xq=Xq_all[a:a + b].contiguous(), s=s))
    for rid in ids:
        srv.wait(rid)
    srv.close()
    worst = max(float(((o - r).abs().max() / r.abs().max()).item()) for o, r in zip(outs, alone))
    return {"queries": n, "max_rel_diff_mix_vs_alone": worst, "bitwise_equal": all(torch.equal(o, r) for o, r in zip(outs, alone))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--pool-gb", type=float, default=48.0)
    ap.add_argument("--skip-plain", action="store_true")
    args = ap.parse_args()
    t = time.perf_counter()
    world = build_world()
    print("world ready in %.1f s" % (time.perf_counter() - t), file=sys.stderr, flush=True)
    stream = make_stream(args.seconds, args.rate)
    served = run_served(world, stream, args.slots, args.pool_gb)
    print(json.dumps(served), flush=True)
    if not args.skip_plain:
        plain = run_plain(world, stream)
        print(json.dumps(plain), flush=True)
    print(json.dumps({"consistency": consistency(world)}), flush=True)


if __name__ == "__main__":
    main()
