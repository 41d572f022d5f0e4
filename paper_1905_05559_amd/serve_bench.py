"""Served vs plain curvature requests under a Poisson load on one GPU.

Usage: python -m paper_1905_05559_amd.serve_bench [--rate R] [--sat-seconds S] [--seconds-80 S]
       [--slots n] [--max-out-gb G]
(bench.py runs the same measurement after its timed steps).

Resident: the MNIST-shaped [784, 100, 10] ReLU network (N = 60000) with its 100
leading Hessian eigenpairs (FP32 operator, FP64 Rayleigh-Ritz).  Request mix
(workloads.serving_mix, Poisson arrivals, seed 5): 97.25 % damped queries against the
resident eigenpairs (delta = 1e-3, shifted up if needed to keep lambda_k + delta > 0;
batch size log-uniform on 1..1024, inputs drawn like the MNIST-shaped X), 2.5 % top-32
eigenpairs of H (matrix-free, FP32, tol 1e-5) and 0.25 % full H + OPG (FP32) of networks
drawn uniformly from the 256-network distribution among those an output budget admits
(H and OPG together at most max_out_gb, i.e. P <= sqrt(max_out_gb / 8 B)).

served: hess_server with n slots and query coalescing; plain: one request at a time in
arrival order through the synchronous entry points on one context.  Latency = arrival
to result in device memory.  Outputs of served full and top-k requests go to rings of
device buffers; a ring entry is reused only after its previous request completed (the
plain mode writes to buffers of its own).  Consistency: seeded queries, and the last full
and top-k requests of the last served run, equal their answers computed alone (bitwise).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import api, workloads

N_MODELS = 256


def admitted_models(max_out_gb: float):
    """Indices of the batch-distribution networks whose H + OPG (FP32) fit max_out_gb."""
    pmax = int(math.sqrt(max_out_gb * 1e9 / 8.0))
    out = []
    for m in range(N_MODELS):
        w = workloads.batched_model(m)
        if w.P <= pmax:
            out.append((m, w))
    return pmax, out


class World:
    """Resident network, its eigenpairs, the admitted request networks and output rings."""

    def __init__(self, model, X, Y, lam, Q, max_out_gb: float = 2.2, full_ring: int = 8, topk_ring: int = 64):
        dev = "cuda:0"
        self.model, self.X, self.Y, self.lam, self.Q = model, X, Y, lam, Q
        self.delta = max(1e-3, 1e-3 - float(lam.min()))
        self.pmax, adm = admitted_models(max_out_gb)
        self.max_out_gb = max_out_gb
        self.nets = []
        for m, w in adm:
            self.nets.append((m, api.MLP.from_workload(w, dtype=torch.float32), torch.from_numpy(w.X).to(dev),
                              torch.from_numpy(w.Y).to(dev)))
        Pbig = max(n[1].P for n in self.nets)
        self.full_bufs = [(torch.empty(Pbig * Pbig, dtype=torch.float32, device=dev),
                           torch.empty(Pbig * Pbig, dtype=torch.float32, device=dev)) for _ in range(full_ring)]
        self.plain_full = (torch.empty(Pbig * Pbig, dtype=torch.float32, device=dev),
                           torch.empty(Pbig * Pbig, dtype=torch.float32, device=dev))
        self.topk_bufs = [(torch.empty(32, dtype=torch.float64, device=dev),
                           torch.empty(32 * Pbig, dtype=torch.float64, device=dev)) for _ in range(topk_ring)]
        self.pred_bufs = [torch.empty(1024, dtype=torch.float64, device=dev) for _ in range(256)]
        self.Xq_all = torch.from_numpy(workloads.queries_like_mnist(1024, 11, T1=model.T[0])).to(dev)

    def net(self, arg):
        return self.nets[arg % len(self.nets)]

    def describe(self):
        Ps = [n[1].P for n in self.nets]
        return {"resident": "mnist-shaped-784-100-10-relu-n60000, top-100 H eigenpairs",
                "request_networks": "batch distribution (256 networks, seeds 4000+m) admitted by H+OPG <= %.1f GB "
                                    "(P <= %d): %d networks, P %d..%d, median %d"
                                    % (self.max_out_gb, self.pmax, len(Ps), min(Ps), max(Ps), int(np.median(Ps)))}


def build_world(max_out_gb: float = 2.2) -> World:
    dev = "cuda:0"
    w = workloads.mnist_relu()
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    ctx = api.Context(0)
    H = api.hess_exact(model, X, Y, "f32_split", ctx=ctx)
    o = api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=1, method="lanczos", block=16)
    lam, Q, _, _ = api.hess_topk_eig(None, None, None, 100, o, ctx=ctx)
    del H
    ctx.release_workspace()
    torch.cuda.empty_cache()
    return World(model, X, Y, lam, Q, max_out_gb)


def make_stream(seconds: float, rate: float, seed: int = 5):
    n = max(1, int(seconds * rate))
    return workloads.serving_mix(n, seed=seed, rate=rate)


def pct(v, p):
    return float(np.percentile(np.asarray(v), p)) if len(v) else float("nan")


def summarize(mode, stream, lat, t_total, offered):
    out = {"mode": mode, "offered_req_s": round(offered, 1), "requests": len(stream),
           "seconds": round(t_total, 3), "throughput_req_s": round(len(stream) / t_total, 1)}
    for kind in ("predvar", "topk", "full"):
        v = [l for (t, k, a), l in zip(stream, lat) if k == kind]
        out[kind] = {"n": len(v), "p50_ms": round(pct(v, 50), 3), "p99_ms": round(pct(v, 99), 3)}
    return out


def run_served(world: World, stream, offered, slots=4, pool_gb=48.0):
    srv = api.Server(pool_bytes=int(pool_gb * (1 << 30)), n_slots=slots, coalesce=True)
    ids, kinds = [], []
    lat = {}
    ring_owner = {}  # ("full"|"topk", ring index) -> request id still in flight
    last = {}
    nf = nt = 0

    def reclaim(key):
        rid = ring_owner.pop(key, None)
        if rid is not None and rid not in lat:
            lat[rid] = srv.wait(rid)

    t0 = time.perf_counter()
    for i, (ta, kind, arg) in enumerate(stream):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        if kind == "predvar":
            rid = srv.submit("predvar", world.model, K=world.lam.shape[0], lam=world.lam, Q=world.Q,
                             delta=world.delta, Xq=world.Xq_all[:arg], s=world.pred_bufs[i % 256])
        else:
            m, mm, X, Y = world.net(arg)
            P = mm.P
            if kind == "full":
                key = ("full", nf % len(world.full_bufs))
                nf += 1
                reclaim(key)
                Hb, Gb = world.full_bufs[key[1]]
                H, G = Hb[:P * P].view(P, P), Gb[:P * P].view(P, P)
                rid = srv.submit("full", mm, X=X, Y=Y, H=H, G=G)
                last["full"] = (rid, m, mm, X, Y, H, G)
            else:
                key = ("topk", nt % len(world.topk_bufs))
                nt += 1
                reclaim(key)
                lb, qb = world.topk_bufs[key[1]]
                q2 = qb[:32 * P].view(32, P)
                rid = srv.submit("topk", mm, X=X, Y=Y, K=32, lam=lb, Q=q2, tol=1e-5, seed=arg)
                last["topk"] = (rid, m, mm, X, Y, lb, q2, arg)
            ring_owner[key] = rid
        ids.append(rid)
        kinds.append(kind)
    for rid in ids:
        if rid not in lat:
            lat[rid] = srv.wait(rid)
    t_total = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    res = summarize("served", stream, [lat[r][1] for r in ids], t_total, offered)
    res["failed"] = sum(1 for r in ids if lat[r][0] != "HESS_OK")
    res["server"] = stats
    return res, last


def run_plain(world: World, stream, offered):
    ctx = api.Context(0)
    lat = []
    t0 = time.perf_counter()
    for ta, kind, arg in stream:
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        if kind == "predvar":
            api.hess_predvar(world.model, world.lam, world.Q, world.delta, world.Xq_all[:arg], ctx=ctx)
        else:
            m, mm, X, Y = world.net(arg)
            P = mm.P
            if kind == "full":
                Hb, Gb = world.plain_full
                api.hess_exact(mm, X, Y, "f32", out=Hb[:P * P].view(P, P), ctx=ctx)
                api.hess_opg(mm, X, Y, "f32", out=Gb[:P * P].view(P, P), ctx=ctx)
            else:
                o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=arg)
                api.hess_topk_eig(mm, X, Y, 32, o, ctx=ctx, raise_on_noconv=False)
        lat.append((time.perf_counter() - t0 - ta) * 1e3)
    t_total = time.perf_counter() - t0
    ctx.close()
    return summarize("plain", stream, lat, t_total, offered)


def consistency(world: World, last=None, n=64):
    """Seeded queries answered in a served mix, and the last full and top-k requests of a
    served run, against the same requests answered alone (bitwise)."""
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(1, 200, n)]
    starts = [int(x) for x in rng.integers(0, 1024 - 200, n)]
    K = world.lam.shape[0]
    alone = [api.hess_predvar(world.model, world.lam, world.Q, world.delta,
                              world.Xq_all[a:a + b].contiguous()).clone() for a, b in zip(starts, sizes)]
    srv = api.Server(pool_bytes=8 << 30, n_slots=4, coalesce=True)
    outs, ids = [], []
    for a, b in zip(starts, sizes):
        s = torch.empty(b, dtype=torch.float64, device="cuda")
        outs.append(s)
        ids.append(srv.submit("predvar", world.model, K=K, lam=world.lam, Q=world.Q, delta=world.delta,
                              Xq=world.Xq_all[a:a + b].contiguous(), s=s))
    for rid in ids:
        srv.wait(rid)
    srv.close()
    res = {"queries": n, "queries_bitwise_equal": all(torch.equal(o, r) for o, r in zip(outs, alone))}
    if last and "full" in last:
        _, m, mm, X, Y, H, G = last["full"]
        ok = torch.equal(H, api.hess_exact(mm, X, Y, "f32")) and torch.equal(G, api.hess_opg(mm, X, Y, "f32"))
        res["full_request_bitwise_equal"] = {"network": m, "P": mm.P, "equal": bool(ok)}
    if last and "topk" in last:
        _, m, mm, X, Y, lb, q2, arg = last["topk"]
        o = api.eig_opts(which="H", source="matrix_free", prec="f32", tol=1e-5, seed=arg)
        l_a, q_a, _, _ = api.hess_topk_eig(mm, X, Y, 32, o, raise_on_noconv=False)
        res["topk_request_bitwise_equal"] = {"network": m, "P": mm.P,
                                             "equal": bool(torch.equal(lb, l_a) and torch.equal(q2, q_a))}
    return res


def measure(world: World, rate: float = 2000.0, sat_seconds: float = 4.0, seconds_80: float = 5.0, slots: int = 4,
            log=lambda *a: None):
    """Served and plain at the offered rate (saturation: both fall behind), then both at 80 %
    of the served mode's measured saturation throughput; plus the consistency check."""
    out = {"world": world.describe(), "slots": slots}
    s_sat = make_stream(sat_seconds, rate)
    served_sat, _ = run_served(world, s_sat, rate, slots)
    log("serving: served at %.0f req/s offered: %.1f req/s" % (rate, served_sat["throughput_req_s"]))
    plain_sat = run_plain(world, s_sat, rate)
    log("serving: plain at %.0f req/s offered: %.1f req/s" % (rate, plain_sat["throughput_req_s"]))
    r80 = 0.8 * min(served_sat["throughput_req_s"], rate)
    s80 = make_stream(seconds_80, r80, seed=6)
    served_80, _ = run_served(world, s80, r80, slots)
    log("serving: served at %.0f req/s offered: %.1f req/s" % (r80, served_80["throughput_req_s"]))
    plain_80 = run_plain(world, s80, r80)
    log("serving: plain at %.0f req/s offered: %.1f req/s" % (r80, plain_80["throughput_req_s"]))
    # both modes below saturation: 80 % of the plain mode's saturation throughput
    rp = 0.8 * min(plain_sat["throughput_req_s"], rate)
    sp = make_stream(seconds_80, rp, seed=7)
    served_p, last = run_served(world, sp, rp, slots)
    plain_p = run_plain(world, sp, rp)
    log("serving: at %.0f req/s offered: served %.1f, plain %.1f req/s"
        % (rp, served_p["throughput_req_s"], plain_p["throughput_req_s"]))
    out["saturation"] = {"served": served_sat, "plain": plain_sat}
    out["at_80pct_of_served_saturation"] = {"served": served_80, "plain": plain_80}
    out["at_80pct_of_plain_saturation"] = {"served": served_p, "plain": plain_p}
    out["consistency"] = consistency(world, last)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--sat-seconds", type=float, default=4.0)
    ap.add_argument("--seconds-80", type=float, default=5.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-out-gb", type=float, default=2.2)
    args = ap.parse_args()
    t = time.perf_counter()
    world = build_world(args.max_out_gb)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log("world ready in %.1f s" % (time.perf_counter() - t))
    print(json.dumps(measure(world, args.rate, args.sat_seconds, args.seconds_80, args.slots, log)), flush=True)


if __name__ == "__main__":
    main()
