#!/usr/bin/env python
"""Benchmark of the Hessian / OPG hot path on one MI355X.

Workload (default): the MNIST-shaped synthetic MLP [784, 100, 10], ReLU hidden
layer, N = 60000 examples, x_{n,j} = 0 with probability 0.8 else U[0,1), labels
uniform over 10 classes, Glorot-uniform weights, zero biases (P = 79510).  One
step runs every row of the hot path on that workload, with inputs already
resident in HBM:
  * the OPG  J^T J / N  (BF16 operands, FP32 accumulation), P x P FP32
  * the exact Hessian H, P x P FP32: FP32 operands and accumulation, each product from BF16
    MFMAs on compensated three-way splits of the operands (FP32-level error)
  * the 100 algebraically largest eigenpairs of H by block Lanczos (blocks of 16, FP32
    operator, FP64 re-orthogonalisation and Rayleigh-Ritz, tol 1e-5)
  * 512 dense Hessian-vector products (matrix-free R-operator, FP32 with split-BF16 GEMM products)
  * the damped curvature query for 1024 inputs against those eigenpairs (FP64)
value = 2 P^2 / step time  ("exact-H+OPG P^2-entries/s": P^2 entries of each matrix),
with the per-phase times, HVPs/s and query rates reported beside it.

The JSON line also carries the roofline of the dominant kernel (algorithmic flops
per launch / average launch time from HIP events on the library's stream), the
FP64 CPU oracle timed on a bounded sample of the same workload, and (after the timed
steps, skipped with --no-serving) the served-vs-plain request mix of
paper_1905_05559_amd/serve_bench.py against this network and the last step's
eigenpairs: p50/p99 per request type and throughput at saturation and at 80 % of each
mode's saturation, plus the alone-vs-mix consistency check.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense MFMA peaks; "bf16x6": FP32 products from six BF16 MFMA products each
# (compensated three-way split operands), so the BF16 peak divided by 6
PEAKS_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "bf16x6": 2500.0 / 6}
HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_dtype(name: str) -> str:
    for k in ("bf16x6", "bf16", "f64", "f32"):
        if "_" + k in name:
            return k
    return "f32"


def source_hash() -> str:
    """Hash of the contraction kernel sources (traffic counters are valid only for this hash)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_05559_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith("k_krg") or f == "mfma.h":
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """Measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled) for `kernel`, if the
    counters were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(w, seconds_hint: float):
    """The FP64 oracle on a bounded sample of the same workload.

    Sample: H columns [0, bh) (basis Hessian-vector products over all N examples) and
    the OPG tile rows [0, bg) x columns [0, cg) (from those columns of J).  Rate in
    P^2-entries/s for one H entry plus one OPG entry: 2 / (t_H/entry + t_OPG/entry)."""
    from oracle import mlp

    om = mlp.model_from(w.T, w.acts, w.W, w.b)
    X = w.X.astype(np.float64)
    Y = w.Y.astype(np.float64)
    P = mlp.num_params(w.T)
    bh = 48
    t0 = time.perf_counter()
    mlp.hessian_cols(om, X, Y, 0, bh, block=16)
    th = time.perf_counter() - t0
    bg, cg = 512, 4096
    t0 = time.perf_counter()
    mlp.opg_tile(om, X, Y, list(range(bg)), list(range(cg)))
    tg = time.perf_counter() - t0
    per_h = th / (bh * P)
    per_g = tg / (bg * cg)
    threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": 2.0 / (per_h + per_g),
        "unit": "P^2-entries/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "FP64 NumPy oracle, same workload: H columns 0..%d (basis HVPs over all N=%d examples, "
                  "%.1f s) and OPG tile %dx%d from J columns (%.1f s); rate = 2/(s per H entry + s per OPG "
                  "entry); host %s" % (bh, X.shape[0], th, bg, cg, tg, cpu),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mnist", choices=["mnist", "sigmoid64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--h-prec", default="f32_split", choices=["f32_split", "f32"],
                    help="products of the exact-H contractions and the HVP GEMMs: split-BF16 MFMA (default) or FP32 MFMA")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the measurements after the timed steps (HVP block sweep, other eigensolver "
                         "configurations, MFMA stream rate), e.g. for a profile of the steps alone")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the served-vs-plain request mix after the timed steps")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d requested)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_05559_amd import api, workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    w = workloads.mnist_relu() if args.workload == "mnist" else workloads.sigmoid_64()
    log("workload %s T=%s N=%d P=%d (generated in %.1f s)" % (w.name, w.T, w.N, w.P, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    model = api.MLP.from_workload(w, dtype=torch.float32)
    X = torch.from_numpy(w.X).to(dev, torch.float32)
    Y = torch.from_numpy(w.Y).to(dev, torch.float32)
    P = w.P

    ctx = api.Context(0)
    ctx.set_option("profile", 1)
    H = torch.empty((P, P), dtype=torch.float32, device=dev)
    G = torch.empty((P, P), dtype=torch.float32, device=dev)
    ws_bytes = max(api.workspace_size("exact", model, X, Y, "f32", ctx=ctx),
                   api.workspace_size("opg", model, X, Y, "bf16", ctx=ctx),
                   api.workspace_size("hvp", model, X, Y, "f32", arg=512, ctx=ctx))
    ctx.workspace(ws_bytes)
    log("outputs 2 x %.1f GB, workspace %.2f GB" % (P * P * 4 / 1e9, ws_bytes / 1e9))

    K, B, NQ = 100, 512, 1024
    V = torch.from_numpy(workloads.gaussian_directions(B, P, 7)).to(dev)
    HV = torch.empty_like(V)
    Xq = torch.from_numpy(workloads.queries_like_mnist(NQ, 11, T1=w.T[0])).to(dev)
    LZ_BLOCK = 16
    eopts = api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=1, max_iter=200, method="lanczos",
                         block=LZ_BLOCK)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    phase_ms = {"opg": 0.0, "exact_H": 0.0, "topk": 0.0, "hvp": 0.0, "predvar": 0.0}
    eig_info = {}
    pairs = {}

    def step(record=False):
        s = ctx.stream
        ev[0].record(s)
        api.hess_opg(model, X, Y, "bf16", out=G, ctx=ctx)
        ev[1].record(s)
        api.hess_exact(model, X, Y, args.h_prec, out=H, ctx=ctx)
        ev[2].record(s)
        lam, Q, info, st = api.hess_topk_eig(None, None, None, K, eopts, ctx=ctx)
        ev[3].record(s)
        api.hess_hvp(model, X, Y, V, args.h_prec, out=HV, ctx=ctx)
        ev[4].record(s)
        delta = max(1e-3, 1e-3 - float(lam.min()))  # keeps lambda_k + delta > 0
        api.hess_predvar(model, lam, Q, delta, Xq, ctx=ctx)
        ev[5].record(s)
        if record:
            torch.cuda.synchronize()
            for i, k in enumerate(("opg", "exact_H", "topk", "hvp", "predvar")):
                phase_ms[k] += ev[i].elapsed_time(ev[i + 1])
            eig_info.update(info)
        pairs["lam"], pairs["Q"] = lam, Q

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        log("warmup step %d: %.3f s" % (i, time.perf_counter() - t))
    torch.cuda.synchronize()
    ctx.profile_reset()
    s = ctx.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(args.steps):
        step(record=True)
        log("step %d done" % i)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    prof = ctx.profile()
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
        log("  %-24s launches %5d  total %9.2f ms  %8.2f TFLOP/s  %8.1f GB/s" % (
            k, v["launches"], v["ms"], v["flops"] / v["ms"] / 1e9 if v["ms"] else 0,
            v["bytes"] / v["ms"] / 1e6 if v["ms"] else 0))
    dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    dname, d = dom
    dt = kernel_dtype(dname)
    achieved = d["flops"] / d["ms"] / 1e9  # TFLOP/s
    traffic = load_traffic(dname)
    roofline = {
        "bound": "mfma", "kernel": dname, "dtype": dt,
        "achieved": round(achieved, 3), "peak": PEAKS_TFLOPS[dt], "unit": "TFLOP/s",
        "frac": round(achieved / PEAKS_TFLOPS[dt], 4),
        "avg_launch_ms": round(d["ms"] / d["launches"], 4),
        "flops_per_launch": d["flops"] / d["launches"],
        "traffic": traffic,
        "share_of_step": round(d["ms"] / args.steps / ms, 4),
    }
    value = 2.0 * P * P / (ms / 1e3)
    ph = {k: v / args.steps for k, v in phase_ms.items()}
    log("phases (ms/step): %s" % json.dumps({k: round(v, 2) for k, v in ph.items()}))
    out = {
        "metric": "exact-H+OPG P^2-entries/s",
        "value": value,
        "unit": "P^2-entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operands via split-bf16 MFMA products, f32 accumulate (H, HVP) + f32 (eigensolver operator) "
                 "+ bf16->f32 (OPG) + f64 (re-orthogonalisation, Rayleigh-Ritz, query)",
        "data": "synthetic",
        "config": {"workload": w.name, "T": w.T, "N": w.N, "P": P,
                   "step": "OPG (BF16 MFMA, FP32 acc) + exact H (FP32, split-BF16 MFMA products), P x P each; top-100 eigenpairs "
                           "of H (block Lanczos, block 16, FP32 operator, FP64 RR, tol 1e-5); 512 dense HVPs "
                           "(FP32, split-BF16 GEMM products); damped query for 1024 inputs (FP64); inputs resident in HBM"},
        "phases_ms": {k: round(v, 3) for k, v in ph.items()},
        "hvps_per_s": {"dense_B512": B / (ph["hvp"] / 1e3), "basis_via_exact_H": P / (ph["exact_H"] / 1e3)},
        "opg_p2_entries_per_s": P * P / (ph["opg"] / 1e3),
        "exact_h_p2_entries_per_s": P * P / (ph["exact_H"] / 1e3),
        "topk": {"K": K, "method": "lanczos", "block": LZ_BLOCK, "restarts": eig_info.get("iters"),
                 "block_applies": eig_info.get("applies"),
                 "vectors_applied": (eig_info.get("applies") or 0) * LZ_BLOCK,
                 "max_rel_residual": eig_info.get("max_rel_residual")},
        "predvar_queries_per_s": NQ / (ph["predvar"] / 1e3),
        "roofline": roofline,
        "kernels": {k: {"launches": v["launches"], "ms_per_step": v["ms"] / args.steps,
                        "tflops": v["flops"] / v["ms"] / 1e9 if v["ms"] else 0.0} for k, v in prof.items()},
    }
    # Dense HVP throughput at several block sizes (outside the timed steps), over all N
    # examples, median of 3 after one warm-up: "dense_B<B>" applies a prepared operator
    # (per-example passes done once, hess_hvp_prepare); "dense_B<B>_call" is one complete
    # hess_hvp call per block (validation, input check and per-example passes included).
    def timed(fn):
        fn()
        times = []
        for _ in range(3):
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(ctx.stream)
            fn()
            a1.record(ctx.stream)
            torch.cuda.synchronize()
            times.append(a0.elapsed_time(a1))
        return sorted(times)[1] / 1e3

    if not args.no_side:
        op = api.HvpOperator(model, X, Y, args.h_prec, max_B=B, ctx=ctx)
        rates = {}
        for Bs in (1, 8, 64, 512):
            Vb = V[:Bs].contiguous()
            HVb = torch.empty_like(Vb)
            rates["dense_B%d" % Bs] = Bs / timed(lambda: op.apply(Vb, out=HVb))
            if Bs < B:
                rates["dense_B%d_call" % Bs] = Bs / timed(lambda: api.hess_hvp(model, X, Y, Vb, args.h_prec, out=HVb,
                                                                               ctx=ctx))
        op.close()
        # the same top-100 problem by the other eigensolver configurations (outside the timed steps)
        for tag, oo in (("subspace_iteration", api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=1,
                                                             oversample=12, max_iter=200)),
                        ("lanczos_block32", api.eig_opts(which="H", source="dense", M=H, tol=1e-5, seed=1,
                                                          max_iter=200, method="lanczos", block=32))):
            out["topk"]["ms_" + tag] = round(1e3 * timed(lambda: api.hess_topk_eig(None, None, None, K, oo, ctx=ctx)), 2)
        # matrix-free operator (R-operator HVPs over all N examples, FP32), one call each
        for tag, oo in (("matrix_free_lanczos_block16", api.eig_opts(which="H", source="matrix_free", prec="f32",
                                                                      tol=1e-5, seed=1, max_iter=200,
                                                                      method="lanczos", block=16)),
                        ("matrix_free_subspace_iteration", api.eig_opts(which="H", source="matrix_free", prec="f32",
                                                                         tol=1e-5, seed=1, oversample=12,
                                                                         max_iter=200))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, inf, st = api.hess_topk_eig(model, X, Y, K, oo, ctx=ctx, raise_on_noconv=False)
            torch.cuda.synchronize()
            out["topk"]["ms_" + tag] = round(1e3 * (time.perf_counter() - t0), 2)
            out["topk"]["info_" + tag] = {"status": st, **{k: inf[k] for k in ("iters", "applies", "max_rel_residual")}}
            log("top-%d %s: %.1f ms %s %s" % (K, tag, out["topk"]["ms_" + tag], inf, st))
        rates["dense_B%d_call" % B] = out["hvps_per_s"].pop("dense_B%d" % B)
        out["hvps_per_s"].update(rates)
        # the same H with plain FP32 MFMA products, one call
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.hess_exact(model, X, Y, "f32", out=H, ctx=ctx)
        torch.cuda.synchronize()
        out["exact_h_f32_mfma_ms"] = round(1e3 * (time.perf_counter() - t0), 1)
        # sustained rate of the dominant kernel's MFMA instruction in a register-only stream
        # (per FP32 product for the split form: six BF16 products each)
        stream_kind = {"f32": "f32_16x16x4", "bf16": "bf16_16x16x32", "bf16x6": "bf16_16x16x32",
                       "f64": "f64_16x16x4"}[roofline["dtype"]]
        srate = ctx.mfma_stream_rate(stream_kind) / (6.0 if roofline["dtype"] == "bf16x6" else 1.0)
        out["roofline"]["mfma_stream_tflops"] = round(srate, 2)
        out["roofline"]["frac_of_stream"] = round(roofline["achieved"] / srate, 4)
        log("hvps/s %s; MFMA stream %s %.1f TFLOP/s" % (json.dumps({k: round(v, 1) for k, v in out["hvps_per_s"].items()}),
                                                        stream_kind, srate))
    del H, G, V, HV
    ctx.release_workspace()
    torch.cuda.empty_cache()
    if not args.no_serving and args.workload == "mnist":
        # Served vs plain request mix against the resident network and the eigenpairs of the
        # last step (outside the timed steps); see paper_1905_05559_amd/serve_bench.py
        from paper_1905_05559_amd import serve_bench
        t = time.perf_counter()
        world = serve_bench.World(model, X, Y, pairs["lam"], pairs["Q"])
        out["serving"] = serve_bench.measure(world, log=log)
        del world
        torch.cuda.empty_cache()
        log("serving block took %.1f s" % (time.perf_counter() - t))
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(w, 20.0)
        log("cpu baseline took %.1f s" % (time.perf_counter() - t))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
