"""Exact H + OPG of the 256-network batch on one GPU, in HBM-budgeted waves.

Usage: python -m paper_1905_05559_amd.batch_bench [--models M] [--budget-gb B] [--prec f32|f32_split]
       [--autotune]

Networks m = 0..M-1 follow the batch distribution (seed 4000 + m: T_1 ~ U{8..128},
1-2 tanh hidden layers of width U{16..256}, T_L ~ U{2..20}, N ~ U{100..5000}).  Their
H and OPG (FP32, P_m^2 entries each) total more than the device holds, so networks are
packed into waves whose outputs plus workspace fit in the budget; each wave is one
hess_batched call (persistent contraction launches, one per tile units bound, over all its
networks' tiles).
Outputs are views into one buffer allocated once; after a wave, every output is
reduced to (trace, Frobenius norm) and the buffer is reused by the next wave.  Prints one JSON line with P^2-entries/s and algorithmic TFLOP/s.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import api, workloads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--models", type=int, default=256)
    ap.add_argument("--budget-gb", type=float, default=160.0)
    ap.add_argument("--prec", default="f32", choices=["f32", "f32_split"])
    ap.add_argument("--autotune", action="store_true")
    args = ap.parse_args()
    dev = "cuda:0"
    ctx = api.Context(0)
    ctx.set_option("profile", 1)
    if args.autotune:
        ctx.set_option("autotune", 1)
    nets = []
    t = time.perf_counter()
    for m in range(args.models):
        w = workloads.batched_model(m)
        nets.append((w.P, w.N, api.MLP.from_workload(w, dtype=torch.float32), torch.from_numpy(w.X).to(dev),
                     torch.from_numpy(w.Y).to(dev)))
    print("generated %d networks in %.1f s" % (len(nets), time.perf_counter() - t), file=sys.stderr, flush=True)
    budget = args.budget_gb * (1 << 30)
    waves, cur, cur_bytes = [], [], 0.0
    for n in sorted(nets, key=lambda n: -n[0]):
        need = 2 * 4.0 * n[0] ** 2 * 1.25  # outputs plus a workspace allowance
        if cur and cur_bytes + need > budget:
            waves.append(cur)
            cur, cur_bytes = [], 0.0
        cur.append(n)
        cur_bytes += need
    if cur:
        waves.append(cur)
    summary = []
    # outputs of every wave are views into one buffer allocated once (no per-wave
    # allocation or release of tens of GB); the library workspace only grows
    cap = max(sum(2 * n[0] * n[0] for n in wv) for wv in waves)
    pool = torch.empty(cap, dtype=torch.float32, device=dev)
    # the library workspace sized once for the largest wave, before the timed loop (a
    # workspace that grows between waves costs an allocation of several GB inside it)
    ws_need = max(api.batched_workspace_size([n[2] for n in wv], [n[3] for n in wv], [n[4] for n in wv], ctx=ctx,
                                             prec=args.prec) for wv in waves)
    ctx.workspace(ws_need)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flops = 0.0
    entries = 0.0
    for i, wv in enumerate(waves):
        tw = time.perf_counter()
        outs, off = [], 0
        for n in wv:
            P2 = n[0] * n[0]
            outs.append((pool[off:off + P2].view(n[0], n[0]), pool[off + P2:off + 2 * P2].view(n[0], n[0])))
            off += 2 * P2
        Hs, Gs = api.hess_batched([n[2] for n in wv], [n[3] for n in wv], [n[4] for n in wv],
                                  outs_H=[o[0] for o in outs], outs_G=[o[1] for o in outs], ctx=ctx,
                                  prec=args.prec)
        torch.cuda.synchronize()
        t_call = time.perf_counter() - tw
        red = [(float(torch.trace(H)), float(H.norm()), float(torch.trace(G)), float(G.norm())) for H, G in zip(Hs, Gs)]
        t_red = time.perf_counter() - tw - t_call
        del Hs, Gs, outs
        dt = time.perf_counter() - tw
        for (P, N, _, _, _) in wv:
            flops += 2 * 2.0 * N * P * (P + 1) / 2
            entries += 2.0 * P * P
        summary.append({"wave": i, "networks": len(wv), "seconds": dt, "call_s": t_call, "reduce_s": t_red,
                        "P_max": wv[0][0]})
        print("wave %d: %d networks (P <= %d) in %.2f s" % (i, len(wv), wv[0][0], dt), file=sys.stderr, flush=True)
    total = time.perf_counter() - t0
    prof = ctx.profile()
    out = {"metric": "batched exact-H+OPG P^2-entries/s", "prec": args.prec, "autotune": args.autotune,
           "networks": len(nets), "waves": len(waves),
           "seconds": total, "p2_entries_per_s": entries / total, "algorithmic_tflops": flops / total / 1e12,
           "persistent_launch_tflops": {k: v["flops"] / v["ms"] / 1e9 for k, v in prof.items()
                                        if "persistent" in k and v["ms"] > 0},
           "persistent_launches_overall_tflops": (sum(v["flops"] for k, v in prof.items() if "persistent" in k)
                                                  / max(1e-9, sum(v["ms"] for k, v in prof.items()
                                                                  if "persistent" in k)) / 1e9),
           "kernel_ms": {k: round(v["ms"], 1) for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])},
           "wave_detail": summary}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
