"""Benchmark of the parallel iDMRG hot path on one MI355X.

Workload: spin-1/2 Heisenberg model on the YC8 kagome cylinder, 12-site unit
cell (6 superblocks per iteration), U(1) S^z blocks, m kept states (default
2048).  A "step" is one unit-cell step (one iteration n of the parallel
iDMRG): the batched prediction, Lanczos solve, truncation and both
environment updates of all six superblocks.

Protocol: the chain of iterations is first grown (untimed) to n = prefill so
that m is saturated, then `warmup` steps run untimed, then exactly `steps`
steps are timed between two device synchronisations.  During the timed steps
every library launch is bracketed by HIP events on the library's stream; the
H_eff matvec throughput is the algorithmic flop count of the matvecs (from the
U(1) block lists) divided by their summed kernel time.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6}   # TFLOP/s, dense MFMA, MI355X


def cpu_baseline(d, budget_s=30.0):
    """Time the oracle's H_eff matvec on superblock 1 of the current state (host cores)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import layout, u1
    from paper_1606_06790_amd import lib
    h = d.problems(d.n + 1)[0]
    A, B = h["left"], h["right"]
    W1, W2 = h["w1"], h["w2"]
    dl, dr = np.array(W1.ql), np.array(W2.qr)
    L = layout.flat_to_envL(h["L"].cpu().numpy(), A, dl)
    R = layout.flat_to_envR(h["R"].cpu().numpy(), B, dr)
    x = np.random.default_rng(0).standard_normal(layout.psi_size(A, B, W1.qp))
    psi = layout.flat_to_psi(x, A, B, W1.qp)
    flops, _ = lib.heff_work(h)
    t0 = time.perf_counter()
    u1.heff_apply(L, W1.w, W2.w, R, psi, A, B, W1.qp, dl, dr)
    t = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return dict(value=flops / t / 1e12, unit="TFLOP/s", cores=threads, kind="oracle",
                sample=f"one H_eff matvec of superblock 1 at iteration {d.n + 1} "
                       f"(N={layout.psi_size(A, B, W1.qp)}, {flops:.3e} flops, {t:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prefill", type=int, default=11)
    ap.add_argument("--m", type=int, default=2048)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3"])
    ap.add_argument("--workload", default="yc8")
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads
    from paper_1606_06790_amd.driver import IDMRG

    cfg = workloads.workload(a.workload, m=a.m)
    d = IDMRG(cfg, prec=a.prec)
    t_pre = time.perf_counter()
    while d.n < a.prefill:
        d.step()
    for _ in range(a.warmup):
        d.step()
    t_pre = time.perf_counter() - t_pre
    d.ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [d.step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = d.ctx.profile_get()
    d.ctx.profile(False)
    ms_step = (t1 - t0) * 1e3 / a.steps
    mv_fl = prof["heff_gemm1"][2] + prof["heff_gemm2"][2] + prof["heff_mix"][2]
    mv_ms = prof["heff_gemm1"][1] + prof["heff_gemm2"][1] + prof["heff_mix"][1] + prof["convert"][1]
    tflops = mv_fl / (mv_ms * 1e-3) / 1e12
    g_fl = prof["heff_gemm1"][2] + prof["heff_gemm2"][2]
    g_ms = prof["heff_gemm1"][1] + prof["heff_gemm2"][1]
    g_launch = prof["heff_gemm1"][0] + prof["heff_gemm2"][0]
    mult = 3.0 if a.prec == "bf16x3" else 1.0       # bf16 MFMA products per FP64-equivalent product
    achieved = mult * g_fl / (g_ms * 1e-3) / 1e12
    steps = [s for s in d.steps if s["n"] > d.n - a.steps]
    out = {
        "metric": "H_eff matvec TFLOP/s + s per unit-cell step, kagome YC8 m=2048; mixed vs FP64",
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32+f64", "bf16x3": "bf16x3+f64"}[a.prec],
        "data": "synthetic",
        "config": {"workload": f"{a.workload}_heisenberg_m{a.m}_u1", "superblocks": d.half,
                   "iterations_timed": [r["n"] for r in recs], "prefill": a.prefill, "matvec_prec": a.prec},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[a.prec], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK[a.prec], 4), "traffic": None,
                     "kernel": "grouped H_eff GEMM (stage 1 + stage 2)",
                     "avg_launch_ms": round(g_ms / max(g_launch, 1), 4)},
        "breakdown_ms_per_step": {k: round(v[1] / a.steps, 2) for k, v in prof.items()},
        "lanczos_iters": [s["iters"] for s in steps],
        "e_site": [round(s["e_site"], 10) for s in steps],
        "residual_max": max(s["residual"] for s in steps),
        "prefill_s": round(t_pre, 1),
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
