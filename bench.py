"""Benchmark of the parallel iDMRG hot path on one MI355X.

Workload: spin-1/2 Heisenberg model on the YC8 kagome cylinder, 12-site unit
cell (6 superblocks per iteration), U(1) S^z blocks, m kept states (default
2048).  A "step" is one unit-cell step (one iteration n of the parallel
iDMRG): the batched prediction, Lanczos solve, truncation and both
environment updates of all six superblocks.

Protocol: the chain of iterations is grown (untimed, FP64) to n = prefill so
that m is saturated, and that state is kept.  Then, for FP64 and for the
mixed-precision matvec in turn, starting from the kept state: `warmup`
steps untimed, then exactly `steps` steps timed between two device
synchronisations.  Both precisions therefore solve the same iterations from
the same state, which gives a like-for-like speed-up and the energy
difference per result.  ms_per_step is that wall clock as in production (no
per-launch events, direct launches).  The same
steps are then run again from the same state with every library launch
bracketed by HIP events on the library's stream; the H_eff matvec throughput
is the algorithmic flop count of the matvecs (from the U(1) block lists)
divided by their summed kernel time in that run.

Prints one JSON line on stdout (value = matvec TFLOP/s of the mixed path,
ms_per_step = its seconds per unit-cell step; the FP64 figures sit under
"fp64"), and one progress line per unit-cell step on stderr.
--gpus N with N > 1 exits: the benchmark runs on one GPU.
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

# Dense MFMA peaks of MI355X (TFLOP/s).  The split-bf16 policy does three bf16
# products per FP64-equivalent product, so its ceiling for algorithmic flops is
# the bf16 peak / 3.
PEAK = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6 / 3.0}
LATTICE = {"yc8": "kagome YC8", "yc4": "square YC4", "chain": "chain"}
MATVEC = ["heff_gemm1", "heff_gemm2", "heff_mix", "heff_gemm1_lo", "heff_gemm2_lo", "heff_mix_lo", "convert"]


def cpu_baseline(d, budget_s=10.0, budget_1t_s=6.0):
    """The oracle's H_eff matvec on superblock 1 of the current state (host cores), repeated for ~budget_s with
    every BLAS thread and for ~budget_1t_s with one; plus one oracle unit-cell step of the random-bond chain
    (m = 256) beside the GPU's step of the same iteration."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
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

    def rate(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            u1.heff_apply(L, W1.w, W2.w, R, psi, A, B, W1.qp, dl, dr)
            reps += 1
            t = time.perf_counter() - t0
            if t >= budget:
                return reps, t

    reps, t = rate(budget_s)
    info = threadpool_info()
    threads = max([p.get("num_threads", 1) for p in info] + [1])
    blas = [f"{p.get('internal_api')} {p.get('version')} ({p.get('threading_layer', '-')}, {p.get('num_threads')} threads)"
            for p in info if p.get("user_api") == "blas"]
    with threadpool_limits(1):
        reps1, t1 = rate(budget_1t_s)
    note("cpu baseline: timing one oracle unit-cell step of the random-bond chain")
    return dict(value=round(reps * flops / t / 1e12, 6), unit="TFLOP/s", cores=threads, kind="oracle",
                sample=f"{reps} H_eff matvec(s) of superblock 1 at iteration {d.n + 1} "
                       f"(N={layout.psi_size(A, B, W1.qp)}, {flops:.3e} flops each) in {t:.1f} s",
                value_1thread=round(reps1 * flops / t1 / 1e12, 6),
                sample_1thread=f"{reps1} of the same matvecs with one BLAS thread in {t1:.1f} s",
                blas=blas, step=oracle_step_comparison())


def oracle_step_comparison(wl="random_chain", m=256, n=17):
    """Seconds of one unit-cell step (iteration n, all superblocks) of the oracle and of the GPU path (FP64,
    batched) on the same workload.  The oracle runs its own trajectory from n = 1 (untimed up to n - 1); the GPU
    runs its own from n = 1 as well, and its step n is timed between device synchronisations."""
    import torch
    import workloads
    from oracle import idmrg as oidmrg
    from paper_1606_06790_amd.driver import IDMRG
    cfg = workloads.workload(wl, m=m)
    secs = []
    oidmrg.run(cfg, mode="u1", n_max=n, log=lambda r: secs.append(r["seconds"]) if r["n"] == n else None)
    d = IDMRG(cfg, prec="f64")
    d.run(n - 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.step()
    torch.cuda.synchronize()
    g = time.perf_counter() - t0
    o = sum(secs)
    return dict(workload=f"{wl}_heisenberg_m{m}_u1", iteration=n, superblocks=len(secs), oracle_s=round(o, 4),
                gpu_f64_s=round(g, 5), gpu_speedup=round(o / g, 1))


def prediction_effect(d, snap):
    """Lanczos iterations per FP64 solve of iteration snap.n + 1 from the kept state, with and without the start
    vector of Eq. (10) (random start otherwise), under the full stop rule (|dtheta| <= tol_E and residual <= tol_res)
    and under the |dtheta| rule alone (the rule the paper's iteration counts compare with)."""
    out = {}
    keep = (d.prec, d.predict, dict(d.cfg))
    for label, predict, dtheta_only in (("with_prediction", True, False), ("with_prediction_dtheta_rule", True, True),
                                        ("random_start", False, False), ("random_start_dtheta_rule", False, True)):
        d.restore(snap)
        d.prec, d.predict = "f64", predict
        d.cfg = dict(keep[2], tol_res=1e300 if dtheta_only else keep[2]["tol_res"])
        d.step()
        recs = [s for s in d.steps if s["n"] == d.n]
        out[label] = dict(iters=[s["iters"] for s in recs], converged=[s["converged"] for s in recs],
                          fidelity_error=[s["fidelity"] for s in recs])
        note(f"prediction effect: {label} at n={d.n}: {out[label]['iters']}")
    d.prec, d.predict, d.cfg = keep
    d.restore(snap)
    mean = lambda k: sum(out[k]["iters"]) / len(out[k]["iters"])
    out["ratio_random_over_predicted"] = round(mean("random_start") / mean("with_prediction"), 3)
    out["ratio_random_over_predicted_dtheta_rule"] = round(
        mean("random_start_dtheta_rule") / mean("with_prediction_dtheta_rule"), 3)
    out["iteration"] = d.n + 1
    out["paper"] = "about 40 iterations with prediction, about 3x as many without (YC8 kagome, its Sec. 4)"
    return out


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class marker:
    """A named range on the roctx marker track (rocprofv3 --marker-trace), so that a kernel trace can be cut
    into the timed regions.  Costs one host call at each end, outside the timed work."""

    def __init__(self, label):
        self.label = label

    def __enter__(self):
        import torch
        torch.cuda.nvtx.range_push(self.label)

    def __exit__(self, *exc):
        import torch
        torch.cuda.nvtx.range_pop()


def wall(d, steps, warmup, label, profile=False):
    """warmup + timed unit-cell steps from the current state; (seconds per step, step records)."""
    import torch
    for k in range(warmup):
        d.step()
        note(f"{label}: warmup step {k + 1}/{warmup} done (n={d.n})")
    if profile:
        d.ctx.profile(True)
    torch.cuda.synchronize()
    with marker(f"timed:{label}"):
        t0 = time.perf_counter()
        for k in range(steps):
            d.step()
            note(f"{label}: timed step {k + 1}/{steps} done (n={d.n})")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    return (t1 - t0) / steps, [s for s in d.steps if s["n"] > d.n - steps]


def timed(d, prec, steps, warmup):
    """The timed steps at one matvec precision, twice from the same state: first as in production
    (no per-launch events) for the wall clock, then
    with every launch bracketed by HIP events for the kernel times."""
    d.prec = prec
    snap = d.snapshot()
    t_run, recs = wall(d, steps, warmup, prec)
    d.restore(snap)
    t_prof, recs_p = wall(d, steps, warmup, prec + " (events)", profile=True)
    prof = d.ctx.profile_get()
    d.ctx.profile(False)
    mv_fl = sum(prof[k][2] for k in MATVEC)
    mv_ms = sum(prof[k][1] for k in MATVEC)
    return dict(prec=prec, ms_per_step=t_run * 1e3, ms_per_step_events=t_prof * 1e3,
                matvec_tflops=mv_fl / (mv_ms * 1e-3) / 1e12, prof=prof, recs=recs,
                identical=[r["energy"] for r in recs] == [r["energy"] for r in recs_p])


def microbench(a):
    """The H_eff matvec microbenchmark: the Heisenberg chain MPO (D = 5, d = 2) on Gaussian FP64 environments and
    state, m = 256, 512, 1024, U(1)-blocked (the Gaussian sector profile) and dense (one sector), in FP64, FP32 and
    split-bf16.  Kernel time by HIP events over `reps` calls after one untimed call; the FP32 and split-bf16 results
    against the FP64 one (|y - y64| / |y64|, 2-norm).  Prints one JSON line."""
    import torch
    import workloads
    from paper_1606_06790_amd import lib, models
    cfg = workloads.workload("chain")
    W = models.heisenberg_mpo(cfg["bonds"], cfg["ell"])
    ctx = lib.Context(0)
    dev = lambda x: torch.from_numpy(x).to("cuda")
    reps, rows = 20, []
    for m in (256, 512, 1024):
        for kind in ("u1", "dense"):
            if kind == "u1":
                qs, ds = workloads.sector_dims(m)
                A = B = list(zip(qs, ds))
                w1, w2 = W[0], W[1]
            else:
                A = B = [(0, m)]
                z = [0] * W[0].w.shape[0]
                w1, w2 = lib.Mpo(W[0].w, z, z, [0, 0]), lib.Mpo(W[1].w, z, z, [0, 0])
            nL, nR, nx = lib.envL_size(A, w1.ql), lib.envR_size(B, w2.qr), lib.psi_size(A, B, w1.qp)
            prob = dict(left=A, right=B, w1=w1, w2=w2, L=dev(workloads.gaussian(nL, 2, m, int(kind == "u1"), 1)),
                        R=dev(workloads.gaussian(nR, 2, m, int(kind == "u1"), 2)))
            x = dev(workloads.gaussian(nx, 2, m, int(kind == "u1"), 3))
            flops = lib.heff_work(prob)[0]
            y64 = None
            for prec in ("f64", "f32", "bf16x3"):
                y = torch.empty_like(x)
                lib.heff_apply(ctx, [prob], [x], [y], prec)
                ctx.profile(True)
                for _ in range(reps):
                    lib.heff_apply(ctx, [prob], [x], [y], prec)
                prof = ctx.profile_get()
                ctx.profile(False)
                ms = sum(prof[k][1] for k in MATVEC) / reps
                # the same calls as in production (no per-launch events), for a kernel trace of their launch gaps
                torch.cuda.synchronize()
                with marker(f"timed:micro_m{m}_{kind}_{prec}"):
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        lib.heff_apply(ctx, [prob], [x], [y], prec)
                    torch.cuda.synchronize()
                    wall_ms = (time.perf_counter() - t0) * 1e3 / reps
                if prec == "f64":
                    y64 = y.clone()
                err = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))
                rows.append(dict(m=m, blocks=kind, prec=prec, N=nx, flops=flops, kernel_ms=round(ms, 4),
                                 wall_ms_per_call=round(wall_ms, 4),
                                 tflops=round(flops / (ms * 1e-3) / 1e12, 2), rel_err_vs_f64=err))
                note(f"microbench m={m} {kind} {prec}: {rows[-1]['tflops']} TFLOP/s")
    print(json.dumps({"microbench": "H_eff matvec, Heisenberg chain MPO D=5, Gaussian environments and state",
                      "reps": reps, "rows": rows}), flush=True)


def batching(a):
    """Seconds per unit-cell step of one workload solved three ways from the same state: batched
    with direct launches (production), batched with graph-replayed Lanczos chunks, and one
    library call per superblock (direct launches).  Prints one JSON line."""
    import workloads
    from paper_1606_06790_amd.driver import IDMRG
    cfg = workloads.workload(a.workload, m=a.m)
    d = IDMRG(cfg)
    while d.n < a.prefill:
        d.step()
        note(f"prefill: n={d.n}/{a.prefill} done")
    snap = d.snapshot()
    out = {}
    for name, batched, graph in (("batched_direct", True, False), ("batched_graph", True, True),
                                 ("one_call_per_superblock", False, False)):
        d.restore(snap)
        d.batched, d.graph = batched, graph
        t, recs = wall(d, a.steps, a.warmup, name)
        out[name] = dict(ms_per_step=round(t * 1e3, 3), e_site=[round(r["e_site"], 12) for r in recs],
                         lanczos_iters=[r["iters"] for r in recs])
    e0 = [r for r in out["batched_direct"]["e_site"]]
    print(json.dumps({"workload": f"{a.workload}_heisenberg_m{a.m}_u1", "prec": d.prec, "superblocks": d.half,
                      "steps": a.steps, "warmup": a.warmup, "prefill": a.prefill, "runs": out,
                      "same_energies": all(v["e_site"] == e0 for v in out.values()),
                      "batched_speedup_vs_one_call_per_superblock": round(
                          out["one_call_per_superblock"]["ms_per_step"] / out["batched_direct"]["ms_per_step"], 3),
                      "graph_speedup_vs_direct": round(
                          out["batched_direct"]["ms_per_step"] / out["batched_graph"]["ms_per_step"], 3)}),
          flush=True)


def launch_gaps(directory):
    """Where the GPU idles inside each timed region of a kernel trace.

    Reads the CSV output of `rocprofv3 --kernel-trace --marker-trace --output-format csv` (run on this file) and,
    for every marker range named "timed:...", takes the kernels that start inside it:
      busy  = the union of their execution intervals;
      gaps  = idle time between one kernel's end and the next one's start (launch latency and host work);
      lead  = from the range start to the first kernel, and tail = from the last kernel to the range end (host
              work before the first launch and the final synchronisation).
    Prints one JSON line with, per range, its length, kernel count, busy share and gap statistics."""
    import csv
    import glob

    def rows(pattern):
        out = []
        for path in glob.glob(os.path.join(directory, "**", pattern), recursive=True):
            with open(path, newline="") as f:
                out.extend(csv.DictReader(f))
        return out

    kern = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows("*kernel_trace.csv"))
    ranges = []
    for r in rows("*marker_api_trace.csv"):
        label = next((v for v in r.values() if isinstance(v, str) and v.startswith("timed:")), None)
        if label:
            ranges.append((label[6:], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out = []
    for label, t0, t1 in sorted(ranges, key=lambda x: x[1]):
        ks = [k for k in kern if t0 <= k[0] < t1]
        if not ks:
            continue
        busy, gaps, end = 0, [], ks[0][0]
        for s, e in ks:
            if s > end:
                gaps.append(s - end)
            busy += max(0, e - max(s, end))
            end = max(end, e)
        span = t1 - t0
        gaps.sort()
        out.append(dict(range=label, span_ms=round(span * 1e-6, 3), kernels=len(ks),
                        busy_share=round(busy / span, 4), gap_share=round(sum(gaps) / span, 4),
                        lead_us=round((ks[0][0] - t0) * 1e-3, 1), tail_us=round((t1 - end) * 1e-3, 1),
                        gap_median_us=round(gaps[len(gaps) // 2] * 1e-3, 2) if gaps else 0.0,
                        gap_p90_us=round(gaps[int(len(gaps) * 0.9)] * 1e-3, 2) if gaps else 0.0,
                        gaps_over_100us_ms=round(sum(g for g in gaps if g > 100_000) * 1e-6, 3)))
    print(json.dumps({"launch_gaps": directory, "ranges": out}), flush=True)


def _csv_rows(directory, pattern):
    import csv
    import glob
    out = []
    for path in sorted(glob.glob(os.path.join(directory, "**", pattern), recursive=True)):
        with open(path, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def stats_summary(directory, top=24):
    """Markdown table of a `rocprofv3 --kernel-trace --stats --output-format csv` run under DIR (its
    kernel_stats.csv): calls, total and average time and share per kernel."""
    rows = _csv_rows(directory, "*kernel_stats.csv")
    tot_ns = sum(float(r["TotalDurationNs"]) for r in rows)
    calls = sum(int(r["Calls"]) for r in rows)
    print(f"Total kernel time {tot_ns * 1e-9:.2f} s over {calls} dispatches.\n")
    print("| Kernel | Calls | Total ms | Avg ms | % |\n|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        print(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.1f} | "
              f"{float(r['AverageNs']) * 1e-6:.4f} | {100 * float(r['TotalDurationNs']) / tot_ns:.2f} |")


def traffic_summary(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, top=18):
    """Markdown summary of HBM traffic per kernel from four `rocprofv3 --pmc <counter> --output-format csv` runs:
    FETCH_SIZE and WRITE_SIZE over the benchmark, and the same two counters over `--copy-calibration` (a plain
    device copy of known size, which gives the counter's bytes per KiB read).  Ends with the records that
    measured_traffic() reads for the split-bf16 GEMM stages, stamped with the current sources hash."""
    import hashlib
    from collections import defaultdict

    def per_kernel(directory, counter):
        acc = defaultdict(lambda: [0, 0.0])
        for r in _csv_rows(directory, "*counter_collection.csv"):
            if r["Counter_Name"] == counter:
                a = acc[r["Kernel_Name"]]
                a[0] += 1
                a[1] += float(r["Counter_Value"])
        return {k: (n, v / n) for k, (n, v) in acc.items()}

    copy_bytes = 268435456
    cf = max(per_kernel(cal_fetch_dir, "FETCH_SIZE").items(), key=lambda kv: kv[1][0] * kv[1][1])
    cw = max(per_kernel(cal_write_dir, "WRITE_SIZE").items(), key=lambda kv: kv[1][0] * kv[1][1])
    ff = cf[1][1] * 1024 / copy_bytes
    fw = cw[1][1] * 1024 / copy_bytes
    print(f"* FETCH_SIZE read {cf[1][1]:.1f} KiB for {copy_bytes // 1024} KiB moved (`{cf[0][:60]}`): factor {ff:.5f} "
          f"(bytes = KiB x 1024 / {ff:.5f})")
    print(f"* WRITE_SIZE read {cw[1][1]:.1f} KiB for {copy_bytes // 1024} KiB moved: factor {fw:.5f}\n")
    fe, wr = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    rows = []
    for k in fe:
        n, f = fe[k]
        w = wr.get(k, (0, 0.0))[1]
        rows.append((k, n, f, w, f * 1024 / ff + w * 1024 / fw))
    rows.sort(key=lambda r: -r[1] * r[4])
    print("| Kernel | Dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes/dispatch (calibrated) |")
    print("|---|---|---|---|---|")
    for k, n, f, w, b in rows[:top]:
        print(f"| `{k[:90]}` | {n} | {f:.1f} | {w:.1f} | {b:.4e} |")
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    print("\nRecords read by bench.py for the roofline kernel (split-bf16 GEMM stage 1 and stage 2, the kernel variant "
          "with the most dispatches):\n")
    import re
    for cls, stage in (("heff_gemm1_lo", "0"), ("heff_gemm2_lo", "1")):
        pat = re.compile(r"gemm_bf16x3(_\w+)?_kernel<" + stage + r"[,>]")
        cand = [r for r in rows if pat.search(r[0].replace(" ", ""))]
        if cand:
            k, n, f, w, b = max(cand, key=lambda r: r[1])
            name = k.replace("void ", "").replace("idmrg::(anonymous namespace)::", "").split("(")[0]
            print(f"traffic-record: class={cls} kernel={name} bytes_per_launch={b:.6e} sources_sha256={h.hexdigest()}\n")
    print(f"`sources_sha256` is the SHA-256 of {', '.join(TRAFFIC_SOURCES)} (concatenated) when the counters were "
          "taken; bench.py reports the traffic only while it still matches.")


MFMA_PEAK_TFLOPS = {"BF16": 2500.0, "F16": 2500.0, "F32": 157.3, "F64": 78.6}


PCT_METRICS = ("MfmaUtil", "LdsUtil", "LDSBankConflict")   # rocprofv3 derived metrics in percent per dispatch


def mfma_counters(directories):
    """MFMA and LDS utilisation per kernel from `rocprofv3 --pmc ... --kernel-trace --output-format csv` runs (one
    directory per counter pass; the passes are merged by kernel name).

    Per dispatch: MFMA flops executed = 512 x SQ_INSTS_VALU_MFMA_MOPS_<type> (the counter counts units of 512
    flops, padding of ragged tiles included); rate = flops / kernel duration; share of the type's dense peak.
    The derived metrics MfmaUtil (MFMA-busy SIMD cycles over active cycles x SIMDs), LdsUtil and LDSBankConflict
    (percent) are averaged weighted by duration; SQ_WAIT_ANY, SQ_WAIT_INST_LDS and SQ_LDS_DATA_FIFO_FULL are
    reported per wave cycle (over SQ_WAVE_CYCLES of the same pass).  Prints one JSON line."""
    import csv
    import glob
    from collections import defaultdict

    if isinstance(directories, str):
        directories = [directories]
    merged = {}
    for directory in directories:
        def rows(pattern):
            out = []
            for path in glob.glob(os.path.join(directory, "**", pattern), recursive=True):
                with open(path, newline="") as f:
                    out.extend(csv.DictReader(f))
            return out

        dur = {}
        for r in rows("*kernel_trace.csv"):
            dur[r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per = defaultdict(lambda: defaultdict(float))
        name = {}
        for r in rows("*counter_collection.csv"):
            did = r["Dispatch_Id"]
            per[did][r["Counter_Name"]] += float(r["Counter_Value"])
            name[did] = r["Kernel_Name"]
            if did not in dur and r.get("Start_Timestamp") and r.get("End_Timestamp"):
                dur[did] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        agg = defaultdict(lambda: defaultdict(float))
        for did, c in per.items():
            if did not in dur or dur[did] <= 0:
                continue
            a = agg[name[did]]
            a["dispatches"] += 1
            a["ns"] += dur[did]
            for k, v in c.items():
                if k in PCT_METRICS:
                    a[k + "_ns"] += v * dur[did]
                else:
                    a[k] += v
        for kname, a in agg.items():
            row = merged.setdefault(kname, dict(kernel=kname[:96], dispatches=int(a["dispatches"]),
                                                avg_ms=round(a["ns"] / a["dispatches"] * 1e-6, 4), _ns=a["ns"]))
            for typ, peak in MFMA_PEAK_TFLOPS.items():
                mops = a.get(f"SQ_INSTS_VALU_MFMA_MOPS_{typ}", 0.0)
                if mops > 0:
                    tf = 512.0 * mops / (a["ns"] * 1e-9) / 1e12
                    row[f"mfma_{typ.lower()}_tflops"] = round(tf, 2)
                    row[f"mfma_{typ.lower()}_peak_share"] = round(tf / peak, 4)
            for k in PCT_METRICS:
                if k + "_ns" in a:
                    row[{"MfmaUtil": "mfma_util_pct", "LdsUtil": "lds_util_pct",
                         "LDSBankConflict": "lds_bank_conflict_pct"}[k]] = round(a[k + "_ns"] / a["ns"], 2)
            if a.get("SQ_WAVE_CYCLES", 0.0) > 0:
                for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_LDS", "SQ_LDS_DATA_FIFO_FULL"):
                    if k in a:
                        row[k.lower() + "_per_wave_cycle"] = round(a[k] / a["SQ_WAVE_CYCLES"], 4)
    out = sorted(merged.values(), key=lambda r: -r["_ns"])
    for r in out:
        del r["_ns"]
    print(json.dumps({"mfma_counters": directories, "kernels": out[:20]}), flush=True)


def copy_calibration():
    """A plain device copy of known size, the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": a.numel() * 8, "copies": 3}), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bench_yc8_m2048_traffic.md")
TRAFFIC_SOURCES = ["paper_1606_06790_amd/csrc/gemm.hip", "paper_1606_06790_amd/csrc/plan.cpp",
                   "paper_1606_06790_amd/csrc/api.cpp"]


def measured_traffic():
    """{profile class: (kernel, HBM bytes per launch)} from the committed FETCH_SIZE/WRITE_SIZE records, or {} when
    the GEMM sources have changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return {}
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    out = {}
    for m in re.finditer(r"traffic-record: class=(\w+) kernel=(.+?) bytes_per_launch=(\S+) sources_sha256=(\w+)", text):
        if m.group(4) == h.hexdigest():
            out[m.group(1)] = (m.group(2), float(m.group(3)))
    return out


def gemm_roofline(r, traffic_ok=True):
    """Roofline entry for the H_eff GEMM kernel with the largest summed time in run r.  traffic_ok: the run is the
    workload the traffic records were measured on (YC8 kagome, m = 2048)."""
    prof = r["prof"]
    lo = r["prec"] != "f64"
    names = ["heff_gemm1_lo", "heff_gemm2_lo"] if lo else ["heff_gemm1", "heff_gemm2"]
    name = max(names, key=lambda k: prof[k][1])
    n, ms, fl = prof[name]
    achieved = fl / (ms * 1e-3) / 1e12
    stage = "stage 1 (L x psi)" if name.startswith("heff_gemm1") else "stage 2 (T x R^T)"
    out = {"bound": "mfma", "achieved": round(achieved, 3), "peak": round(PEAK[r["prec"]], 1), "unit": "TFLOP/s",
           "frac": round(achieved / PEAK[r["prec"]], 4), "traffic": None,
           "kernel": f"grouped H_eff GEMM {stage}, {r['prec']}", "launches": n,
           "avg_launch_ms": round(ms / max(n, 1), 4)}
    rec = measured_traffic().get(name) if r["prec"] == "bf16x3" and traffic_ok else None
    if rec:
        out["traffic"] = rec[1]
        out["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        out["traffic_kernel"] = rec[0]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prefill", type=int, default=23)
    ap.add_argument("--m", type=int, default=2048)
    ap.add_argument("--mixed", default="bf16x3", choices=["f32", "bf16x3"])
    ap.add_argument("--workload", default="yc8")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-p10", action="store_true", help="skip the Lanczos iterations with / without prediction")
    ap.add_argument("--microbench", action="store_true",
                    help="only run the H_eff matvec microbenchmark (m = 256/512/1024, U(1) and dense, 3 precisions)")
    ap.add_argument("--batching", action="store_true",
                    help="only compare batched (graph / direct) against one call per superblock on --workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy three times (reference for HBM byte counters)")
    ap.add_argument("--launch-gaps", metavar="DIR", default=None,
                    help="only summarise the GPU idle time inside the timed regions of a rocprofv3 kernel + marker "
                         "trace (CSV) found under DIR; runs on the CPU")
    ap.add_argument("--mfma-counters", metavar="DIR", nargs="+", default=None,
                    help="only summarise MFMA and LDS utilisation per kernel from rocprofv3 --pmc runs (CSV), one "
                         "directory per counter pass; runs on the CPU")
    ap.add_argument("--stats-summary", metavar="DIR", default=None,
                    help="only print a markdown table of a rocprofv3 --stats run (CSV) under DIR; runs on the CPU")
    ap.add_argument("--traffic-summary", metavar="DIR", nargs=4, default=None,
                    help="only summarise HBM traffic from four rocprofv3 --pmc runs (CSV): FETCH_SIZE and "
                         "WRITE_SIZE of the benchmark, then of --copy-calibration; runs on the CPU")
    a = ap.parse_args()
    if a.stats_summary:
        stats_summary(a.stats_summary)
        return
    if a.traffic_summary:
        traffic_summary(*a.traffic_summary)
        return
    if a.launch_gaps:
        launch_gaps(a.launch_gaps)
        return
    if a.mfma_counters:
        mfma_counters(a.mfma_counters)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (one process, no collectives); use --gpus 1"}))
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    if a.batching:
        batching(a)
        return
    if a.microbench:
        microbench(a)
        return
    import workloads
    from paper_1606_06790_amd.driver import IDMRG

    cfg = workloads.workload(a.workload, m=a.m)
    d = IDMRG(cfg, prec="f64")
    t_pre = time.perf_counter()
    while d.n < a.prefill:
        d.step()
        note(f"prefill: n={d.n}/{a.prefill} done, {time.perf_counter() - t_pre:.1f} s")
    t_pre = time.perf_counter() - t_pre
    snap = d.snapshot()
    r64 = timed(d, "f64", a.steps, a.warmup)
    d.restore(snap)
    rmx = timed(d, a.mixed, a.steps, a.warmup)
    e64 = {(s["n"], s["i"]): s["e_site"] for s in r64["recs"]}
    de = [s["e_site"] - e64[(s["n"], s["i"])] for s in rmx["recs"]]

    traffic_ok = (a.workload, a.m) == ("yc8", 2048)

    def summary(r):
        return {"matvec_tflops": round(r["matvec_tflops"], 4), "ms_per_step": round(r["ms_per_step"], 2),
                "ms_per_step_events": round(r["ms_per_step_events"], 2), "events_run_identical": r["identical"],
                "lanczos_iters": [s["iters"] for s in r["recs"]],
                "fp64_matvecs": [s["fp64_matvecs"] for s in r["recs"]],
                "reorth_passes": [s["reorth_passes"] for s in r["recs"]],
                "e_site": [round(s["e_site"], 12) for s in r["recs"]],
                "fidelity_error": [s["fidelity"] for s in r["recs"]],
                "unconverged_solves": sum(1 for s in r["recs"] if not s["converged"]),
                "unconverged_svds": sum(1 for s in r["recs"] if not s["svd_converged"]),
                "residual_max": max(s["residual"] for s in r["recs"]),
                "svd_sweeps": max(s["svd_sweeps"] for s in r["recs"]),
                "roofline": gemm_roofline(r, traffic_ok),
                "breakdown_ms_per_step": {k: round(v[1] / a.steps, 2) for k, v in r["prof"].items() if v[0]}}

    out = {
        "metric": f"H_eff matvec TFLOP/s + s per unit-cell step, {LATTICE.get(a.workload, a.workload)} m={a.m}; "
                  "mixed vs FP64",
        "value": round(rmx["matvec_tflops"], 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(rmx["ms_per_step"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{a.mixed}+f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}_heisenberg_m{a.m}_u1", "superblocks": d.half,
                   "iterations_timed": sorted({s["n"] for s in rmx["recs"]}), "prefill": a.prefill,
                   "matvec_prec": a.mixed},
        "roofline": gemm_roofline(rmx, traffic_ok),
        "mixed": summary(rmx),
        "fp64": summary(r64),
        "mixed_vs_fp64": {"speedup_step": round(r64["ms_per_step"] / rmx["ms_per_step"], 4),
                          "speedup_matvec": round(rmx["matvec_tflops"] / r64["matvec_tflops"], 4),
                          "e_site_diff_max": max(abs(x) for x in de)},
        "prefill_s": round(t_pre, 1),
        "tile_tuning": d.ctx.tuning(),
    }
    if not a.no_p10:
        out["prediction_effect"] = prediction_effect(d, snap)
    if not a.no_cpu:
        note("cpu baseline: timing the oracle matvec")
        d.restore(snap)
        out["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
