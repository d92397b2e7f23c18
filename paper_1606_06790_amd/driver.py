"""Parallel infinite-size DMRG on one GPU (host control flow).

Follows Sec. 3 of the paper: Hida's iDMRG with Steps 2, 3 and 5 replaced by
their parallel versions.  At iteration n the l/2 superblocks i = 1..l/2 each
consist of L^(n-1)_{2i-1}, the centre sites 2i+n-1 and 2i+n with W_{f(.)},
and R^(n-1)_{2(i+1)} from the neighbour (R_{l+2} = R_2) (Step 2', Eqs. (8),
(9)).  All of them go through the library together: one batched prediction
(Eq. (10), Step 3'), one batched Lanczos solve (Step 3), one batched
truncation (Step 4), two batched environment updates (Step 6, Eqs. (4),
(5)).  The neighbour hand-off is a swap of device tensors.  Step 5' forms
e_g = (e^(n)_1 - e^(n-l)_1) / (2l) whenever mod(n+1, l) = 0.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

import workloads

from . import lib, models


CHECKPOINT_VERSION = 1


class IDMRG:
    def __init__(self, cfg, device=0, prec=None, dense=False, predict=True, chunk=8, log=None, graph=False,
                 batched=True):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.ell = cfg["ell"]
        self.half = self.ell // 2
        self.dev = torch.device("cuda", device)
        self.prec = prec or cfg.get("prec", "f64")
        self.seed = cfg.get("seed", workloads.SEED)   # random start vectors of iterations 1 and 2
        self.predict = predict
        self.dense = dense
        self.chunk = chunk
        self.graph = graph
        self.fp32_basis = True   # mixed precision: the first pass's Krylov vectors stored in FP32
        self.batched = batched   # False: one library call per superblock (for comparison only)
        self.log = log
        self.W = models.heisenberg_mpo(cfg["bonds"], self.ell, dense=dense)
        self.qp = self.W[0].qp
        self.ctx = lib.Context(device)
        self.n = 0
        self.energies = {}
        self.steps = []
        self.e_g = {}
        # Step 1: L^(0)_{2i-1} = last row of W_{2i-1}, R^(0)_{2i} = first column of W_{2i}
        self.L, self.R = {}, {}
        for i in range(1, self.half + 1):
            leg, x = models.initial_left(self.Wsite(2 * i - 1))
            self.L[i] = (leg, self._dev(x))
            leg, x = models.initial_right(self.Wsite(2 * i))
            self.R[i] = (leg, self._dev(x))
        self.prev, self.lam2 = {}, {}

    def _dev(self, x):
        return self.torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(self.dev)

    def Wsite(self, k):
        return self.W[(k - 1) % self.ell]

    def problems(self, n):
        """Superblock Hamiltonians of iteration n (Step 2'): pointers only."""
        out = []
        for i in range(1, self.half + 1):
            ip1 = i % self.half + 1
            (A, Lt), (B, Rt) = self.L[i], self.R[ip1]
            out.append(dict(left=A, right=B, w1=self.Wsite(2 * i + n - 1), w2=self.Wsite(2 * i + n), L=Lt, R=Rt,
                            i=i, ip1=ip1))
        return out

    def start_vectors(self, n, H):
        """Step 3': random for n <= 2 (seeded, drawn on the host), Eq. (10) otherwise."""
        if n <= 2 or not self.predict:
            return [self._dev(workloads.start_vector(lib.psi_size(h["left"], h["right"], self.qp), n, h["i"],
                                                     self.seed)) for h in H]
        items = []
        for h in H:
            i, ip1 = h["i"], h["ip1"]
            pi, pn = self.prev[i], self.prev[ip1]
            items.append(dict(leg_a=pi["C"], leg_beta=self.lam2[ip1][0], leg_b=pn["C"], lam_i=pi["lam"],
                              V_i=pi["V"], lam_prev=self.lam2[ip1][1], U_ip1=pn["U"], lam_ip1=pn["lam"]))
        return self._calls(lib.predict_wavefunction, items, self.qp, self.cfg["lam_floor"])

    def _calls(self, fn, items, *args):
        """fn over the superblocks: one batched call, or one call per superblock."""
        if self.batched:
            return fn(self.ctx, items, *args)
        return [r for it in items for r in fn(self.ctx, [it], *args)]

    def step(self):
        """One unit-cell step: iteration n for all l/2 superblocks."""
        torch = self.torch
        n = self.n + 1
        cfg = self.cfg
        t0 = time.perf_counter()
        H = self.problems(n)
        psis = self.start_vectors(n, H)
        if n > 2 and self.predict:
            # a start vector that is exactly zero cannot seed Lanczos; fall back to the random rule
            norms = [float(torch.linalg.vector_norm(p)) for p in psis]
            for j, nr in enumerate(norms):
                if nr == 0.0:
                    psis[j] = self._dev(workloads.start_vector(psis[j].numel(), n, H[j]["i"], self.seed))
        t1 = time.perf_counter()
        if self.batched:
            es, infos = lib.lanczos_solve_batch(self.ctx, H, psis, cfg["tol_E"], cfg["tol_res"], cfg["k_max"],
                                                self.prec, self.chunk, graph=self.graph,
                                                fp32_basis=self.fp32_basis)
        else:
            es, infos = [], []
            for h, p in zip(H, psis):
                e1, i1 = lib.lanczos_solve_batch(self.ctx, [h], [p], cfg["tol_E"], cfg["tol_res"], cfg["k_max"],
                                                 self.prec, self.chunk, graph=self.graph,
                                                 fp32_basis=self.fp32_basis)
                es += e1
                infos += i1
        t2 = time.perf_counter()
        trs = self._calls(lib.truncate_twosite, [dict(left=h["left"], right=h["right"], psi=p) for h, p in zip(H, psis)],
                          self.qp, cfg["m"], cfg["lam_floor"], cfg["deg_rel"])
        t3 = time.perf_counter()
        newL = self._calls(lambda c, it: lib.update_env(c, lib.LEFT, it),
                           [dict(old_leg=h["left"], new_leg=tr["C"], w=h["w1"], env_old=h["L"], iso=tr["U"])
                            for h, tr in zip(H, trs)])
        newR = self._calls(lambda c, it: lib.update_env(c, lib.RIGHT, it),
                           [dict(old_leg=h["right"], new_leg=tr["C"], w=h["w2"], env_old=h["R"], iso=tr["V"])
                            for h, tr in zip(H, trs)])
        torch.cuda.synchronize(self.dev)
        t4 = time.perf_counter()
        for h, e in zip(H, es):
            self.energies[(n, h["i"])] = e
        if (n + 1) % self.ell == 0:       # Step 5'
            e_old = self.energies[(n - self.ell, 1)] if n - self.ell >= 1 else 0.0
            self.e_g[n] = (self.energies[(n, 1)] - e_old) / (2 * self.ell)
        # seconds of the whole batched step (all superblocks together) by stage
        secs = dict(predict=t1 - t0, lanczos=t2 - t1, truncate=t3 - t2, env=t4 - t3)
        for h, e, inf, tr, Ln, Rn in zip(H, es, infos, trs, newL, newR):
            i = h["i"]
            rec = dict(n=n, i=i, energy=e, e_site=e / (2 * n + 2), iters=inf["iters"], residual=inf["residual"],
                       fidelity=1.0 - inf["overlap0"], eps=tr["eps"], eps_prime=tr["eps_prime"],
                       m_kept=tr["m_kept"], cut_gap=tr["cut_gap"], svd_sweeps=tr["svd_sweeps"],
                       fp64_matvecs=inf["fp64_matvecs"], reorth_passes=inf["reorth_passes"],
                       converged=bool(inf["converged"]), svd_converged=bool(tr["svd_converged"]),
                       N=int(psis[h["i"] - 1].numel()), step_seconds=secs)
            if i == 1 and n in self.e_g:
                rec["e_g"] = self.e_g[n]
            self.steps.append(rec)
            if self.log:
                self.log(rec)
        # hand-off: new environments and decompositions replace the old ones (pointer swap)
        self.lam2 = {i: (self.prev[i]["C"], self.prev[i]["lam"]) for i in self.prev}
        self.prev = {h["i"]: tr for h, tr in zip(H, trs)}
        self.L = {h["i"]: (tr["C"], Ln) for h, tr, Ln in zip(H, trs, newL)}
        self.R = {h["i"]: (tr["C"], Rn) for h, tr, Rn in zip(H, trs, newR)}
        self.n = n
        return dict(n=n, seconds=t4 - t0, t_predict=t1 - t0, t_lanczos=t2 - t1, t_truncate=t3 - t2,
                    t_env=t4 - t3, iters=[inf["iters"] for inf in infos])

    def snapshot(self):
        """State after the last iteration (device tensors are never modified in place, so references suffice)."""
        return dict(n=self.n, L=dict(self.L), R=dict(self.R), prev=dict(self.prev), lam2=dict(self.lam2),
                    energies=dict(self.energies), e_g=dict(self.e_g), steps=list(self.steps))

    def restore(self, snap):
        self.n = snap["n"]
        self.L, self.R = dict(snap["L"]), dict(snap["R"])
        self.prev, self.lam2 = dict(snap["prev"]), dict(snap["lam2"])
        self.energies, self.e_g, self.steps = dict(snap["energies"]), dict(snap["e_g"]), list(snap["steps"])

    def save(self, path):
        """Write the state after the last iteration to `path` (an uncompressed .npz; the file is replaced only
        once it is complete).  It holds what the next iteration reads: L^(n)_{2i-1} and R^(n)_{2i} of every
        superblock, the decomposition U, Lambda, V of iteration n and Lambda^(n-1) (both enter Eq. (10)),
        each with its quantum-number leg, and the energy history for Step 5'.  Arrays are float64; the rest
        (configuration, legs, records) is one JSON string, so reading it back unpickles nothing."""
        arrays, legs = {}, {}

        def put(key, leg, t):
            legs[key] = [[int(q), int(x)] for q, x in leg]
            arrays[key] = t.detach().to("cpu").numpy()

        for i, (leg, t) in self.L.items():
            put(f"L{i}", leg, t)
        for i, (leg, t) in self.R.items():
            put(f"R{i}", leg, t)
        prev = {}
        for i, tr in self.prev.items():
            put(f"U{i}", tr["C"], tr["U"])
            put(f"V{i}", tr["C"], tr["V"])
            put(f"lam{i}", tr["C"], tr["lam"])
            prev[str(i)] = {k: v for k, v in tr.items() if k not in ("C", "U", "V", "lam")}
        for i, (leg, lam) in self.lam2.items():
            put(f"lam2_{i}", leg, lam)
        header = dict(version=CHECKPOINT_VERSION, cfg=self.cfg, prec=self.prec, dense=self.dense,
                      predict=self.predict, chunk=self.chunk, fp32_basis=self.fp32_basis, batched=self.batched,
                      n=self.n, superblocks=sorted(self.L), prev=prev, lam2=sorted(self.lam2), legs=legs,
                      energies=[[n, i, e] for (n, i), e in sorted(self.energies.items())],
                      e_g=[[n, e] for n, e in sorted(self.e_g.items())], steps=self.steps)
        tmp = path + ".partial"
        with open(tmp, "wb") as f:
            np.savez(f, header=np.array(json.dumps(header)), **arrays)
        os.replace(tmp, path)

    @classmethod
    def resume(cls, path, device=0, log=None, graph=False):
        """A driver in the state `save` wrote, on `device`, ready to continue with iteration n + 1.  The run
        then continues bitwise as it would have without the interruption: every step is deterministic given
        this state (the GEMM tile variants a fresh tuner may choose give identical results)."""
        import torch
        with np.load(path, allow_pickle=False) as z:
            h = json.loads(str(z["header"]))
            arrays = {k: z[k] for k in z.files if k != "header"}
        if h.get("version") != CHECKPOINT_VERSION:
            raise ValueError(f"{path}: checkpoint version {h.get('version')}, expected {CHECKPOINT_VERSION}")
        cfg = dict(h["cfg"], bonds=[tuple(b) for b in h["cfg"]["bonds"]])
        d = cls(cfg, device=device, prec=h["prec"], dense=h["dense"], predict=h["predict"], chunk=h["chunk"],
                log=log, graph=graph, batched=h["batched"])
        d.fp32_basis = h["fp32_basis"]

        def leg(key):
            return [(int(q), int(x)) for q, x in h["legs"][key]]

        def dev(key):
            return torch.from_numpy(arrays[key]).to(d.dev)

        d.n = int(h["n"])
        d.L = {i: (leg(f"L{i}"), dev(f"L{i}")) for i in h["superblocks"]}
        d.R = {i: (leg(f"R{i}"), dev(f"R{i}")) for i in h["superblocks"]}
        d.prev = {int(i): dict(meta, C=leg(f"U{i}"), U=dev(f"U{i}"), V=dev(f"V{i}"), lam=dev(f"lam{i}"))
                  for i, meta in h["prev"].items()}
        d.lam2 = {i: (leg(f"lam2_{i}"), dev(f"lam2_{i}")) for i in h["lam2"]}
        d.energies = {(int(n), int(i)): e for n, i, e in h["energies"]}
        d.e_g = {int(n): e for n, e in h["e_g"]}
        d.steps = list(h["steps"])
        return d

    def run(self, n_max):
        out = []
        while self.n < n_max:
            out.append(self.step())
        return out


def prediction_probe(d):
    """FP64 Lanczos iterations of iteration d.n + 1 from the current state with the prediction of Eq. (10)
    and with a random start, each under the full stop rule and under the |dtheta| rule alone (plain Lanczos
    counts, as the paper's comparison); the state and the precision are restored afterwards.  Returns
    {label: [iterations per superblock]}."""
    snap = d.snapshot()
    keep = (d.predict, dict(d.cfg), d.prec)
    out = {}
    d.prec = "f64"
    for label, predict, dtheta_only in (("with_prediction", True, False), ("with_prediction_dtheta_rule", True, True),
                                        ("random_start", False, False), ("random_start_dtheta_rule", False, True)):
        d.restore(snap)
        d.predict = predict
        d.cfg = dict(keep[1], tol_res=1e300 if dtheta_only else keep[1]["tol_res"])
        d.step()
        out[label] = [s["iters"] for s in d.steps if s["n"] == d.n]
    d.predict, d.cfg, d.prec = keep
    d.restore(snap)
    return out


def long_run(d, n_max, out, probe_at=(), checkpoint=None):
    """Run to n_max, writing one JSON record per unit-cell period (l iterations) to `out`: the Step 5'
    energy e_g, e^(n)_1 / (2n + 2), Lanczos iterations, fidelity errors (Eq. (12)), the truncation error
    eps = max over the period of eps^(n)_1 (Eq. (14)), kept states and seconds per iteration.  With
    `checkpoint`, the state is saved there after each period's record."""
    import sys
    period = []
    t_start = time.perf_counter()
    while d.n < n_max:
        if d.n + 1 in probe_at:
            rec = dict(kind="prediction_probe", iteration=d.n + 1, **prediction_probe(d))
            out.write(json.dumps(rec) + "\n")
            out.flush()
        r = d.step()
        period.append(r)
        if (d.n + 1) % d.ell == 0:
            recs = [s for s in d.steps if s["n"] > d.n - d.ell]
            first = [s for s in recs if s["i"] == 1]
            its = [s["iters"] for s in recs]
            fid = sorted(s["fidelity"] for s in recs)
            rec = dict(kind="period", n=d.n, e_g=d.e_g[d.n], e_site_1=first[-1]["e_site"],
                       eps=max(s["eps"] for s in first), m_kept=min(s["m_kept"] for s in recs),
                       iters_mean=sum(its) / len(its), iters_min=min(its), iters_max=max(its),
                       fidelity_median=fid[len(fid) // 2], fidelity_max=fid[-1],
                       unconverged=sum(1 for s in recs if not s["converged"]),
                       s_per_iteration=sum(p["seconds"] for p in period) / len(period),
                       elapsed_s=time.perf_counter() - t_start)
            out.write(json.dumps(rec) + "\n")
            out.flush()
            if checkpoint:
                d.save(checkpoint)
            print(f"n={d.n} e_g={rec['e_g']:.10f} iters={rec['iters_mean']:.1f} "
                  f"fid_med={rec['fidelity_median']:.1e} eps={rec['eps']:.2e} "
                  f"{rec['s_per_iteration']:.3f} s/it", file=sys.stderr, flush=True)
            period = []


def main():
    import argparse
    ap = argparse.ArgumentParser(description="parallel iDMRG on one GPU")
    ap.add_argument("--workload", default="chain")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--prec", default=None)
    ap.add_argument("--dense", action="store_true")
    ap.add_argument("--periods", default=None,
                    help="write one record per unit-cell period to this file instead of one per superblock")
    ap.add_argument("--tol-res", type=float, default=None, help="Lanczos residual tolerance (default: the workload's)")
    ap.add_argument("--probe-at", type=int, nargs="*", default=[],
                    help="iterations at which Lanczos counts with and without prediction are compared")
    ap.add_argument("--config", default=None,
                    help="run configuration as a JSON file (the format of --dump-config); replaces --workload")
    ap.add_argument("--dump-config", action="store_true",
                    help="print the run configuration (workload or --config, with --m / --tol-res applied) as JSON "
                         "and exit")
    ap.add_argument("--checkpoint", default=None,
                    help="save the state to this .npz after every unit-cell period (with --periods), else at the end")
    ap.add_argument("--resume", default=None,
                    help="continue from a state saved with --checkpoint (its workload, m and precision apply; "
                         "with --periods the records are appended)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of GEMM tile choices: read at start (if it matches this device and build), "
                         "written at the end")
    a = ap.parse_args()
    over = {}
    if a.m:
        over["m"] = a.m
    if a.tol_res:
        over["tol_res"] = a.tol_res
    cfg = None
    if not a.resume:
        cfg = workloads.load_config(a.config) if a.config else workloads.workload(a.workload)
        cfg = workloads.check_config(dict(cfg, **over))
    if a.dump_config:
        if cfg is None:
            ap.error("--dump-config needs a workload or --config, not --resume")
        print(json.dumps(dict(cfg, bonds=[list(b) for b in cfg["bonds"]]), indent=1))
        return

    def make(log=None):
        if a.resume:
            return IDMRG.resume(a.resume, log=log)
        return IDMRG(cfg, prec=a.prec, dense=a.dense, log=log)

    if a.periods:
        d = make()
        n_max = a.n or d.cfg["n_max"]
        if a.tune_cache:
            d.ctx.load_tuning(a.tune_cache)
        with open(a.periods, "a" if a.resume else "w") as f:
            head = dict(kind="resume" if a.resume else "config", workload=d.cfg["name"])
            f.write(json.dumps(dict(head, m=d.cfg["m"], prec=d.prec, tol_res=d.cfg["tol_res"], n_max=n_max,
                                    n=d.n)) + "\n")
            long_run(d, n_max, f, set(a.probe_at), a.checkpoint)
    else:
        d = make(log=lambda r: print(json.dumps(r), flush=True))
        if a.tune_cache:
            d.ctx.load_tuning(a.tune_cache)
        d.run(a.n or d.cfg["n_max"])
        if a.checkpoint:
            d.save(a.checkpoint)
        print(json.dumps(dict(e_g=d.e_g)))
    if a.tune_cache:
        d.ctx.save_tuning(a.tune_cache)


if __name__ == "__main__":
    main()
