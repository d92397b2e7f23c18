"""Extrapolation of the Step 5' energy in the truncation error (Sec. 4, truncation-error subsection).

For each kept-state count m, a converged run of the parallel iDMRG gives the
subtracted energy per site e_g and the truncation error of Eq. (14) taken as
eps = max over one unit-cell period of eps^(n)_1 (the paper's definition of
the truncation error of the parallel method).  The energy in the limit
eps -> 0 follows from a least-squares polynomial fit e_g = e0 + a eps + b eps^2
(quadratic, as in the paper).  Host arithmetic on a handful of scalars.

    python -m paper_1606_06790_amd.extrapolate [--m-min M] [--eps-max E] runs/*.jsonl
    python -m paper_1606_06790_amd.extrapolate --observables [--eps-max E] obs/*.json
"""
from __future__ import annotations

import json

import numpy as np


def converged_point(records, periods=3):
    """(m, e_g, eps, spread) from the period records of one long run: the last period's e_g and eps, and the
    spread of e_g over the last `periods` periods (a convergence check in n)."""
    cfg = next(r for r in records if r.get("kind") == "config")
    per = [r for r in records if r.get("kind") == "period"]
    if not per:
        raise ValueError("no period records")
    tail = [r["e_g"] for r in per[-periods:]]
    return cfg["m"], per[-1]["e_g"], per[-1]["eps"], max(tail) - min(tail)


def fit(eps, e, degree=2):
    """Least-squares fit e = sum_k c_k eps^k (k = 0..degree).  Returns (c, stderr of c_0, rms residual)."""
    eps = np.asarray(eps, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    X = np.vander(eps, degree + 1, increasing=True)
    c, res, rank, _ = np.linalg.lstsq(X, e, rcond=None)
    r = e - X @ c
    dof = len(e) - (degree + 1)
    rms = float(np.sqrt(np.mean(r ** 2)))
    if dof > 0 and rank == degree + 1:
        s2 = float(r @ r) / dof
        cov = s2 * np.linalg.inv(X.T @ X)
        err0 = float(np.sqrt(cov[0, 0]))
    else:
        err0 = float("nan")
    return c, err0, rms


def main(paths, m_min=0, eps_max=None):
    """Fit the converged points of the runs in `paths` (kept-state counts >= m_min, eps below eps_max if given)."""
    pts = []
    for p in paths:
        with open(p) as f:
            pts.append(converged_point([json.loads(line) for line in f if line.strip()]))
    pts.sort()
    skipped = [q for q in pts if q[0] < m_min or (eps_max is not None and q[2] >= eps_max)]
    pts = [q for q in pts if q not in skipped]
    for m, e, eps, _ in skipped:
        print(f"m={m:5d}  e_g={e:.10f}  eps={eps:.4e}  (left out of the fit)")
    for m, e, eps, spread in pts:
        print(f"m={m:5d}  e_g={e:.10f}  eps={eps:.4e}  spread over the last periods {spread:.1e}")
    eps = [p[2] for p in pts]
    e = [p[1] for p in pts]
    out = {}
    for deg in (1, 2):
        if len(pts) > deg:
            c, err0, rms = fit(eps, e, deg)
            out[deg] = dict(e0=float(c[0]), e0_stderr=err0, coef=[float(x) for x in c], rms=rms)
            print(f"degree {deg}: e(eps -> 0) = {c[0]:.7f} +- {err0:.1e}  (rms residual {rms:.1e})")
    print(json.dumps(dict(points=[dict(m=m, e_g=e_, eps=x, spread=s) for m, e_, x, s in pts], fits=out)))
    return out


def observables(paths, eps_max=None, degree=2, r0=2, d_min=5.0):
    """Extrapolate the observables of the uniform MPS (Sec. 4: bond strengths, Eqs. (15), (16); the correlation
    function along the cylinder) in eps, from the JSON lines of `python -m paper_1606_06790_amd.observables`
    (one run per line, any number of files).  Each bond class's average and its Delta+- and each point of the
    correlation function are fitted separately (degree `degree`, runs with eps below eps_max); the correlation
    length in unit cells is then fitted to the extrapolated correlation function over r >= r0.  Where the runs
    hold the correlation along the cylinder's axis (YC8), its points are extrapolated the same way and its decay
    length fitted over distances above d_min, with the standard error of the fit."""
    runs = []
    for p in paths:
        with open(p) as f:
            runs.extend(json.loads(line) for line in f if line.strip().startswith("{"))
    runs.sort(key=lambda r: r["eps"], reverse=True)
    use = [r for r in runs if eps_max is None or r["eps"] < eps_max]
    for r in runs:
        tag = "" if r in use else "  (left out of the fits)"
        print(f"m={r['m']:5d}  n={r['n']}  eps={r['eps']:.4e}  xi={r['correlation']['xi_cells']:.4f} cells{tag}")
    eps = [r["eps"] for r in use]
    out = dict(points=[dict(m=r["m"], eps=r["eps"]) for r in use], classes={}, correlation={})
    for name in use[0]["classes"]:
        row = {}
        for key in ("average", "delta_plus", "delta_minus"):
            c, err0, rms = fit(eps, [r["classes"][name][key] for r in use], degree)
            row[key] = dict(value=float(c[0]), stderr=err0, rms=rms)
        out["classes"][name] = row
        print(f"bond {name:>6}: average -> {row['average']['value']:.5f} +- {row['average']['stderr']:.1e}, "
              f"Delta+ -> {row['delta_plus']['value']:.2e}, Delta- -> {row['delta_minus']['value']:.2e}")
    nr = min(len(r["correlation"]["values"]) for r in use)
    corr = []
    for k in range(nr):
        c, err0, _ = fit(eps, [r["correlation"]["values"][k] for r in use], degree)
        corr.append((float(c[0]), err0))
    rr = np.arange(1, nr + 1, dtype=np.float64)
    keep = rr >= r0
    slope = np.polyfit(rr[keep], np.log(np.abs([c for c, _ in corr]))[keep], 1)[0]
    out["correlation"] = dict(label=use[0]["correlation"]["label"], values=[c for c, _ in corr],
                              stderr=[e for _, e in corr], xi_cells=float(-1.0 / slope), fit_from=r0)
    print("correlation function (extrapolated): " + ", ".join(f"{c:.3e}" for c, _ in corr))
    print(f"correlation length (r >= {r0}): {out['correlation']['xi_cells']:.4f} unit cells")
    if all(r.get("axis") for r in use):
        ax = use[0]["axis"]
        na = min(len(r["axis"]["values"]) for r in use)
        vals = []
        for k in range(na):
            c, err0, _ = fit(eps, [r["axis"]["values"][k] for r in use], degree)
            vals.append((float(c[0]), err0))
        d = np.asarray(ax["distance"][:na])
        keep = d > d_min
        X = np.vander(d[keep], 2, increasing=True)
        y = np.log(np.abs([v for v, _ in vals]))[keep]
        c, _, _, _ = np.linalg.lstsq(X, y, rcond=None)
        res = y - X @ c
        dof = int(keep.sum()) - 2
        slope_err = float(np.sqrt(res @ res / dof * np.linalg.inv(X.T @ X)[1, 1])) if dof > 0 else float("nan")
        xi = float(-1.0 / c[1])
        out["axis"] = dict(sites=ax["sites"][:na], distance=[float(x) for x in d], values=[v for v, _ in vals],
                           stderr=[e for _, e in vals], xi=xi, xi_stderr=xi * xi * slope_err, fit_above=d_min)
        print("along the axis (extrapolated): " + ", ".join(f"{s_}@{x:.2f}: {v:.3e}" for s_, x, (v, _) in
                                                          zip(ax["sites"], d, vals)))
        print(f"decay length (distance > {d_min}): {xi:.3f} +- {xi * xi * slope_err:.3f}")
    print(json.dumps(out))
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="fit e_g against the truncation error eps of converged runs")
    ap.add_argument("paths", nargs="+", help="period-record files of driver --periods runs")
    ap.add_argument("--m-min", type=int, default=0, help="leave out runs with fewer kept states")
    ap.add_argument("--eps-max", type=float, default=None, help="leave out runs with eps at or above this")
    ap.add_argument("--observables", action="store_true",
                    help="the paths hold observables runs (bond classes, correlation function): fit those")
    ap.add_argument("--fit-from", type=int, default=2, help="observables: first unit cell of the correlation fit")
    a = ap.parse_args()
    if a.observables:
        observables(a.paths, a.eps_max, r0=a.fit_from)
    else:
        main(a.paths, a.m_min, a.eps_max)
