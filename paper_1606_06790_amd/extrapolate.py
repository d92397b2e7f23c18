"""Extrapolation of the Step 5' energy in the truncation error (Sec. 4, truncation-error subsection).

For each kept-state count m, a converged run of the parallel iDMRG gives the
subtracted energy per site e_g and the truncation error of Eq. (14) taken as
eps = max over one unit-cell period of eps^(n)_1 (the paper's definition of
the truncation error of the parallel method).  The energy in the limit
eps -> 0 follows from a least-squares polynomial fit e_g = e0 + a eps + b eps^2
(quadratic, as in the paper).  Host arithmetic on a handful of scalars.

    python -m paper_1606_06790_amd.extrapolate [--m-min M] [--eps-max E] runs/*.jsonl
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


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="fit e_g against the truncation error eps of converged runs")
    ap.add_argument("paths", nargs="+", help="period-record files of driver --periods runs")
    ap.add_argument("--m-min", type=int, default=0, help="leave out runs with fewer kept states")
    ap.add_argument("--eps-max", type=float, default=None, help="leave out runs with eps at or above this")
    a = ap.parse_args()
    main(a.paths, a.m_min, a.eps_max)
