"""Heisenberg MPOs with an l-site period for the GPU driver (host side).

The Hamiltonian is written as the product of operator-valued matrices of the
paper's Eq. (1)/(7): lower triangular W_i whose last row is the left boundary
and whose first column is the right boundary.  Channel 0 is "complete",
channel D-1 is "identity"; in between, one channel per (pending site, S+ / S- /
S^z) carries an operator of a bond that has opened to the left of the cut and
closes to the right of it.  Charges are 2*S^z with local basis [up, down].
"""
from __future__ import annotations

import numpy as np

from .lib import Mpo

QP = [1, -1]
_OPS = {
    "I": np.eye(2),
    "+": np.array([[0.0, 1.0], [0.0, 0.0]]),
    "-": np.array([[0.0, 0.0], [1.0, 0.0]]),
    "z": np.array([[0.5, 0.0], [0.0, -0.5]]),
}
_DQ = {"+": 2, "-": -2, "z": 0}
_CLOSE = {"+": ("-", 0.5), "-": ("+", 0.5), "z": ("z", 1.0)}


def _translated(cell_bonds, ell, lo, hi):
    """All bonds (j, k, J) of the periodic model with j <= hi and k > lo."""
    span = max((k2 - k for k, k2, _ in cell_bonds), default=0)
    out = {}
    for t in range((lo - span) // ell - 2, hi // ell + 2):
        for k, k2, J in cell_bonds:
            j, kk = k + t * ell, k2 + t * ell
            if j <= hi and kk > lo:
                out[(j, kk)] = out.get((j, kk), 0.0) + J
    return out


def _channels(cell_bonds, ell, cut):
    """Channel labels at the cut after site `cut`: complete, pending ops, identity."""
    bonds = _translated(cell_bonds, ell, cut, cut)
    pend = sorted({j for (j, k) in bonds if j <= cut < k})
    labels = [("done",)] + [("open", j, op) for j in pend for op in ("+", "-", "z")] + [("id",)]
    return labels


def heisenberg_mpo(cell_bonds, ell, dense=False):
    """Return [W_1, ..., W_l] as Mpo objects.  With dense=True every charge is 0
    (no symmetry blocks, the paper's own setting)."""
    Ws = []
    for c in range(1, ell + 1):
        left = _channels(cell_bonds, ell, c - 1 if c > 1 else ell)
        if c == 1:   # the cut before site 1 is the cut after site l of the previous cell
            left = [lab if lab[0] != "open" else ("open", lab[1] - ell, lab[2]) for lab in left]
        right = _channels(cell_bonds, ell, c)
        li = {lab: n for n, lab in enumerate(left)}
        W = np.zeros((len(left), len(right), 2, 2))
        closing = _translated(cell_bonds, ell, c - 1, c)
        for b, lab in enumerate(right):
            if lab == ("done",):
                W[li[("done",)], b] += _OPS["I"]
                for (j, k), J in closing.items():
                    if k == c and J != 0.0:
                        for op in ("+", "-", "z"):
                            cl, f = _CLOSE[op]
                            W[li[("open", j, op)], b] += f * J * _OPS[cl]
            elif lab == ("id",):
                W[li[("id",)], b] += _OPS["I"]
            else:
                _, j, op = lab
                if j == c:
                    W[li[("id",)], b] += _OPS[op]
                else:
                    W[li[lab], b] += _OPS["I"]

        def charges(labels):
            return [0 if (dense or lab[0] != "open") else _DQ[lab[2]] for lab in labels]

        qp = [0, 0] if dense else QP
        Ws.append(Mpo(W, charges(left), charges(right), qp))
    return Ws


def site_leg(qp, sign):
    """Leg of a single site used as a block: sectors (sign*qp) with their states."""
    qs = sorted({sign * q for q in qp})
    states = {q: [s for s in range(len(qp)) if sign * qp[s] == q] for q in qs}
    return [(q, len(states[q])) for q in qs], states


def initial_left(W: Mpo):
    """L^(0) = last row of W (Step 1) in the left-environment layout."""
    leg, st = site_leg(W.qp, +1)
    pos = {}
    for q, lst in st.items():
        for n, s in enumerate(lst):
            pos[s] = (q, n)
    dim = dict(leg)
    out = []
    for qc, dc in leg:
        for w in range(W.dr - 1):
            qr = qc + W.qr[w]
            if qr not in dim:
                continue
            blk = np.zeros((dim[qr], dc))
            for s in st[qr]:
                for t in st[qc]:
                    blk[pos[s][1], pos[t][1]] = W.w[W.dl - 1, w, s, t]
            out.append(blk.reshape(-1))
    return leg, np.concatenate(out)


def initial_right(W: Mpo):
    """R^(0) = first column of W (Step 1) in the right-environment layout."""
    leg, st = site_leg(W.qp, -1)
    pos = {}
    for q, lst in st.items():
        for n, s in enumerate(lst):
            pos[s] = (q, n)
    dim = dict(leg)
    out = []
    for qb, db in leg:
        cols = []
        for w in range(1, W.dl):
            qc = qb - W.ql[w]
            if qc not in dim:
                continue
            blk = np.zeros((db, dim[qc]))
            for s in st[qb]:
                for t in st[qc]:
                    blk[pos[s][1], pos[t][1]] = W.w[w, 0, s, t]
            cols.append(blk)
        if cols:
            out.append(np.concatenate(cols, axis=1).reshape(-1))
    return leg, np.concatenate(out)
