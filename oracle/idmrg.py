"""Parallel infinite-size DMRG driver (oracle).

Test infrastructure only (see ``oracle/__init__``).

Implements Sec. 3 of the paper: Hida's iDMRG (Sec. 2, Steps 1-7) with Steps
2, 3 and 5 replaced by the parallel versions 2', 3', 5'.  Superblock i
(i = 1..l/2) at iteration n covers sites 2i-1 .. 2i+2n:

* left block  L^(n-1)_{2i-1}, centre sites c1 = 2i+n-1, c2 = 2i+n with MPO
  tensors W_{f(c1)}, W_{f(c2)} (f(k) = 1 + mod(k-1, l)), right block
  R^(n-1)_{2(i+1)} produced by superblock i+1 at iteration n-1, with
  R_{l+2} = R_2 (Step 2', Eqs. (8), (9));
* start vector: random for n = 1, 2, else the prediction of Eq. (10)
  (Step 3');
* after all superblocks of iteration n: if mod(n+1, l) = 0, the energy per
  site e_g = (e^(n)_1 - e^(n-l)_1) / (2l) with e^(-1)_1 = 0 (Step 5').
"""
from __future__ import annotations

import time

import numpy as np

import workloads

from . import dense, layout, mpo, u1
from .lanczos import lanczos


class _U1:
    """Per-step operations inside U(1) blocks."""

    def __init__(self, qp):
        self.qp = qp

    def init_left(self, W, dq_out):
        return u1.init_left(W, dq_out, self.qp)

    def init_right(self, W, dq_in):
        return u1.init_right(W, dq_in, self.qp)

    def size(self, A, B):
        return layout.psi_size(A, B, self.qp)

    def from_flat(self, x, A, B):
        return layout.flat_to_psi(x, A, B, self.qp)

    def to_flat(self, psi, A, B):
        return layout.psi_to_flat(psi, A, B, self.qp)

    def heff(self, L, W1, W2, R, psi, A, B, dl, dr):
        return u1.heff_apply(L, W1, W2, R, psi, A, B, self.qp, dl, dr)

    def truncate(self, psi, A, B, m, lam_floor, deg_rel):
        return u1.truncate_twosite(psi, A, B, self.qp, m, lam_floor, deg_rel)

    def update_left(self, L, W1, tr, A, dl, dm):
        return u1.update_env_left(L, W1, tr["U"], A, self.qp, tr["C"], dl, dm)

    def update_right(self, R, W2, tr, B, dm, dr):
        return u1.update_env_right(R, W2, tr["V"], B, self.qp, tr["C"], dm, dr)

    def predict(self, tr_i, lam_prev_ip1, tr_ip1, lam_floor):
        return u1.predict_wavefunction(tr_i["lam"], tr_i["V"], lam_prev_ip1, tr_ip1["U"], tr_ip1["lam"],
                                       tr_i["C"], tr_ip1["C"], self.qp, lam_floor)


class _Dense:
    """Per-step operations on full tensors (all charges ignored)."""

    def init_left(self, W, dq_out):
        L = dense.init_left(W)
        return L, [(0, L.shape[0])]

    def init_right(self, W, dq_in):
        R = dense.init_right(W)
        return R, [(0, R.shape[0])]

    def size(self, A, B):
        return A[0][1] * 4 * B[0][1]

    def from_flat(self, x, A, B):
        return dense.psi_from_flat(x, A[0][1], 2, B[0][1])

    def to_flat(self, psi, A, B):
        return dense.psi_to_flat(psi)

    def heff(self, L, W1, W2, R, psi, A, B, dl, dr):
        return dense.heff_apply(L, W1, W2, R, psi)

    def truncate(self, psi, A, B, m, lam_floor, deg_rel):
        tr = dense.truncate_twosite(psi, m, lam_floor, deg_rel)
        tr["C"] = [(0, tr["m_kept"])]
        return tr

    def update_left(self, L, W1, tr, A, dl, dm):
        return dense.update_env_left(L, W1, tr["U"])

    def update_right(self, R, W2, tr, B, dm, dr):
        return dense.update_env_right(R, W2, tr["V"])

    def predict(self, tr_i, lam_prev_ip1, tr_ip1, lam_floor):
        return dense.predict_wavefunction(tr_i["lam"], tr_i["V"], lam_prev_ip1, tr_ip1["U"], tr_ip1["lam"],
                                          lam_floor)


def superblock_sites(n, i):
    """(first, last, c1, c2) of superblock (n, i)."""
    return 2 * i - 1, 2 * i + 2 * n, 2 * i + n - 1, 2 * i + n


def run(cfg, mode="u1", n_max=None, predict=True, seed=None, keep_states=False, log=None):
    """Run the parallel iDMRG on the workload ``cfg`` (see ``workloads.workload``).

    Returns a dict with ``steps`` (one record per (n, i)), ``e_g`` ({n: value})
    and, if ``keep_states``, the per-iteration environments and decompositions.
    The random start vectors of iterations 1 and 2 are drawn with ``seed``, else
    the configuration's own ``seed``, else ``workloads.SEED``.
    """
    if seed is None:
        seed = cfg.get("seed", workloads.SEED)
    ell = cfg["ell"]
    half = ell // 2
    n_max = cfg["n_max"] if n_max is None else n_max
    Ws, dq = mpo.build_mpo(ell, cfg["bonds"])
    ops = _U1(mpo.QP) if mode == "u1" else _Dense()
    m, tol_E, tol_res, k_max = cfg["m"], cfg["tol_E"], cfg["tol_res"], cfg["k_max"]
    lam_floor, deg_rel = cfg["lam_floor"], cfg["deg_rel"]

    def W(k):
        return Ws[mpo.f_index(k, ell) - 1]

    def cut(k):  # channel charges at the cut after absolute site k
        return dq[mpo.f_index(k, ell)]

    # Step 1: L^(0)_{2i-1} = last row of W_{2i-1}, R^(0)_{2i} = first column of W_{2i}
    Lenv, Renv = {}, {}
    for i in range(1, half + 1):
        Lenv[i] = ops.init_left(W(2 * i - 1), cut(2 * i - 1))
        Renv[i] = ops.init_right(W(2 * i), cut(2 * i - 1))

    prev, lam_prev2 = {}, {}
    energies = {}
    steps, e_g, states = [], {}, []
    for n in range(1, n_max + 1):
        newL, newR, cur = {}, {}, {}
        for i in range(1, half + 1):
            t0 = time.perf_counter()
            ip1 = i % half + 1
            (L, A), (R, B) = Lenv[i], Renv[ip1]
            first, last, c1, c2 = superblock_sites(n, i)
            W1, W2 = W(c1), W(c2)
            dl, dm, dr = cut(c1 - 1), cut(c1), cut(c2)
            N = ops.size(A, B)
            if n <= 2 or not predict:
                v0 = workloads.start_vector(N, n, i, seed)
            else:
                guess = ops.predict(prev[i], lam_prev2[ip1], prev[ip1], lam_floor)
                v0 = ops.to_flat(guess, A, B)
                if not np.any(v0):
                    v0 = workloads.start_vector(N, n, i, seed)

            def mv(x, L=L, R=R, W1=W1, W2=W2, A=A, B=B, dl=dl, dr=dr):
                return ops.to_flat(ops.heff(L, W1, W2, R, ops.from_flat(x, A, B), A, B, dl, dr), A, B)

            sol = lanczos(mv, v0, tol_E, tol_res, k_max)
            psi_flat = sol["psi"]
            fid = 1.0 - abs(float(v0 @ psi_flat)) / float(np.linalg.norm(v0))       # Eq. (12)
            psi = ops.from_flat(psi_flat, A, B)
            tr = ops.truncate(psi, A, B, m, lam_floor, deg_rel)
            newL[i] = (ops.update_left(L, W1, tr, A, dl, dm), tr["C"])
            newR[i] = (ops.update_right(R, W2, tr, B, dm, dr), tr["C"])
            cur[i] = tr
            energies[(n, i)] = sol["energy"]
            rec = dict(n=n, i=i, energy=sol["energy"], e_site=sol["energy"] / (2 * n + 2),
                       iters=sol["iters"], residual=sol["residual"], fidelity=fid,
                       eps=tr["eps"], eps_prime=tr["eps_prime"], m_kept=tr["m_kept"],
                       cut_gap=tr["cut_gap"], sites=(first, last), N=N,
                       seconds=time.perf_counter() - t0)
            steps.append(rec)
            if log:
                log(rec)
            if keep_states:
                states.append(dict(n=n, i=i, L=L, R=R, A=A, B=B, W1=W1, W2=W2, dl=dl, dm=dm, dr=dr,
                                   v0=v0, psi=psi_flat, tr=tr))
        lam_prev2 = {i: prev[i]["lam"] for i in prev}
        prev = cur
        Lenv, Renv = newL, newR
        if (n + 1) % ell == 0:                                                  # Step 5'
            e_old = energies[(n - ell, 1)] if n - ell >= 1 else 0.0
            e_g[n] = (energies[(n, 1)] - e_old) / (2 * ell)
    out = dict(steps=steps, e_g=e_g, mode=mode, cfg=cfg)
    if keep_states:
        out["states"] = states
    return out
