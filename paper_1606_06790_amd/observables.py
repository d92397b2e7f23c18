"""Observables of the uniform MPS of Eq. (11), computed by the library (Sec. 4).

After iteration n the wavefunction repeats a unit cell of the l/2 two-site
pieces B_i = V^(n)dagger_i U~^(n)_{i+1} (i + 1 cyclic), which are the Eq. (10)
states of predict_wavefunction with lambda_i = 1; piece i holds the sites
n + 2i and n + 2i + 1.  Everything tensor-valued runs on the GPU:

* the pieces: one predict_wavefunction call;
* the left transfer matrix of a piece: update_env(LEFT) with the piece as the
  left isometry of its fused site (the two-site layout is that isometry) and a
  three-channel MPO of the fused site: channel 0 carries the plain transfer,
  channel 1 the operator string, channel 2 the (unstored) identity;
* the right transfer matrix: update_env(RIGHT) with the piece rewritten by
  twosite_to_right_iso; channels 1 and 2 carry the transfer, channel 0 is the
  (unstored) identity;
* expectation values: env_overlap of the left environment after the operators
  with the right fixed point, divided by the same overlap of the plain channel.

The host builds the tiny fused-site MPOs (model data), the starting
environments (Lambda^2 on the left, the identity on the right) and divides the
scalars the library returns.  The fixed points are reached by applying the cell
transfer matrix until the dominant eigenvalue estimate settles.
"""
from __future__ import annotations

import numpy as np

from . import lib

SZ = np.diag([0.5, -0.5])
SP = np.array([[0.0, 1.0], [0.0, 0.0]])     # <up| S+ |down> = 1 (local state 0 is up, charge +1)
SM = SP.T.copy()
ID2 = np.eye(2)
DQ = {"z": 0, "+": 2, "-": -2, "1": 0}
OPS = {"z": SZ, "+": SP, "-": SM, "1": ID2}
TERMS = (("z", "z", 1.0), ("+", "-", 0.5), ("-", "+", 0.5))   # s_a . s_b


def fused_mpo(op1, op2, q_in, side, qp):
    """Three-channel MPO of a fused two-site piece whose operator channel applies op1 (x) op2.

    side LEFT: channels (plain transfer, operator string, identity), the string entering with charge q_in;
    side RIGHT: channels (identity, operator string, plain transfer)."""
    O = np.kron(OPS[op1], OPS[op2])
    dq = DQ[op1] + DQ[op2]
    W = np.zeros((3, 3, 4, 4))
    W[0, 0] = np.eye(4)
    W[2, 2] = np.eye(4)
    W[1, 1] = O
    if side == lib.LEFT:
        ql, qr = [0, q_in, 0], [0, q_in + dq, 0]
    else:
        qr, ql = [0, q_in, 0], [0, q_in - dq, 0]
    return lib.Mpo(W, ql, qr, lib.fused_qp(qp))


class UniformMPS:
    """The Eq. (11) unit cell of a driver state after its last iteration (driver.IDMRG after run/step)."""

    def __init__(self, d, tol=1e-13, max_cells=400):
        self.d = d
        self.ctx = d.ctx
        self.torch = d.torch
        self.half = d.half
        self.ell = d.ell
        self.n = d.n
        self.qp = list(d.qp)
        self.tol = tol
        self.max_cells = max_cells
        items, self.legs = [], []
        for i in range(1, self.half + 1):
            ip1 = i % self.half + 1
            pi, pn = d.prev[i], d.prev[ip1]
            items.append(dict(leg_a=pi["C"], leg_beta=d.lam2[ip1][0], leg_b=pn["C"],
                              lam_i=self.torch.ones_like(pi["lam"]), V_i=pi["V"], lam_prev=d.lam2[ip1][1],
                              U_ip1=pn["U"], lam_ip1=pn["lam"]))
            self.legs.append((pi["C"], pn["C"]))
        self.pieces = lib.predict_wavefunction(self.ctx, items, self.qp, d.cfg["lam_floor"])
        self.right_iso = lib.twosite_to_right_iso(
            self.ctx, [dict(left=A, right=B, psi=p) for (A, B), p in zip(self.legs, self.pieces)], self.qp)
        self.bond = self.legs[0][0]                 # the cell boundary: left leg of piece 1
        self.lam1 = d.prev[1]["lam"]
        self.t1 = None
        self.rho_L = self.rho_R = None
        self.cells_L = self.cells_R = 0

    # -- environments on the cell boundary (host-built starting points)
    def _dev(self, x):
        return self.torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(self.lam1.device)

    def _left_start(self):
        """Lambda_1^2 in both stored channels (charges 0) of the left layout."""
        lam = self.lam1.cpu().numpy()
        out, off = [], 0
        for _, k in self.bond:
            blk = np.diag(lam[off:off + k] ** 2)
            out += [blk, blk]                        # rows: channel 0 then channel 1, columns: the sector
            off += k
        return self._dev(np.concatenate([b.reshape(-1) for b in out]))

    def _right_start(self):
        """The identity in both stored channels (charges 0) of the right layout."""
        out = [np.hstack([np.eye(k), np.eye(k)]) for _, k in self.bond]
        return self._dev(np.concatenate([b.reshape(-1) for b in out]))

    def _probe(self, side):
        """Seeded Gaussian environment on the cell boundary (both stored channels, charges 0): a generic vector
        whose overlaps with E^k x and E^(k+1) x give t1 at the rate at which x converges."""
        import workloads
        size = lib.envL_size(self.bond, [0, 0, 0]) if side == lib.LEFT else lib.envR_size(self.bond, [0, 0, 0])
        return self._dev(workloads.gaussian(size, 61, side))

    def _left_cell(self, envs, ops_per_piece, q_in):
        """Apply one cell of left transfers to a batch of environments.  ops_per_piece[j][p] = (op1, op2) for
        environment j at piece p; q_in[j] the charge of j's operator channel.  Returns (envs, q_out)."""
        q = list(q_in)
        for p in range(self.half):
            A, B = self.legs[p]
            items = []
            for j, L in enumerate(envs):
                o1, o2 = ops_per_piece[j][p]
                W = fused_mpo(o1, o2, q[j], lib.LEFT, self.qp)
                items.append(dict(old_leg=A, new_leg=B, w=W, env_old=L, iso=self.pieces[p]))
                q[j] = W.qr[1]
            envs = [e for k in range(0, len(items), 64)             # the library takes at most 64 per call
                    for e in lib.update_env(self.ctx, lib.LEFT, items[k:k + 64])]
        return envs, q

    def _right_cell(self, R):
        for p in reversed(range(self.half)):
            A, B = self.legs[p]
            W = fused_mpo("1", "1", 0, lib.RIGHT, self.qp)
            R = lib.update_env(self.ctx, lib.RIGHT, [dict(old_leg=B, new_leg=A, w=W, env_old=R,
                                                         iso=self.right_iso[p])])[0]
        return R

    def _overlap(self, pairs):
        """[(L, qL, wl, R, wr)] -> overlaps on the cell boundary."""
        return lib.env_overlap(self.ctx, [dict(leg=self.bond, ql=qL, L=L, qr=[0, 0, 0], R=R, wl=wl, wr=wr)
                                          for (L, qL, wl, R, wr) in pairs])

    def fixed_points(self):
        """Dominant eigenvalue t1 of the cell transfer matrix and its left and right eigenvectors (as environments
        on the cell boundary), by repeated application from Lambda^2 and the identity."""
        if self.rho_L is not None:
            return self.t1
        z0 = [0, 0, 0]
        R, L = self._right_start(), self._left_start()
        ident = [[("1", "1")] * self.half]
        Lp, Rp = self._probe(lib.LEFT), self._probe(lib.RIGHT)
        prev = None
        for k in range(self.max_cells):               # right: t1 from <probe | E^k R>
            Rn = self._right_cell(R)
            a, b = self._overlap([(Lp, z0, 0, Rn, 2), (Lp, z0, 0, R, 2)])
            t = a / b
            R = Rn
            self.cells_R = k + 1
            if prev is not None and abs(t - prev) <= self.tol * abs(t) and k >= 4:
                break
            prev = t
        prev = None
        for k in range(self.max_cells):               # left: t1 from <E^k L | probe>
            (Ln,), _ = self._left_cell([L], ident, [0])
            a, b = self._overlap([(Ln, z0, 0, Rp, 2), (L, z0, 0, Rp, 2)])
            t = a / b
            L = Ln
            self.cells_L = k + 1
            if prev is not None and abs(t - prev) <= self.tol * abs(t) and k >= 4:
                break
            prev = t
        self.t1, self.rho_L, self.rho_R = t, L, R
        return t

    def position(self, label):
        """Position (from the first site of piece 1) of the first site at or after it with this label (1..l)."""
        f0 = (self.n + 2 - 1) % self.ell + 1
        return (label - f0) % self.ell

    def correlations(self, pos_pairs):
        """<s_a . s_b> for position pairs (a < b), all in one batch of operator chains."""
        self.fixed_points()
        chains, owner = [], []
        for j, (a, b) in enumerate(pos_pairs):
            if not 0 <= a < b:
                raise ValueError("positions must satisfy 0 <= a < b")
            for o1, o2, c in TERMS:
                chains.append({a: o1, b: o2})
                owner.append((j, c))
        ncell = max(b for _, b in pos_pairs) // (2 * self.half) + 1
        envs = [self.rho_L] * len(chains)
        q = [0] * len(chains)
        for cell in range(ncell):
            ops = []
            for ch in chains:
                base = 2 * self.half * cell
                ops.append([(ch.get(base + 2 * p, "1"), ch.get(base + 2 * p + 1, "1")) for p in range(self.half)])
            envs, q = self._left_cell(envs, ops, q)
        z0 = [0, 0, 0]
        num, den = [], []
        for k in range(0, len(envs), 64):
            num += self._overlap([(L, z0, 1, self.rho_R, 2) for L in envs[k:k + 64]])
            den += self._overlap([(L, z0, 0, self.rho_R, 2) for L in envs[k:k + 64]])
        out = [0.0] * len(pos_pairs)
        for (j, c), x, y in zip(owner, num, den):
            out[j] += c * x / y
        return out

    def bond_strengths(self, label_pairs):
        """{(i, j): <s_i . s_j>} for site-label pairs (i < j; j > l is a site of a later cell)."""
        pos = []
        for i, j in label_pairs:
            a = self.position(i)
            pos.append((a, a + (j - i)))
        return dict(zip(label_pairs, self.correlations(pos)))

    def correlation_function(self, label, rings):
        """<s_a . s_{a + l r}> for r = 1..rings (the same site label in later unit cells)."""
        a = self.position(label)
        return self.correlations([(a, a + self.ell * r) for r in range(1, rings + 1)])


def bond_spread(values):
    """Eqs. (15), (16) for one bond class: (average, Delta+, Delta-) of its translated bond strengths."""
    v = np.asarray(values, dtype=np.float64)
    av = float(np.mean(v))
    return av, float(np.max(v)) - av, float(np.min(v)) - av


def correlation_length(corr, r0=2):
    """Correlation length in unit cells: least-squares slope of ln|C(r)| against r over r >= r0 (Sec. 4 fits the
    decay of the correlation function with an exponential)."""
    r = np.arange(1, len(corr) + 1, dtype=np.float64)
    y = np.log(np.abs(np.asarray(corr, dtype=np.float64)))
    keep = r >= r0
    slope = np.polyfit(r[keep], y[keep], 1)[0]
    return -1.0 / slope


def decay_length(dist, corr, d_min):
    """Length of the exponential decay |C| ~ exp(-d / xi): least-squares slope of ln|C| against d over d > d_min."""
    d = np.asarray(dist, dtype=np.float64)
    y = np.log(np.abs(np.asarray(corr, dtype=np.float64)))
    keep = d > d_min
    return -1.0 / np.polyfit(d[keep], y[keep], 1)[0]


def main():
    """Run the parallel iDMRG on a workload, then measure the uniform MPS: bond strengths of the bond classes with
    their spread (Eqs. (15), (16)), the correlation function of one site label along the cylinder and its
    correlation length.  Prints one JSON line (with the truncation error eps of the last period, Eq. (14))."""
    import argparse
    import json
    import sys
    import time

    import workloads

    from .driver import IDMRG
    ap = argparse.ArgumentParser(description="observables of the uniform MPS (Sec. 4)")
    ap.add_argument("--workload", default="yc8")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--prec", default=None)
    ap.add_argument("--label", type=int, default=2, help="site label of the correlation function")
    ap.add_argument("--rings", type=int, default=8, help="unit cells of the correlation function")
    ap.add_argument("--tune-cache", default=None)
    a = ap.parse_args()
    cfg = workloads.workload(a.workload, **({"m": a.m} if a.m else {}))
    d = IDMRG(cfg, prec=a.prec)
    if a.tune_cache:
        d.ctx.load_tuning(a.tune_cache)
    n_max = a.n or cfg["n_max"]
    t0 = time.perf_counter()
    while d.n < n_max:
        d.step()
        if d.n % cfg["ell"] == 0:
            print(f"[observables] n={d.n}/{n_max} {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t_run = time.perf_counter() - t0
    t0 = time.perf_counter()
    u = UniformMPS(d)
    u.fixed_points()
    if a.workload == "yc8":
        classes = workloads.yc8_bond_classes()
    else:
        classes = {f"{i}-{j}": [(i, j)] for (i, j, _) in cfg["bonds"]}
    pairs = [p for v in classes.values() for p in v]
    bs = u.bond_strengths(pairs)
    spread = {name: dict(zip(("average", "delta_plus", "delta_minus"), bond_spread([bs[p] for p in v])))
              for name, v in classes.items()}
    corr = u.correlation_function(a.label, a.rings)
    axis = None
    if a.workload == "yc8":
        # the same correlation along the straight line of the axis (Sec. 4 sweeps i = 2, 14, 35, 47, ...), with
        # distances in nearest-neighbour units, and its decay length fitted over distances above 5 as in the paper
        sweep = workloads.yc8_axis_sweep(a.rings, a.label)
        a0 = u.position(a.label)
        vals = u.correlations([(a0, a0 + site - a.label) for site, _ in sweep[1:]])
        dist = [r for _, r in sweep[1:]]
        axis = dict(sites=[site for site, _ in sweep[1:]], distance=dist, values=vals,
                    xi=decay_length(dist, vals, 5.0))
    period = [s for s in d.steps if s["n"] > d.n - cfg["ell"] and s["i"] == 1]
    out = dict(workload=a.workload, m=cfg["m"], n=d.n, prec=d.prec, e_g=d.e_g[max(d.e_g)] if d.e_g else None,
               eps=max(s["eps"] for s in period),
               e_from_bonds=sum(J * bs[(i, j)] for (i, j, J) in cfg["bonds"]) / cfg["ell"]
               if all((i, j) in bs for (i, j, _) in cfg["bonds"]) else None,
               t1=u.t1, cells_left=u.cells_L, cells_right=u.cells_R,
               bonds={f"{i}-{j}": bs[(i, j)] for (i, j) in pairs}, classes=spread,
               correlation=dict(label=a.label, values=corr, xi_cells=correlation_length(corr)), axis=axis,
               seconds_run=round(t_run, 1), seconds_observables=round(time.perf_counter() - t0, 2))
    if a.tune_cache:
        d.ctx.save_tuning(a.tune_cache)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
