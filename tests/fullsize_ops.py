"""Full-size superblock operators of the cylinder workloads, built with the oracle only.

The MPO comes from the oracle's finite-state construction; the environments
are grown by the oracle's own Eqs. (4) and (5) from the boundary vectors
through a dozen sites on each side, with seeded random block isometries (QR
of Gaussian draws) in place of the optimised ones.  H_eff is then the
projection of the segment Hamiltonian onto an orthonormal basis, symmetric
like the real one, with legs of about a dozen U(1) sectors summing to m
states.  Shared by the full-size GPU tests and the script that stores the
oracle's ground energies of these operators (tests/golden).
"""
import numpy as np

import workloads
from oracle import layout, u1
from oracle import mpo as omp

QP = [1, -1]

# name: (workload, m, matvec policy of its benchmark configuration, smallest MPO channel count at
# the centre, left sites c of the superblock, sites grown on the right)
CONFIGS = {"yc8": ("yc8", 2048, "bf16x3", 14, 13, 12), "yc8_m4096": ("yc8", 4096, "bf16x3", 14, 15, 14),
           "yc4": ("yc4", 1024, "f32", 14, 13, 12)}


def new_leg(m, rows_of, charges):
    """min(m, rows) states shared over the charges in proportion to a Gaussian profile (one state
    at a time to the sector of largest weight per state), within each sector's number of rows."""
    qs = sorted(charges)
    w = [np.exp(-((q / 2.0) ** 2) / 8.0) for q in qs]
    cap = [rows_of(q) for q in qs]
    k = [0] * len(qs)
    for _ in range(min(m, sum(cap))):
        i = max((i for i in range(len(qs)) if k[i] < cap[i]), key=lambda i: w[i] / (k[i] + 1))
        k[i] += 1
    return [(q, kq) for q, kq in zip(qs, k) if kq > 0]


def isometry(rows_of_sector, C, key):
    """Seeded block isometry {(row leg index, physical index, new charge): block} over the rows
    rows_of_sector(q) of each new sector (q, k)."""
    out = {}
    for qc, kc in C:
        rows = rows_of_sector(qc)
        r = sum(x[2] for x in rows)
        Q = np.linalg.qr(workloads.gaussian(r * kc, 77, key, qc + 1000).reshape(r, kc))[0]
        r0 = 0
        for row in rows:
            out[(row[0], row[1], qc)] = Q[r0:r0 + row[2]]
            r0 += row[2]
    return out


def u_leg(A, m):
    """New leg of m states for a left isometry with rows (a, s) of leg A."""
    Ad = dict(A)
    return new_leg(m, lambda q: sum(Ad.get(q - s, 0) for s in QP), {qa + s for qa, _ in A for s in QP})


def v_leg(B, m):
    """New leg of m states for a right isometry with rows (s, b) of leg B."""
    Bd = dict(B)
    return new_leg(m, lambda q: sum(Bd.get(q + s, 0) for s in QP), {qb - s for qb, _ in B for s in QP})


def grow(name, m, c, nright):
    """Environments of superblock (sites c, c+1) of a cylinder workload with legs of about m states."""
    cfg = workloads.workload(name)
    ell = cfg["ell"]
    Ws, dq = omp.build_mpo(ell, cfg["bonds"])
    f = lambda k: (k - 1) % ell + 1
    W = lambda k: Ws[f(k) - 1]
    cut = lambda k: dq[f(k)]
    L, A = u1.init_left(W(1), cut(1), QP)
    for j in range(2, c):
        C = u_leg(A, m)
        L = u1.update_env_left(L, W(j), isometry(lambda q: layout.U_rows(A, QP, q), C, j), A, QP, C, cut(j - 1),
                               cut(j))
        A = C
    K = c + 1 + nright
    R, B = u1.init_right(W(K), cut(K - 1), QP)
    for j in range(K - 1, c + 1, -1):
        C = v_leg(B, m)
        R = u1.update_env_right(R, W(j), isometry(lambda q: layout.V_rows(B, QP, q), C, 1000 + j), B, QP, C,
                                cut(j - 1), cut(j))
        B = C
    return dict(L=L, A=A, R=R, B=B, W1=W(c), W2=W(c + 1), dl=cut(c - 1), dm=cut(c), dr=cut(c + 1))


def operator(name):
    """The full-size superblock of CONFIGS[name] and its matvec (oracle arithmetic)."""
    wl, m, prec, dmin, c, nright = CONFIGS[name]
    s = grow(wl, m, c, nright)
    s.update(name=wl, m=m, prec=prec, dmin=dmin)
    A, B = s["A"], s["B"]
    s["N"] = layout.psi_size(A, B, QP)

    def mv(x):
        return layout.psi_to_flat(u1.heff_apply(s["L"], s["W1"], s["W2"], s["R"], layout.flat_to_psi(x, A, B, QP),
                                                A, B, QP, s["dl"], s["dr"]), A, B, QP)
    s["mv"] = mv
    return s
