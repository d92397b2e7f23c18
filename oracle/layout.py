"""Canonical flat storage order of block-sparse tensors (oracle's own reading).

Test infrastructure only (see ``oracle/__init__``).

The C-ABI exchanges every tensor as one flat FP64 array whose order is fixed by
the rules below.  This module implements those rules for the oracle's
dictionary-of-blocks representation; the library implements the same rules
in its own code.  Nothing here computes any part of the method.

Charges are 2*S^z and follow the left-flux convention: the charge of a bond
sector is the total charge of everything to the left of that bond.  A leg is a
list of (charge, dim) with strictly ascending charge.  The local basis has
charges ``qp``.

* Two-site state Psi[alpha, s1, s2, beta] with legs A (alpha) and B (beta):
  blocks for b in B, a in A, s1, s2 (each ascending) with
  q_a + qp[s1] + qp[s2] == q_b; each block [dim_a x dim_b] row-major.
* Left environment L[alpha, w, alpha'] with channel charges dl (D channels;
  channel D-1 is the identity and is not stored): for a' in A, for w = 0..D-2,
  if q_a' + dl[w] is a sector a of A: block [dim_a x dim_a'] row-major.
* Right environment R[beta, w, beta'] with channel charges dr (channel 0 is
  the identity and is not stored): for b in B, one row-major matrix
  [dim_b x K_b] whose columns run over w = 1..D-1 and the sector b' with
  q_b' = q_b - dr[w] (if present).
* Left isometry U[(alpha, s), gamma]: for c in the new leg C, a row-major
  [r_c x k_c] matrix with rows over a in A, s (ascending) where
  q_a + qp[s] == q_c.
* Right isometry V[(s, beta), gamma]: for c in C, a row-major [r'_c x k_c]
  matrix with rows over s, b in B (ascending) where q_b - qp[s] == q_c.
* Singular values: for c in C, k_c values.
"""
from __future__ import annotations

import numpy as np


def leg_dict(leg):
    return {int(q): int(d) for q, d in leg}


# ----------------------------------------------------------------- two-site state

def psi_keys(A, B, qp):
    Bd = leg_dict(B)
    keys = []
    for qb, _ in B:
        for qa, _ in A:
            for s1 in range(len(qp)):
                for s2 in range(len(qp)):
                    if qa + qp[s1] + qp[s2] == qb:
                        keys.append((qa, s1, s2))
    assert all(k[0] + qp[k[1]] + qp[k[2]] in Bd for k in keys)
    return keys


def psi_size(A, B, qp):
    Ad, Bd = leg_dict(A), leg_dict(B)
    return sum(Ad[a] * Bd[a + qp[s1] + qp[s2]] for (a, s1, s2) in psi_keys(A, B, qp))


def psi_to_flat(psi, A, B, qp):
    parts = [np.asarray(psi[k]).reshape(-1) for k in psi_keys(A, B, qp)]
    return np.concatenate(parts) if parts else np.zeros(0)


def flat_to_psi(x, A, B, qp):
    Ad, Bd = leg_dict(A), leg_dict(B)
    out, off = {}, 0
    for (a, s1, s2) in psi_keys(A, B, qp):
        r, c = Ad[a], Bd[a + qp[s1] + qp[s2]]
        out[(a, s1, s2)] = np.array(x[off:off + r * c]).reshape(r, c)
        off += r * c
    assert off == len(x)
    return out


# ----------------------------------------------------------------- environments

def envL_to_flat(L, A, dl):
    Ad = leg_dict(A)
    parts = []
    for qc, _ in A:
        for w in range(len(dl) - 1):
            qr = qc + int(dl[w])
            if qr in Ad:
                parts.append(np.asarray(L.get((w, qr, qc), np.zeros((Ad[qr], Ad[qc])))).reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)


def flat_to_envL(x, A, dl):
    """Inverse of envL_to_flat; the identity channel D-1 is filled in explicitly."""
    Ad = leg_dict(A)
    L, off = {}, 0
    for qc, dc in A:
        for w in range(len(dl) - 1):
            qr = qc + int(dl[w])
            if qr in Ad:
                n = Ad[qr] * dc
                L[(w, qr, qc)] = np.array(x[off:off + n]).reshape(Ad[qr], dc)
                off += n
    assert off == len(x)
    for q, d in A:
        L[(len(dl) - 1, q, q)] = np.eye(d)
    return L


def envR_cols(B, dr, qb):
    Bd = leg_dict(B)
    cols = []
    for w in range(1, len(dr)):
        qc = qb - int(dr[w])
        if qc in Bd:
            cols.append((w, qc, Bd[qc]))
    return cols


def envR_to_flat(R, B, dr):
    Bd = leg_dict(B)
    parts = []
    for qb, db in B:
        cols = envR_cols(B, dr, qb)
        if not cols:
            continue
        M = np.concatenate([np.asarray(R.get((w, qb, qc), np.zeros((db, dc)))) for (w, qc, dc) in cols],
                           axis=1)
        parts.append(M.reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)


def flat_to_envR(x, B, dr):
    """Inverse of envR_to_flat; the identity channel 0 is filled in explicitly."""
    R, off = {}, 0
    for qb, db in B:
        cols = envR_cols(B, dr, qb)
        K = sum(dc for (_, _, dc) in cols)
        if K == 0:
            continue
        M = np.array(x[off:off + db * K]).reshape(db, K)
        off += db * K
        c0 = 0
        for (w, qc, dc) in cols:
            R[(w, qb, qc)] = M[:, c0:c0 + dc].copy()
            c0 += dc
    assert off == len(x)
    for q, d in B:
        R[(0, q, q)] = np.eye(d)
    return R


def envL_size(A, dl):
    Ad = leg_dict(A)
    return sum(Ad[qc + int(dl[w])] * dc for qc, dc in A for w in range(len(dl) - 1)
               if qc + int(dl[w]) in Ad)


def envR_size(B, dr):
    return sum(db * sum(dc for (_, _, dc) in envR_cols(B, dr, qb)) for qb, db in B)


# ----------------------------------------------------------------- isometries

def U_rows(A, qp, qc):
    Ad = leg_dict(A)
    return [(qa, s, Ad[qa]) for qa, _ in A for s in range(len(qp)) if qa + qp[s] == qc]


def V_rows(B, qp, qc):
    Bd = leg_dict(B)
    return [(s, qb, Bd[qb]) for s in range(len(qp)) for qb, _ in B if qb - qp[s] == qc]


def U_to_flat(U, A, qp, C):
    parts = []
    for qc, kc in C:
        rows = U_rows(A, qp, qc)
        if rows:
            parts.append(np.concatenate([U[(qa, s, qc)] for (qa, s, _) in rows], axis=0).reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)


def flat_to_U(x, A, qp, C):
    U, off = {}, 0
    for qc, kc in C:
        for (qa, s, da) in U_rows(A, qp, qc):
            U[(qa, s, qc)] = np.array(x[off:off + da * kc]).reshape(da, kc)
            off += da * kc
    assert off == len(x)
    return U


def V_to_flat(V, B, qp, C):
    parts = []
    for qc, kc in C:
        rows = V_rows(B, qp, qc)
        if rows:
            parts.append(np.concatenate([V[(s, qb, qc)] for (s, qb, _) in rows], axis=0).reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)


def flat_to_V(x, B, qp, C):
    V, off = {}, 0
    for qc, kc in C:
        for (s, qb, db) in V_rows(B, qp, qc):
            V[(s, qb, qc)] = np.array(x[off:off + db * kc]).reshape(db, kc)
            off += db * kc
    assert off == len(x)
    return V


def lam_to_flat(lam, C):
    return np.concatenate([np.asarray(lam[qc]) for qc, _ in C]) if C else np.zeros(0)


def flat_to_lam(x, C):
    out, off = {}, 0
    for qc, kc in C:
        out[qc] = np.array(x[off:off + kc])
        off += kc
    return out
