"""Hot-path steps inside U(1) S^z blocks (oracle).

Test infrastructure only (see ``oracle/__init__``).

Representation (dictionaries of dense FP64 blocks, charges 2*S^z in the
left-flux convention, see ``layout``):

* leg            list of (charge, dim), ascending charge
* psi            {(qa, s1, s2): [dim_a, dim_b]} with qb = qa + qp[s1] + qp[s2]
* environment    {(w, q_row, q_col): [dim_row, dim_col]}, every channel stored,
                 q_row = q_col + dq[w]
* U              {(qa, s, qc): [dim_a, k_c]}   (qc = qa + qp[s])
* V              {(s, qb, qc): [dim_b, k_c]}   (qc = qb - qp[s])
* lam            {qc: [k_c]}

The paper itself runs without symmetry blocks (Sec. 4) and notes that abelian
symmetries are compatible with the method; ``dense`` holds the unblocked
version and the tests require both to agree.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from . import layout


# ------------------------------------------------------------------ Step 1

def init_left(W, dq_out, qp):
    """L^(0) = last row of W (Sec. 2, Step 1; boundary vectors after Eq. (1)).

    Returns (env, leg); the block index is the single site's state.
    """
    Dl = W.shape[0]
    leg = sorted({(int(q), sum(1 for x in qp if x == q)) for q in qp})
    env = {}
    for w in range(W.shape[1]):
        for s in range(len(qp)):
            for t in range(len(qp)):
                v = W[Dl - 1, w, s, t]
                if v != 0.0:
                    env[(w, qp[s], qp[t])] = _site_block(env.get((w, qp[s], qp[t])), qp, s, t, v, +1)
    return _fill_missing(env, leg, dq_out), leg


def init_right(W, dq_in, qp):
    """R^(0) = first column of W (Sec. 2, Step 1).  Sector charge of a right
    block state is minus its own 2*S^z (left-flux convention)."""
    leg = sorted({(int(-q), sum(1 for x in qp if x == q)) for q in qp})
    env = {}
    for w in range(W.shape[0]):
        for s in range(len(qp)):
            for t in range(len(qp)):
                v = W[w, 0, s, t]
                if v != 0.0:
                    env[(w, -qp[s], -qp[t])] = _site_block(env.get((w, -qp[s], -qp[t])), qp, s, t, v, -1)
    return _fill_missing(env, leg, dq_in), leg


def _site_block(blk, qp, s, t, v, sign):
    """Place value v at (index of s in its sector, index of t in its sector)."""
    qs, qt = sign * qp[s], sign * qp[t]
    ds = sum(1 for x in qp if sign * x == qs)
    dt = sum(1 for x in qp if sign * x == qt)
    if blk is None:
        blk = np.zeros((ds, dt))
    i = [k for k in range(len(qp)) if sign * qp[k] == qs].index(s)
    j = [k for k in range(len(qp)) if sign * qp[k] == qt].index(t)
    blk[i, j] += v
    return blk


def _fill_missing(env, leg, dq):
    d = dict(leg)
    for w in range(len(dq)):
        for qc, dc in leg:
            qr = qc + int(dq[w])
            if qr in d and (w, qr, qc) not in env:
                env[(w, qr, qc)] = np.zeros((d[qr], dc))
    return env


def state_index(qp, s, sign):
    """(sector charge, index inside the sector) of local state s in a single-site leg."""
    q = sign * qp[s]
    return q, [k for k in range(len(qp)) if sign * qp[k] == q].index(s)


# ------------------------------------------------------------------ Step 3: H_eff

def w12_terms(W1, W2):
    """Nonzero coefficients of sum_w' W1[w,w',s1,t1] W2[w',w'',s2,t2], grouped by (s1, s2)."""
    C = np.einsum("wvsS,vutT->wustST", W1, W2)
    terms = {}
    for idx in zip(*np.nonzero(C)):
        w, u, s1, s2, t1, t2 = (int(x) for x in idx)
        terms.setdefault((s1, s2), []).append((w, u, t1, t2, float(C[idx])))
    return terms


def heff_apply(L, W1, W2, R, psi, A, B, qp, dl, dr):
    """y = H^(n)_i psi (Sec. 2, Step 3; Fig. 2(b)).

    y[a,s1,s2,b] = sum L[a,w,a'] W1[w,w',s1,t1] W2[w',w'',s2,t2] R[b,w'',b'] psi[a',t1,t2,b'].
    """
    Ad, Bd = layout.leg_dict(A), layout.leg_dict(B)
    terms = w12_terms(W1, W2)
    cache = {}
    y = {}
    for (qa, s1, s2) in layout.psi_keys(A, B, qp):
        qb = qa + qp[s1] + qp[s2]
        acc = np.zeros((Ad[qa], Bd[qb]))
        for (w, u, t1, t2, c) in terms.get((s1, s2), ()):
            qa2, qb2 = qa - int(dl[w]), qb - int(dr[u])
            x = psi.get((qa2, t1, t2))
            Lb, Rb = L.get((w, qa, qa2)), R.get((u, qb, qb2))
            if x is None or Lb is None or Rb is None:
                continue
            assert qb2 == qa2 + qp[t1] + qp[t2]
            key = (w, qa, qa2, t1, t2)
            if key not in cache:
                cache[key] = Lb @ x
            acc += c * (cache[key] @ Rb.T)
        y[(qa, s1, s2)] = acc
    return y


# ------------------------------------------------------------------ Step 4: SVD + truncation

def center_sectors(A, B, qp):
    """Row groups (qa, s1) and column groups (s2, qb) of Psi for each centre charge."""
    out = {}
    for qa, da in A:
        for s1 in range(len(qp)):
            out.setdefault(qa + qp[s1], [[], []])[0].append((qa, s1, da))
    for s2 in range(len(qp)):
        for qb, db in B:
            out.setdefault(qb - qp[s2], [[], []])[1].append((s2, qb, db))
    return {q: v for q, v in sorted(out.items()) if v[0] and v[1]}


def svd(M):
    """Thin SVD by LAPACK gesdd, falling back to gesvd."""
    try:
        return sl.svd(M, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return sl.svd(M, full_matrices=False, lapack_driver="gesvd")


def select_kept(cands, m, lam_floor, deg_rel):
    """Choose the kept Schmidt states from candidates [(lam, q, j)].

    Step 4/6 keep the largest min(d^{n+1}, m) singular values (the printed
    ascending order is read as descending, since Eqs. (13)-(14) sum the m
    largest).  Readings taken here:
    * candidates with lam <= lam_floor count as zero (Eq. (10)'s lam = 0 case);
    * the kept count is min(m, number of candidates); when it exceeds the
      number of nonzero values, zero-weight states fill it (in ascending
      sector charge, then decomposition order) only if every candidate is
      kept, since then the kept space is the whole two-site block space and
      does not depend on which null vectors the decomposition returned;
      otherwise only the nonzero values are kept (a subset of the null space
      would be an arbitrary choice that changes later iterations' energies);
    * a cut never splits a near-degenerate multiplet: while the last kept and
      first discarded nonzero values differ by <= deg_rel * last kept, one
      fewer state is kept (if that would keep nothing, the plain cut is used).
    Returns (kept list, relative gap at the cut or None).
    """
    pos = sorted([c for c in cands if c[0] > lam_floor], key=lambda t: (-t[0], t[1], t[2]))
    zer = sorted([c for c in cands if c[0] <= lam_floor], key=lambda t: (t[1], t[2]))
    target = min(m, len(cands))
    if target < len(pos):
        mk = target
        while mk > 0 and pos[mk - 1][0] - pos[mk][0] <= deg_rel * pos[mk - 1][0]:
            mk -= 1
        if mk == 0:
            mk = target
        gap = (pos[mk - 1][0] - pos[mk][0]) / pos[mk - 1][0]
        return pos[:mk], gap
    if target == len(cands):
        return pos + zer, None
    return pos, None


def truncate_twosite(psi, A, B, qp, m, lam_floor=1e-14, deg_rel=1e-5):
    """Psi = U Lambda V^dagger per centre charge, keep the largest states (Steps 4, 6).

    Returns dict(C, U, V, lam, eps, eps_prime, m_kept, cut_gap, spectrum) where
    eps = 1 - sum_kept lam^2 (Eq. (14)) and eps_prime = 1 - sqrt(sum_kept lam^2)
    (Eq. (13)) with the full spectrum normalised to sum lam^2 = 1.
    """
    secs = center_sectors(A, B, qp)
    dec = {}
    for q, (rows, cols) in secs.items():
        M = np.zeros((sum(r[2] for r in rows), sum(c[2] for c in cols)))
        r0 = 0
        for (qa, s1, da) in rows:
            c0 = 0
            for (s2, qb, db) in cols:
                blk = psi.get((qa, s1, s2))
                if blk is not None and qa + qp[s1] + qp[s2] == qb:
                    M[r0:r0 + da, c0:c0 + db] = blk
                c0 += db
            r0 += da
        dec[q] = svd(M)
    total = sum(float(np.sum(S ** 2)) for (_, S, _) in dec.values())
    norm = np.sqrt(total)
    cands = [(float(S[j]) / norm, q, j) for q, (_, S, _) in dec.items() for j in range(len(S))]
    kept, gap = select_kept(cands, m, lam_floor, deg_rel)
    per = {}
    for (lam, q, j) in kept:
        per.setdefault(q, []).append((j, lam if lam > lam_floor else 0.0))
    C = [(q, len(per[q])) for q in sorted(per)]
    U, V, lamd = {}, {}, {}
    for q, lst in per.items():
        Uq, _, Vtq = dec[q]
        js = [j for j, _ in lst]
        lamd[q] = np.array([l for _, l in lst])
        rows, cols = secs[q]
        r0 = 0
        for (qa, s1, da) in rows:
            U[(qa, s1, q)] = Uq[r0:r0 + da, js].copy()
            r0 += da
        c0 = 0
        for (s2, qb, db) in cols:
            V[(s2, qb, q)] = Vtq[js, c0:c0 + db].T.copy()
            c0 += db
    kept_w = sum(l * l for (l, _, _) in kept if l > lam_floor)
    kept_set = {(q, j) for (_, q, j) in kept}
    eps = sum(l * l for (l, q, j) in cands if (q, j) not in kept_set)
    eps_prime = eps / (1.0 + np.sqrt(max(0.0, 1.0 - eps)))
    spectrum = sorted((l for (l, _, _) in cands), reverse=True)
    return dict(C=C, U=U, V=V, lam=lamd, eps=eps, eps_prime=eps_prime, kept_weight=kept_w,
                m_kept=len(kept), cut_gap=gap, spectrum=np.array(spectrum))


# ------------------------------------------------------------------ Step 6: block-spin transformation

def update_env_left(L, W1, U, A, qp, C, dl, dm):
    """L^(n)[w'](c, c') = sum u*[(a,s),c] L[w](a,a') W1[w,w',s,s'] u[(a',s'),c'] (Eq. (4)).

    Every channel w' of the new cut is computed, the identity channel included.
    """
    Cd = layout.leg_dict(C)
    out = {}
    for w in range(W1.shape[0]):
        for w2 in range(W1.shape[1]):
            for s in range(len(qp)):
                for t in range(len(qp)):
                    c = W1[w, w2, s, t]
                    if c == 0.0:
                        continue
                    for (qa2, t_, qc2), Ub2 in U.items():
                        if t_ != t:
                            continue
                        qa = qa2 + int(dl[w])
                        Lb = L.get((w, qa, qa2))
                        qc = qa + qp[s]
                        Ub = U.get((qa, s, qc))
                        if Lb is None or Ub is None:
                            continue
                        key = (w2, qc, qc2)
                        out[key] = out.get(key, 0.0) + c * (Ub.T @ Lb @ Ub2)
    for w2 in range(W1.shape[1]):
        for qc2, d2 in C:
            qc = qc2 + int(dm[w2])
            if qc in Cd and (w2, qc, qc2) not in out:
                out[(w2, qc, qc2)] = np.zeros((Cd[qc], d2))
    return out


def update_env_right(R, W2, V, B, qp, C, dm, dr):
    """R^(n)[w](c, c') = sum v[(s,b),c] W2[w,w'',s,s'] R[w''](b,b') v*[(s',b'),c'] (Eq. (5),
    with the garbled index placement read so that v acts on the left and v* on
    the right, consistent with Psi = U Lambda V^dagger)."""
    Cd = layout.leg_dict(C)
    out = {}
    for w in range(W2.shape[0]):
        for u in range(W2.shape[1]):
            for s in range(len(qp)):
                for t in range(len(qp)):
                    c = W2[w, u, s, t]
                    if c == 0.0:
                        continue
                    for (t_, qb2, qc2), Vb2 in V.items():
                        if t_ != t:
                            continue
                        qb = qb2 + int(dr[u])
                        Rb = R.get((u, qb, qb2))
                        qc = qb - qp[s]
                        Vb = V.get((s, qb, qc))
                        if Rb is None or Vb is None:
                            continue
                        key = (w, qc, qc2)
                        out[key] = out.get(key, 0.0) + c * (Vb.T @ Rb @ Vb2)
    for w in range(W2.shape[0]):
        for qc2, d2 in C:
            qc = qc2 + int(dm[w])
            if qc in Cd and (w, qc, qc2) not in out:
                out[(w, qc, qc2)] = np.zeros((Cd[qc], d2))
    return out


# ------------------------------------------------------------------ Step 3': prediction

def inverse_lambda(lam, lam_floor):
    """1/lambda for lambda > lam_floor, 0 otherwise (the two cases of Eq. (10))."""
    return {q: np.where(v > lam_floor, 1.0 / np.where(v > lam_floor, v, 1.0), 0.0) for q, v in lam.items()}


def predict_wavefunction(lam_i, V_i, lam_ip1_prev, U_ip1, lam_ip1, A, B, qp, lam_floor=1e-14):
    """Initial vector of superblock (n, i) by Eq. (10).

    psi~[a,s,s',a'] = sum_b lam^(n-1)_i[a] v^(n-1)*_i[(s,b),a] u~^(n-1)_{i+1}[b,s',a'],
    u~[b,s',a'] = u^(n-1)_{i+1}[(b,s'),a'] lam^(n-1)_{i+1}[a'] / lam^(n-2)_{i+1}[b] (0 if that
    lambda is zero).  A is the leg of lam_i (the new left block), B the leg of
    lam_ip1 (the new right block).
    """
    Ad, Bd = layout.leg_dict(A), layout.leg_dict(B)
    inv = inverse_lambda(lam_ip1_prev, lam_floor)
    out = {}
    for (qa, s1, s2) in layout.psi_keys(A, B, qp):
        qbeta = qa + qp[s1]
        qb = qbeta + qp[s2]
        Vb = V_i.get((s1, qbeta, qa))
        Ub = U_ip1.get((qbeta, s2, qb))
        if Vb is None or Ub is None or qbeta not in inv:
            out[(qa, s1, s2)] = np.zeros((Ad[qa], Bd[qb]))
            continue
        left = lam_i[qa][:, None] * Vb.T                      # [dim_a, dim_beta]
        ut = (inv[qbeta][:, None] * Ub) * lam_ip1[qb][None, :]  # [dim_beta, dim_b]
        out[(qa, s1, s2)] = left @ ut
    return out
