"""Finite-state MPO of a Heisenberg model with an l-site period (oracle).

Test infrastructure only (see ``oracle/__init__``).

The paper writes the Hamiltonian as a product of operator-valued matrices W_i
that are lower triangular; the left boundary vector is the last row of W and
the right boundary vector is its first column (Sec. 2, Eq. (1) and the text
after it).  For an l-periodic model the same l tensors repeat (Sec. 3,
Eq. (7)).

Channel meaning at a cut (the bond between site c and c+1), in this order:
  0           the part to the left of the cut already holds complete terms
  1+3p+{0,1,2} site j_p (left of the cut) has applied S+, S-, S^z and waits for
              its partner to the right
  D-1         nothing has been applied yet (identity)
W_c[w, w', s, s'] maps channel w at cut c-1 to channel w' at cut c with the
site operator <s| . |s'> of site c.  A bond J s_j . s_k (j < k) opens at j with
(S+, S-, S^z), is carried by identities, and closes at k with
(J/2 S-, J/2 S+, J S^z); its terms are J/2 (S+_j S-_k + S-_j S+_k) + J S^z_j S^z_k.

Channel charges (2*S^z added to the left part by the operator in that
channel) are 0 for complete/identity, +2 for S+, -2 for S-, 0 for S^z.
"""
from __future__ import annotations

import numpy as np

# local basis [up, down], charges 2*S^z = [+1, -1]
QP = (1, -1)
SP = np.array([[0.0, 1.0], [0.0, 0.0]])   # |up><down|
SM = SP.T.copy()
SZ = np.diag([0.5, -0.5])
ID = np.eye(2)


def _absolute_bonds(ell, cell_bonds, lo, hi):
    """Translated bonds (j, k, J) of the infinite model with j <= hi and k > lo."""
    out = []
    rng = max(k2 - k for (k, k2, _) in cell_bonds) if cell_bonds else 0
    tmin = (lo - rng - ell) // ell - 1
    tmax = hi // ell + 1
    for (k, k2, J) in cell_bonds:
        for t in range(tmin, tmax + 1):
            j, j2 = k + t * ell, k2 + t * ell
            if j <= hi and j2 > lo:
                out.append((j, j2, J))
    return out


def pending_sources(ell, cell_bonds, c):
    """Sites j <= c (absolute index) that have a bond partner k > c."""
    srcs = set()
    for (j, k, _) in _absolute_bonds(ell, cell_bonds, c, c):
        if j <= c < k:
            srcs.add(j)
    return sorted(srcs)


def coupling(ell, cell_bonds, j, k):
    """Total coupling J between absolute sites j < k."""
    tot = 0.0
    for (a, b, J) in _absolute_bonds(ell, cell_bonds, k - 1, j):
        if a == j and b == k:
            tot += J
    return tot


def channel_charges(sources):
    return np.array([0] + [q for _ in sources for q in (2, -2, 0)] + [0], dtype=np.int64)


def build_mpo(ell, cell_bonds):
    """Return (W, dq): W[c-1] is W_c (c = 1..l) with shape [D_{c-1}, D_c, 2, 2];
    dq[c] holds the channel charges at cut c (c = 0..l, cut 0 == cut l)."""
    P = {c: pending_sources(ell, cell_bonds, c) for c in range(1, ell + 1)}
    P[0] = [j - ell for j in P[ell]]
    dq = [channel_charges(P[c]) for c in range(ell + 1)]
    Ws = []
    for c in range(1, ell + 1):
        pin, pout = P[c - 1], P[c]
        din, dout = 2 + 3 * len(pin), 2 + 3 * len(pout)
        W = np.zeros((din, dout, 2, 2))
        W[0, 0] = ID
        W[din - 1, dout - 1] = ID
        if c in pout:                      # site c opens its bonds
            p = pout.index(c)
            W[din - 1, 1 + 3 * p + 0] = SP
            W[din - 1, 1 + 3 * p + 1] = SM
            W[din - 1, 1 + 3 * p + 2] = SZ
        for a, j in enumerate(pin):
            J = coupling(ell, cell_bonds, j, c)
            if J != 0.0:                   # bond (j, c) closes here
                W[1 + 3 * a + 0, 0] += 0.5 * J * SM
                W[1 + 3 * a + 1, 0] += 0.5 * J * SP
                W[1 + 3 * a + 2, 0] += J * SZ
            if j in pout:                  # still waiting for a later partner
                b = pout.index(j)
                for t in range(3):
                    W[1 + 3 * a + t, 1 + 3 * b + t] = ID
        Ws.append(W)
    return Ws, dq


def f_index(k, ell):
    """f(k) = 1 + mod(k-1, l) (Sec. 3, Step 2')."""
    return 1 + (k - 1) % ell


def mpo_segment_matrix(Ws, ell, first, last):
    """Contract L_first W ... R_last into a dense 2^N x 2^N matrix (Eq. (1)).

    L is the last row of W_first and R the first column of W_last.
    Site order in the tensor product: first site is the most significant.
    """
    N = last - first + 1
    W0 = Ws[f_index(first, ell) - 1]
    cur = [W0[W0.shape[0] - 1, w] for w in range(W0.shape[1])]    # operators per channel
    for site in range(first + 1, last + 1):
        W = Ws[f_index(site, ell) - 1]
        if site < last:
            nxt = []
            for w2 in range(W.shape[1]):
                acc = np.zeros((cur[0].shape[0] * 2,) * 2)
                for w in range(W.shape[0]):
                    if np.any(W[w, w2]):
                        acc += np.kron(cur[w], W[w, w2])
                nxt.append(acc)
            cur = nxt
        else:
            acc = np.zeros((cur[0].shape[0] * 2,) * 2)
            for w in range(W.shape[0]):
                if np.any(W[w, 0]):
                    acc += np.kron(cur[w], W[w, 0])
            cur = [acc]
    assert cur[0].shape == (2 ** N, 2 ** N)
    return cur[0]


def bond_sum_matrix(bonds, first, last):
    """Dense sum_{(i,j,J)} J s_i . s_j on sites first..last (first site most significant)."""
    N = last - first + 1
    H = np.zeros((2 ** N, 2 ** N))

    def op_at(op, site):
        m = np.eye(1)
        for s in range(first, last + 1):
            m = np.kron(m, op if s == site else ID)
        return m

    for (i, j, J) in bonds:
        H += J * (0.5 * (op_at(SP, i) @ op_at(SM, j) + op_at(SM, i) @ op_at(SP, j))
                  + op_at(SZ, i) @ op_at(SZ, j))
    return H
