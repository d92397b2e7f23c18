"""Sparse exact diagonalisation of open Heisenberg segments (oracle pin).

Test infrastructure only (see ``oracle/__init__``).

While no state is discarded, every superblock of the iDMRG holds the exact
ground state of its open segment (Sec. 2, Steps 2-4 keep min(d^n, m) states,
which is the full block space for d^n <= m).  This module computes that
ground-state energy directly from the bond list, in the 2*S^z_total = 0
sector, with no MPO involved.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def sz0_states(N):
    """All N-bit configurations with N/2 down spins (bit set = down), ascending."""
    allc = np.arange(2 ** N, dtype=np.int64)
    pop = np.zeros_like(allc)
    for b in range(N):
        pop += (allc >> b) & 1
    return allc[pop == N // 2]


def segment_hamiltonian_sz0(bonds, first, last):
    """Sparse H = sum J s_i . s_j restricted to S^z_total = 0 on sites first..last."""
    N = last - first + 1
    assert N % 2 == 0
    st = sz0_states(N)
    dim = st.size
    diag = np.zeros(dim)
    rows, cols, vals = [], [], []
    for (i, j, J) in bonds:
        bi = np.int64(1) << (i - first)
        bj = np.int64(1) << (j - first)
        si = ((st & bi) != 0)
        sj = ((st & bj) != 0)
        same = si == sj
        diag += np.where(same, 0.25 * J, -0.25 * J)
        idx = np.nonzero(~same)[0]
        flipped = st[idx] ^ (bi | bj)
        tgt = np.searchsorted(st, flipped)
        rows.append(tgt)
        cols.append(idx)
        vals.append(np.full(idx.size, 0.5 * J))
    rows.append(np.arange(dim))
    cols.append(np.arange(dim))
    vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim))
    return H


def ground_energy(bonds, first, last):
    """Lowest eigenvalue of the open segment first..last in S^z_total = 0."""
    H = segment_hamiltonian_sz0(bonds, first, last)
    if H.shape[0] <= 400:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    vals = sla.eigsh(H, k=1, which="SA", tol=0.0, return_eigenvectors=False)
    return float(vals[0])
