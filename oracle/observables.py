"""Observables of the translation-invariant MPS of the parallel iDMRG (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 3, Eq. (11): after iteration n, away from its two ends, the wavefunction
is the repetition of one unit cell of l sites made of the l/2 two-site pieces

    B_i = V^(n)dagger_i  U~^(n)_{i+1},    i = 1..l/2  (i + 1 taken cyclically),

where U~^(n)_{i+1} is U^(n)_{i+1} divided on its left bond by the Schmidt
values of superblock i+1 at iteration n-1 and multiplied on its right bond by
those at iteration n (the tensor of Eq. (10)).  So B_i is the two-site state
Eq. (10) predicts for superblock i at iteration n+1, without its left factor
lambda^(n)_i.  Piece i holds the sites n + 2i and n + 2i + 1 (site labels
f(k) = 1 + mod(k - 1, l)); its left bond is the kept-state bond of superblock
i and its right bond that of superblock i+1.

Expectation values in the infinite MPS (Sec. 4: bond strengths, Eqs. (15),
(16); the correlation length) come from the transfer matrix of one cell,

    E(X)[b, b'] = sum_{a, a', s} B[a, s, b] X[a, a'] B[a', s, b']      (pieces in order),

through its dominant eigenvalue t1 with left and right eigenvectors rho_L and
rho_R:  <O> = rho_R . E_O(rho_L) / (t1^k rho_R . rho_L) for an operator O on k
cells, E_O being E with the operators inserted into the pieces they act on.
The correlation length in cells is -1 / ln(|t2| / |t1|), t2 the eigenvalue of
second largest modulus.

Dense arrays (no symmetry blocks); the transfer matrix is built explicitly
(m^2 x m^2) and diagonalised with a library routine, which suits the small
cases the tests use.
"""
from __future__ import annotations

import numpy as np

from . import dense

# spin-1/2 operators in the local basis (0: up, 1: down; charges 2 S^z = +1, -1)
SZ = np.diag([0.5, -0.5])
SP = np.array([[0.0, 1.0], [0.0, 0.0]])     # <up| S+ |down> = 1
SM = SP.T.copy()
ID = np.eye(2)


def pieces(cur, prev_lam, lam_floor):
    """Eq. (11) unit cell from the decompositions of iteration n.

    cur: {i: truncation of superblock i at iteration n} (dense: U[a,s,c],
    V[s,b,c], lam[c]); prev_lam: {i: Schmidt values of superblock i at
    iteration n-1}.  Returns [B_1, ..., B_{l/2}], B_i[a, s1, s2, b]."""
    half = len(cur)
    out = []
    for i in range(1, half + 1):
        ip1 = i % half + 1
        ones = np.ones_like(cur[i]["lam"])
        out.append(dense.predict_wavefunction(ones, cur[i]["V"], prev_lam[ip1], cur[ip1]["U"], cur[ip1]["lam"],
                                              lam_floor))
    return out


def piece_sites(n, half):
    """Absolute sites (k1, k2) of pieces 1..l/2 of the unit cell after iteration n."""
    return [(n + 2 * i, n + 2 * i + 1) for i in range(1, half + 1)]


def apply_piece(X, B, op1=None, op2=None):
    """E_B(X) with op1 on the first and op2 on the second site of the piece (None: identity)."""
    o1 = ID if op1 is None else op1
    o2 = ID if op2 is None else op2
    T = np.einsum("aA,AtuB->atuB", X, B)            # X[a, a'] B[a', t, u, b']
    T = np.einsum("st,atuB->asuB", o1, T)            # <s| op1 |t>
    T = np.einsum("vu,asuB->asvB", o2, T)            # <v| op2 |u>
    return np.einsum("asvb,asvB->bB", B, T)


def transfer_matrix(Bs):
    """M_cell with vec(E(X)) = M_cell vec(X), vec row-major over (a, a')."""
    m = Bs[0].shape[0]
    M = np.eye(m * m)
    for B in Bs:
        ma, mb = B.shape[0], B.shape[3]
        Mp = np.einsum("astb,AstB->bBaA", B, B).reshape(mb * mb, ma * ma)
        M = Mp @ M
    return M


def fixed_points(Bs):
    """(t1, rho_L, rho_R, spectrum by decreasing modulus) of the cell transfer matrix."""
    M = transfer_matrix(Bs)
    m = Bs[0].shape[0]
    w, vr = np.linalg.eig(M)
    wl, vl = np.linalg.eig(M.T)
    k, kl = int(np.argmax(np.abs(w))), int(np.argmax(np.abs(wl)))
    t1 = float(np.real(w[k]))
    rho_L = np.real(vr[:, k]).reshape(m, m)
    rho_R = np.real(vl[:, kl]).reshape(m, m)
    order = np.argsort(-np.abs(w))
    return t1, rho_L, rho_R, w[order]


def correlation_length(spectrum):
    """Correlation length in unit cells from the two largest moduli of the transfer spectrum."""
    a = np.abs(spectrum)
    if a[1] <= 0.0:
        return 0.0
    return -1.0 / np.log(a[1] / a[0])


def expectation(Bs, sites, ops, fp=None):
    """<prod_j ops[j] at sites[j]> in the infinite MPS.

    Bs: the unit cell (pieces 1..l/2); sites: positions counted from the first
    site of piece 1 (0, 1, ... ; any number of cells to the right); ops: 2x2
    matrices.  fp: fixed_points(Bs) if already computed."""
    t1, rho_L, rho_R, _ = fp if fp is not None else fixed_points(Bs)
    half = len(Bs)
    on = {}
    for s, o in zip(sites, ops):
        on[s] = o if s not in on else on[s] @ o
    ncell = max(sites) // (2 * half) + 1
    X = rho_L
    for c in range(ncell):
        for p in range(half):
            k = 2 * (c * half + p)
            X = apply_piece(X, Bs[p], on.get(k), on.get(k + 1))
    return float(np.sum(X * rho_R) / (t1 ** ncell * np.sum(rho_L * rho_R)))


def spin_correlation(Bs, a, b, fp=None):
    """<s_a . s_b> = <Sz Sz> + (<S+ S-> + <S- S+>) / 2 at positions a != b."""
    fp = fp if fp is not None else fixed_points(Bs)
    return (expectation(Bs, [a, b], [SZ, SZ], fp) + 0.5 * expectation(Bs, [a, b], [SP, SM], fp)
            + 0.5 * expectation(Bs, [a, b], [SM, SP], fp))


def position(label, first_site, ell):
    """Position (from the first site of piece 1) of the first site at or after it with this label (1..l)."""
    f0 = (first_site - 1) % ell + 1
    return (label - f0) % ell


def bond_strengths(Bs, n, ell, pairs, fp=None):
    """<s_i . s_j> for label pairs (i, j) with i < j (j may exceed l: a site of a later cell).

    The unit cell follows iteration n: its first site is n + 2."""
    fp = fp if fp is not None else fixed_points(Bs)
    out = {}
    for i, j in pairs:
        a = position(i, n + 2, ell)
        out[(i, j)] = spin_correlation(Bs, a, a + (j - i), fp)
    return out


def bond_spread(values):
    """Eqs. (15), (16) for one bond class: (average, Delta+, Delta-) of its translated bond strengths."""
    v = np.asarray(values, dtype=np.float64)
    av = float(np.mean(v))
    return av, float(np.max(v)) - av, float(np.min(v)) - av
