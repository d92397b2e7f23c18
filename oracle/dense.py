"""Hot-path steps on full tensors, no symmetry blocks (oracle).

Test infrastructure only (see ``oracle/__init__``).

This is the paper's own setting (Sec. 4: no block diagonalisation with
respect to quantum numbers).  Index conventions follow the paper:
L[alpha, w, alpha'], R[beta, w, beta'], W[w, w', s, s'], psi[alpha, s1, s2, beta],
U[alpha, s, gamma], V[s, beta, gamma] (psi = U Lambda V^dagger, Step 4).
"""
from __future__ import annotations

import numpy as np

from .u1 import select_kept, svd


def init_left(W):
    """L^(0) = last row of W (Step 1): L[s, w, s'] = W[D-1, w, s, s']."""
    return np.ascontiguousarray(np.transpose(W[W.shape[0] - 1], (1, 0, 2)))


def init_right(W):
    """R^(0) = first column of W (Step 1): R[s, w, s'] = W[w, 0, s, s']."""
    return np.ascontiguousarray(np.transpose(W[:, 0], (1, 0, 2)))


def heff_apply(L, W1, W2, R, psi):
    """H^(n)_i psi by the contraction of Fig. 2(b) (Step 3), one tensor at a time:
    y[a,s,t,b] = sum L[a,w,A] W1[w,v,s,S] W2[v,u,t,T] R[b,u,B] psi[A,S,T,B]."""
    T1 = np.einsum("awA,ASTB->awSTB", L, psi)
    T2 = np.einsum("wvsS,awSTB->avsTB", W1, T1)
    T3 = np.einsum("vutT,avsTB->austB", W2, T2)
    return np.einsum("austB,buB->astb", T3, R)


def truncate_twosite(psi, m, lam_floor=1e-14, deg_rel=1e-5):
    """SVD of psi[(alpha s1), (s2 beta)] and selection of the kept states (Steps 4, 6)."""
    ma, d, _, mb = psi.shape
    M = psi.reshape(ma * d, d * mb)
    Um, S, Vt = svd(M)
    norm = np.sqrt(float(np.sum(S ** 2)))
    cands = [(float(S[j]) / norm, 0, j) for j in range(len(S))]
    kept, gap = select_kept(cands, m, lam_floor, deg_rel)
    js = [j for (_, _, j) in kept]
    lam = np.array([l if l > lam_floor else 0.0 for (l, _, _) in kept])
    U = Um[:, js].reshape(ma, d, len(js))
    V = Vt[js, :].T.reshape(d, mb, len(js))
    kept_set = set(js)
    eps = sum(l * l for (l, _, j) in cands if j not in kept_set)
    eps_prime = eps / (1.0 + np.sqrt(max(0.0, 1.0 - eps)))
    return dict(U=U, V=V, lam=lam, eps=eps, eps_prime=eps_prime, m_kept=len(js), cut_gap=gap,
                spectrum=np.sort(S / norm)[::-1])


def update_env_left(L, W1, U):
    """Eq. (4): L'[b, w', b'] = sum u*[a,s,b] L[a,w,a'] W1[w,w',s,s'] u[a',s',b']."""
    T = np.einsum("awA,ASB->awSB", L, U)
    T = np.einsum("wvsS,awSB->avsB", W1, T)
    return np.einsum("asb,avsB->bvB", U, T)


def update_env_right(R, W2, V):
    """Eq. (5) (index placement read as v on the left, v* on the right):
    R'[b, w, b'] = sum v[s,a,b] W2[w,w'',s,s'] R[a,w'',a'] v[s',a',b']."""
    T = np.einsum("auA,SAB->auSB", R, V)
    T = np.einsum("wusS,auSB->awsB", W2, T)
    return np.einsum("sab,awsB->bwB", V, T)


def predict_wavefunction(lam_i, V_i, lam_ip1_prev, U_ip1, lam_ip1, lam_floor=1e-14):
    """Eq. (10): psi~[a,s,s',a'] = sum_b lam_i[a] v_i[s,b,a] u~_{i+1}[b,s',a']."""
    inv = np.where(lam_ip1_prev > lam_floor, 1.0 / np.where(lam_ip1_prev > lam_floor, lam_ip1_prev, 1.0), 0.0)
    left = lam_i[None, None, :] * V_i                      # [s, b, a]
    right = inv[:, None, None] * U_ip1 * lam_ip1[None, None, :]   # [b, t, c]
    return np.einsum("sba,btc->astc", left, right)


# ---- canonical single-sector flat order (all charges zero): blocks (s1, s2), each [ma x mb]

def psi_from_flat(x, ma, d, mb):
    return np.ascontiguousarray(np.asarray(x).reshape(d, d, ma, mb).transpose(2, 0, 1, 3))


def psi_to_flat(psi):
    return np.ascontiguousarray(psi.transpose(1, 2, 0, 3)).reshape(-1)
