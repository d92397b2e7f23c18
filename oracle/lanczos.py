"""Lanczos ground-state solver with full re-orthogonalisation (oracle).

Test infrastructure only (see ``oracle/__init__``).

Step 3 of the paper solves H Psi = e Psi for each superblock by an iterative
method, Lanczos in its benchmarks (Sec. 4, prediction subsection, where the
eigenvalue error falls below 1e-13 after about 40 iterations with the
prediction).  The paper does not state a stopping rule or a
re-orthogonalisation scheme; this oracle uses

* full classical Gram-Schmidt applied twice (CGS2) against every stored
  Lanczos vector, in FP64;
* stop at the first k with |theta_k - theta_{k-1}| <= tol_E and residual
  estimate beta_k |y_k| <= tol_res, or an invariant subspace
  beta_k <= 1e-14 |theta_k|, or k = min(k_max, N).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl


def lowest_ritz(alpha, beta):
    """Lowest eigenpair of the symmetric tridiagonal matrix (alpha, beta) (LAPACK)."""
    if len(alpha) == 1:
        return float(alpha[0]), np.ones(1)
    w, v = sl.eigh_tridiagonal(np.asarray(alpha), np.asarray(beta), select="i",
                               select_range=(0, 0))
    return float(w[0]), v[:, 0]


def lanczos(matvec, v0, tol_E=1e-12, tol_res=1e-8, k_max=300):
    """Return dict(energy, psi, iters, residual, y, converged).

    ``psi`` has unit norm; ``y`` are its coordinates in the Lanczos basis,
    whose first vector is v0/|v0| (so |y[0]| is the overlap used by the
    fidelity error of Eq. (12)).
    """
    v0 = np.asarray(v0, dtype=np.float64)
    N = v0.size
    kcap = min(k_max, N)
    Q = np.zeros((kcap, N))
    Q[0] = v0 / np.linalg.norm(v0)
    alpha, beta = [], []
    theta_prev = None
    converged = False
    for k in range(1, kcap + 1):
        q = Q[k - 1]
        w = matvec(q)
        a = float(q @ w)
        w = w - a * q
        if k > 1:
            w = w - beta[-1] * Q[k - 2]
        for _ in range(2):                       # CGS2 against all stored vectors
            c = Q[:k] @ w
            w = w - Q[:k].T @ c
        b = float(np.linalg.norm(w))
        alpha.append(a)
        theta, y = lowest_ritz(alpha, beta)
        res = b * abs(y[-1])
        stop_dtheta = theta_prev is not None and abs(theta - theta_prev) <= tol_E and res <= tol_res
        stop_invariant = b <= 1e-14 * abs(theta)
        theta_prev = theta
        if stop_dtheta or stop_invariant:
            converged = True
            break
        if k == kcap:
            break
        beta.append(b)
        Q[k] = w / b
    psi = Q[:k].T @ y
    psi = psi / np.linalg.norm(psi)
    return dict(energy=theta, psi=psi, iters=k, residual=res, y=y, converged=converged)
