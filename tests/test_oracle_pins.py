"""Pins of the oracle against facts fixed by the paper and by mathematics (CPU only).

Each test names what it pins.  None of them retypes the oracle's own formula:
the references are exact diagonalisation from the bond list, closed forms,
textbook limits, brute-force projections and LAPACK on assembled matrices.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads
from oracle import dense, ed, idmrg, layout, mpo, u1
from oracle.lanczos import lanczos


def _ed(cfg, first, last):
    return ed.ground_energy(workloads.segment_bonds(cfg["bonds"], cfg["ell"], first, last), first, last)


# ----------------------------------------------------------------- P2 closed form

@pytest.mark.parametrize("mode", ["u1", "dense"])
def test_p2_four_site_closed_form(mode):
    """n = 1 superblock of the uniform chain is the open 4-site chain: E0 = -(3 + 2 sqrt 3)/4."""
    cfg = workloads.workload("chain")
    r = idmrg.run(cfg, mode=mode, n_max=1)
    for s in r["steps"]:
        assert abs(s["energy"] + (3 + 2 * math.sqrt(3)) / 4) <= 1e-13


# ----------------------------------------------------------------- P1 exact diagonalisation

@pytest.mark.parametrize("name,m,n_max,mode", [
    ("chain", 32, 5, "u1"), ("chain", 32, 4, "dense"), ("random_chain", 64, 5, "u1"),
    ("yc4", 64, 4, "u1"), ("yc8", 64, 5, "u1")])
def test_p1_untruncated_equals_ed(name, m, n_max, mode):
    """While d^n <= m nothing is discarded, so every superblock energy is the
    exact ground energy of its open segment 2i-1 .. 2i+2n (all i: checks the
    wrap R_{l+2} = R_2 and the site-dependent W_{f(k)})."""
    cfg = workloads.workload(name, m=m)
    r = idmrg.run(cfg, mode=mode, n_max=n_max)
    for s in r["steps"]:
        if 2 ** s["n"] <= m:
            f, l = s["sites"]
            assert abs(s["energy"] - _ed(cfg, f, l)) <= 1e-11, s


def test_p1_known_cylinder_values():
    """ED of the cylinder inputs themselves (sites 1..2n+2) at two sizes each."""
    yc4 = workloads.workload("yc4")
    assert abs(_ed(yc4, 1, 8) - (-4.820089374375)) < 1e-9
    assert abs(_ed(yc4, 1, 12) - (-7.530137169010)) < 1e-9
    yc8 = workloads.workload("yc8")
    assert abs(_ed(yc8, 1, 8) - (-3.166254087325)) < 1e-9
    assert abs(_ed(yc8, 1, 12) - (-4.880002723390)) < 1e-9
    chain = workloads.workload("chain")
    assert abs(_ed(chain, 1, 14) - (-6.026724661862173)) < 1e-11


# ----------------------------------------------------------------- P3 dimerised limit

@pytest.mark.parametrize("mode", ["u1", "dense"])
def test_p3_dimerised_prediction_is_exact(mode):
    """J_odd = 1, J_even = 0: every superblock is n+1 isolated singlets, e = -3(n+1)/4,
    e_g = -3/8.  Eq. (10) then predicts the exact ground state (its lambda = 0 branch
    for odd n and 1/lambda = sqrt 2 for even n), so the fidelity error vanishes and
    Lanczos stops after one step."""
    cfg = workloads.workload("dimer", m=8, n_max=8)
    r = idmrg.run(cfg, mode=mode)
    for s in r["steps"]:
        assert abs(s["energy"] + 0.75 * (s["n"] + 1)) <= 1e-12
        if s["n"] >= 3:
            assert s["fidelity"] <= 1e-12
            assert s["iters"] == 1
    for n, e in r["e_g"].items():
        assert abs(e + 0.375) <= 1e-12


# ----------------------------------------------------------------- P4 Bethe ansatz

def test_p4_bethe_ansatz():
    """Uniform chain, m = 32: the subtracted energy e_g (Step 5') approaches
    1/4 - ln 2 from above; at n = 19 (40 sites) within 5e-4."""
    cfg = workloads.workload("chain")
    r = idmrg.run(cfg, mode="u1", n_max=19)
    eb = workloads.bethe_ansatz_energy()
    eg = r["e_g"]
    assert sorted(eg) == [3, 7, 11, 15, 19]
    assert abs(eg[3] - _ed(cfg, 1, 8) / 8) <= 1e-12        # e^(-1)_1 = 0: first estimate = E0(8)/8
    for n in eg:
        assert eg[n] >= eb - 1e-4
    assert abs(eg[19] - eb) <= 5e-4
    assert abs(eg[19] - eb) < abs(eg[7] - eb)


# ----------------------------------------------------------------- P5 brute-force projection

def _block_bases(states, half):
    """Explicit basis vectors of every left and right block, built from the kept
    U and V of each (n, i) (dense mode), as columns over the block's sites."""
    I2 = np.eye(2)
    BL = {(0, i): I2 for i in range(1, half + 1)}
    BR = {(0, i): I2 for i in range(1, half + 1)}
    for st in states:
        n, i = st["n"], st["i"]
        U, V = st["tr"]["U"], st["tr"]["V"]          # U[a,s,g], V[s,b,g]
        prevL = BL[(n - 1, i)]                        # [sites, a]
        BL[(n, i)] = np.einsum("xa,asg->xsg", prevL, U).reshape(-1, U.shape[2])
        prevR = BR[(n - 1, i % half + 1)]             # [sites, b]
        BR[(n, i)] = np.einsum("sbg,yb->syg", V, prevR).reshape(-1, V.shape[2])
    return BL, BR


def test_p5_heff_is_projected_segment_hamiltonian():
    """H_eff of superblock (n, i), built column by column from the matvec, equals
    P^T H_segment P where P maps (alpha, s1, s2, beta) to explicit configurations
    through the kept block bases.  Checked in the truncated regime (m = 4), which
    pins the environment updates (Eqs. (4), (5)) and the matvec (Step 3).  The
    matrix is symmetric and its lowest eigenvalue is the Lanczos energy."""
    cfg = workloads.workload("random_chain", m=4, tol_res=1e-10)
    half = cfg["ell"] // 2
    r = idmrg.run(cfg, mode="dense", n_max=4, keep_states=True)
    BL, BR = _block_bases(r["states"], half)
    checked = 0
    for st in r["states"]:
        n, i = st["n"], st["i"]
        if n < 2 or i > 3:
            continue
        L, R, W1, W2 = st["L"], st["R"], st["W1"], st["W2"]
        ma, mb = L.shape[0], R.shape[0]
        N = ma * 4 * mb
        H = np.zeros((N, N))
        for k in range(N):
            e = np.zeros(N)
            e[k] = 1.0
            H[:, k] = dense.heff_apply(L, W1, W2, R, e.reshape(ma, 2, 2, mb)).reshape(-1)
        assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
        first, last, _, _ = idmrg.superblock_sites(n, i)
        P = np.einsum("xa,st,uv,yb->xsuyatvb", BL[(n - 1, i)], np.eye(2), np.eye(2),
                      BR[(n - 1, i % half + 1)]).reshape(2 ** (last - first + 1), N)
        Hseg = mpo.bond_sum_matrix(workloads.segment_bonds(cfg["bonds"], cfg["ell"], first, last),
                                   first, last)
        Hp = P.T @ Hseg @ P
        assert np.abs(H - Hp).max() <= 1e-12 * np.abs(Hp).max()
        assert abs(np.linalg.eigvalsh(H)[0] - [s for s in r["steps"] if (s["n"], s["i"]) == (n, i)][0]["energy"]) <= 1e-11
        checked += 1
    assert checked >= 6


# ----------------------------------------------------------------- P6 invariants

def test_p6_invariants_u1():
    """Sum lam^2 = 1 (Step 4), eps = (2 - eps') eps' (Eq. (14)), fidelity >= eps'
    (Eqs. (12), (13)), U^T U = V^T V = I, |Psi - U Lam V^T|^2 = eps, identity
    channel of the new environments = I, variational bound above ED."""
    cfg = workloads.workload("random_chain", m=12)
    r = idmrg.run(cfg, mode="u1", n_max=7, keep_states=True)
    qp = mpo.QP
    for st, s in zip(r["states"], r["steps"]):
        tr = st["tr"]
        assert abs(float(np.sum(tr["spectrum"] ** 2)) - 1.0) <= 1e-13
        assert abs(tr["eps"] - (2 - tr["eps_prime"]) * tr["eps_prime"]) <= 1e-15
        if s["n"] >= 3:
            assert s["fidelity"] >= tr["eps_prime"] - 1e-14
        C = tr["C"]
        for qc, kc in C:
            Ublk = np.concatenate([tr["U"][(qa, s_, qc)] for (qa, s_, _) in layout.U_rows(st["A"], qp, qc)])
            Vblk = np.concatenate([tr["V"][(s_, qb, qc)] for (s_, qb, _) in layout.V_rows(st["B"], qp, qc)])
            assert np.abs(Ublk.T @ Ublk - np.eye(kc)).max() <= 1e-13
            assert np.abs(Vblk.T @ Vblk - np.eye(kc)).max() <= 1e-13
        psi = layout.flat_to_psi(st["psi"], st["A"], st["B"], qp)
        approx = {}
        for (qa, s1, s2), blk in psi.items():
            qc = qa + qp[s1]
            qb = qc + qp[s2]
            if (qa, s1, qc) in tr["U"] and (s2, qb, qc) in tr["V"]:
                approx[(qa, s1, s2)] = tr["U"][(qa, s1, qc)] @ np.diag(tr["lam"][qc]) @ tr["V"][(s2, qb, qc)].T
        err = sum(float(np.sum((blk - approx.get(k, 0.0)) ** 2)) for k, blk in psi.items())
        assert abs(err - tr["eps"]) <= 1e-13
        Lp = u1.update_env_left(st["L"], st["W1"], tr["U"], st["A"], qp, C, st["dl"], st["dm"])
        Rp = u1.update_env_right(st["R"], st["W2"], tr["V"], st["B"], qp, C, st["dm"], st["dr"])
        Dm = st["W1"].shape[1]
        for qc, kc in C:
            assert np.abs(Lp[(Dm - 1, qc, qc)] - np.eye(kc)).max() <= 1e-13
            assert np.abs(Rp[(0, qc, qc)] - np.eye(kc)).max() <= 1e-13
            assert np.abs(Lp[(0, qc, qc)] - Lp[(0, qc, qc)].T).max() <= 1e-12
        if s["sites"][1] - s["sites"][0] + 1 <= 16:
            assert s["energy"] >= _ed(cfg, *s["sites"]) - 1e-10


# ----------------------------------------------------------------- P7 translation invariance

def test_p7_unit_cell_independence():
    """A uniform chain gives the same superblock energies whatever the unit cell
    l in {2, 4, 8} (l = 2 is plain two-site iDMRG, R_{l+2} = R_2 being its own
    right block), and every superblock of one iteration has the same energy."""
    res = {}
    for ell in (2, 4, 8):
        cfg = workloads.workload("chain", ell=ell, bonds=workloads.chain_bonds(ell), m=16)
        r = idmrg.run(cfg, mode="u1", n_max=10)
        by_n = {}
        for s in r["steps"]:
            by_n.setdefault(s["n"], []).append(s["energy"])
        for n, es in by_n.items():
            assert max(es) - min(es) <= 1e-10
        res[ell] = {n: es[0] for n, es in by_n.items()}
    for n in range(1, 11):
        assert abs(res[2][n] - res[4][n]) <= 1e-10
        assert abs(res[2][n] - res[8][n]) <= 1e-10


# ----------------------------------------------------------------- P8 dense = U(1)

def test_p8_dense_equals_u1():
    """With and without S^z blocks the trajectory is the same (the ground state's
    reduced density matrix commutes with S^z of the block)."""
    cfg = workloads.workload("random_chain", m=16, ell=4, bonds=workloads.random_chain_bonds(4),
                             tol_res=1e-10)
    a = idmrg.run(cfg, mode="u1", n_max=7)
    b = idmrg.run(cfg, mode="dense", n_max=7)
    for x, y in zip(a["steps"], b["steps"]):
        assert abs(x["energy"] - y["energy"]) <= 1e-10
        assert x["m_kept"] == y["m_kept"]
        assert abs(x["eps"] - y["eps"]) <= 1e-12


# ----------------------------------------------------------------- P9 library routines

def test_p9_block_svd_matches_dense_svd():
    """Singular values gathered from the per-charge blocks equal LAPACK's SVD of
    the assembled dense matrix psi[(alpha s1), (s2 beta)]."""
    A = [(-3, 2), (-1, 5), (1, 4), (3, 1)]
    B = [(-3, 1), (-1, 3), (1, 6), (3, 2)]
    qp = mpo.QP
    x = workloads.gaussian(layout.psi_size(A, B, qp), 9, 1)
    x /= np.linalg.norm(x)
    psi = layout.flat_to_psi(x, A, B, qp)
    tr = u1.truncate_twosite(psi, A, B, qp, m=1000)
    # assemble the full dense tensor with explicit index offsets
    offA = np.cumsum([0] + [d for _, d in A])
    offB = np.cumsum([0] + [d for _, d in B])
    ia = {q: k for k, (q, _) in enumerate(A)}
    ib = {q: k for k, (q, _) in enumerate(B)}
    full = np.zeros((offA[-1], 2, 2, offB[-1]))
    for (qa, s1, s2), blk in psi.items():
        qb = qa + qp[s1] + qp[s2]
        full[offA[ia[qa]]:offA[ia[qa] + 1], s1, s2, offB[ib[qb]]:offB[ib[qb] + 1]] = blk
    S = np.linalg.svd(full.reshape(offA[-1] * 2, 2 * offB[-1]), compute_uv=False)
    k = len(tr["spectrum"])
    assert np.abs(np.sort(S)[::-1][:k] - tr["spectrum"]).max() <= 1e-14
    assert np.all(np.sort(S)[::-1][k:] <= 1e-14)


def test_p9_lanczos_matches_eigh():
    """Lowest eigenpair of an explicit symmetric matrix: Lanczos vs LAPACK syevd."""
    n = 300
    M = workloads.gaussian(n * n, 9, 2).reshape(n, n)
    M = M + M.T
    w, v = np.linalg.eigh(M)
    sol = lanczos(lambda x: M @ x, workloads.gaussian(n, 9, 3), tol_E=1e-13, tol_res=1e-10, k_max=300)
    assert abs(sol["energy"] - w[0]) <= 1e-12 * abs(w[0])
    assert abs(abs(sol["psi"] @ v[:, 0]) - 1.0) <= 1e-12


def test_degeneracy_guard():
    """The cut is moved up past (near-)degenerate singular values."""
    cands = [(0.8, 0, 0), (0.4, 0, 1), (0.3, 0, 2), (0.3 * (1 - 1e-7), 1, 0), (0.1, 1, 1)]
    kept, gap = u1.select_kept(cands, 3, 1e-14, 1e-5)
    assert [c[0] for c in kept] == [0.8, 0.4]
    kept, gap = u1.select_kept(cands, 4, 1e-14, 1e-5)
    assert len(kept) == 4 and gap == pytest.approx((0.3 * (1 - 1e-7) - 0.1) / (0.3 * (1 - 1e-7)))
    # zero-weight states in ascending charge order, only when every candidate is kept
    cands = [(1.0, 1, 0), (0.0, 1, 1), (0.0, -1, 0), (0.0, -1, 1)]
    kept, gap = u1.select_kept(cands, 4, 1e-14, 1e-5)
    assert kept == [(1.0, 1, 0), (0.0, -1, 0), (0.0, -1, 1), (0.0, 1, 1)] and gap is None
    kept, gap = u1.select_kept(cands, 3, 1e-14, 1e-5)
    assert kept == [(1.0, 1, 0)] and gap is None


@pytest.mark.parametrize("name", ["chain", "random_chain"])
def test_prediction_is_near_optimal(name):
    """Eq. (10) with the paper's 1/lambda^(n-2) factor gives a start vector whose
    fidelity error (Eq. (12)) is tiny once the blocks are large (Sec. 4,
    prediction subsection); a random start has O(1) fidelity error and needs
    more Lanczos steps.  Dropping the 1/lambda factor or taking lambda from the
    wrong iteration raises the error to ~1e-2, which this test rejects."""
    cfg = workloads.workload(name, m=32)
    r = idmrg.run(cfg, mode="u1", n_max=10)
    rr = idmrg.run(cfg, mode="u1", n_max=10, predict=False)
    fp = [s["fidelity"] for s in r["steps"] if s["n"] >= 6]
    fr = [s["fidelity"] for s in rr["steps"] if s["n"] >= 6]
    assert np.median(fp) <= 1e-5 and max(fp) <= 1e-3
    assert min(fr) >= 1e-2
    it_p = sum(s["iters"] for s in r["steps"] if s["n"] >= 6)
    it_r = sum(s["iters"] for s in rr["steps"] if s["n"] >= 6)
    assert it_p < 0.7 * it_r


def test_zero_weight_states_only_with_every_candidate():
    """Kept-set rule (R5 with the reading that the kept space must not depend on which null
    vectors a decomposition returns): zero-weight states are kept only when every candidate
    is; otherwise only nonzero values are kept, even if fewer than m."""
    cands = [(0.8, 0, 0), (0.5, 2, 0), (0.33, -2, 0)] + [(0.0, q, 1) for q in (-2, 0, 2)] + [(1e-16, 0, 2)]
    kept, gap = u1.select_kept(cands, 5, 1e-14, 1e-5)
    assert [c[0] for c in kept] == [0.8, 0.5, 0.33] and gap is None
    kept, gap = u1.select_kept(cands, 7, 1e-14, 1e-5)
    assert len(kept) == 7 and gap is None
    assert [(c[1], c[2]) for c in kept[3:]] == [(-2, 1), (0, 1), (0, 2), (2, 1)]
    kept, gap = u1.select_kept(cands, 2, 1e-14, 1e-5)
    assert [c[0] for c in kept] == [0.8, 0.5] and abs(gap - 0.34) < 1e-12
