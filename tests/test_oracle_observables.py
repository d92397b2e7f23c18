"""Pins of the oracle's observables of the uniform MPS (Eq. (11); Sec. 4, bond strengths Eqs. (15), (16), correlation
length), each against something other than the oracle's transfer-matrix formula:

* brute force: the state vector of a periodic ring of N unit cells built from the same pieces, whose correlations
  approach the infinite-chain values as (|t2| / |t1|)^N;
* the dimer limit, where the ground state is a product of singlets (exact -3/4 and 0, and no correlation length);
* the Heisenberg chain: the bond energies of one cell add up to the Step 5' energy per site of the same run, and lie
  above the Bethe-ansatz energy (the MPS is a normalised state);
* the bond-spread definitions of Eqs. (15), (16) on a translation-invariant set and on a known one.
"""
import numpy as np
import pytest

import workloads
from oracle import idmrg
from oracle import observables as ob


def _ring_state(Bs, ncell):
    """Amplitudes of the periodic MPS Tr(B_1 B_2 ... ) over ncell repetitions of the cell, sites in order."""
    m = Bs[0].shape[0]
    T = np.eye(m).reshape(1, m, m)          # [configuration so far, first bond, current bond]
    for _ in range(ncell):
        for B in Bs:
            T = np.einsum("xoa,astb->xstob", T, B).reshape(-1, m, B.shape[3])
    return np.einsum("xaa->x", T)


def _apply(psi, nsite, p, op):
    v = psi.reshape(2 ** p, 2, 2 ** (nsite - p - 1))
    return np.einsum("ij,ajb->aib", op, v).reshape(-1)


def _ring_spin_correlation(psi, nsite, p, q):
    out = 0.0
    for o1, o2, c in ((ob.SZ, ob.SZ, 1.0), (ob.SP, ob.SM, 0.5), (ob.SM, ob.SP, 0.5)):
        out += c * (psi @ _apply(_apply(psi, nsite, q, o2), nsite, p, o1))
    return out / (psi @ psi)


def _gapped_cell(rng, half, m, delta):
    """Pieces close to a product state (a rank-one bond structure plus delta noise): a small |t2| / |t1|."""
    out = []
    for _ in range(half):
        u, v, w = rng.standard_normal(m), rng.standard_normal((2, 2)), rng.standard_normal(m)
        out.append(np.einsum("a,st,b->astb", u, v, w) + delta * rng.standard_normal((m, 2, 2, m)))
    return out


@pytest.mark.parametrize("half, ncell, delta, seed", [(1, 10, 0.05, 11), (2, 5, 0.2, 17)])
def test_ring_brute_force(half, ncell, delta, seed):
    Bs = _gapped_cell(np.random.default_rng(seed), half, 3, delta)
    fp = ob.fixed_points(Bs)
    ratio = abs(fp[3][1]) / abs(fp[3][0])
    assert ratio < 0.1
    nsite = 2 * half * ncell
    psi = _ring_state(Bs, ncell)
    for p, q in ((0, 1), (1, 2), (0, 3), (2, 5), (1, 6)):
        inf = ob.spin_correlation(Bs, p, q, fp)
        ring = _ring_spin_correlation(psi, nsite, p, q)
        assert abs(inf - ring) <= 50 * ratio ** (ncell - 2) + 1e-12, (p, q, inf, ring)


def _final_cell(res, n, half):
    st = {(s["n"], s["i"]): s for s in res["states"]}
    cur = {i: st[(n, i)]["tr"] for i in range(1, half + 1)}
    prev = {i: st[(n - 1, i)]["tr"]["lam"] for i in range(1, half + 1)}
    return cur, prev


def test_dimer_limit():
    cfg = workloads.workload("dimer")
    n = 8
    res = idmrg.run(cfg, mode="dense", n_max=n, keep_states=True)
    cur, prev = _final_cell(res, n, 2)
    Bs = ob.pieces(cur, prev, cfg["lam_floor"])
    fp = ob.fixed_points(Bs)
    bs = ob.bond_strengths(Bs, n, 4, [(1, 2), (2, 3), (3, 4), (4, 5)], fp)
    assert abs(bs[(1, 2)] + 0.75) < 1e-12 and abs(bs[(3, 4)] + 0.75) < 1e-12
    assert abs(bs[(2, 3)]) < 1e-12 and abs(bs[(4, 5)]) < 1e-12
    assert ob.correlation_length(fp[3]) == 0.0 or ob.correlation_length(fp[3]) < 1e-3


def test_chain_bond_energies_match_step5():
    cfg = workloads.workload("chain", m=16)
    n = 39
    res = idmrg.run(cfg, mode="dense", n_max=n, keep_states=True)
    cur, prev = _final_cell(res, n, 2)
    Bs = ob.pieces(cur, prev, cfg["lam_floor"])
    bs = ob.bond_strengths(Bs, n, 4, [(1, 2), (2, 3), (3, 4), (4, 5)])
    e_mps = sum(bs.values()) / 4
    assert abs(e_mps - res["e_g"][n]) < 5e-5
    assert workloads.bethe_ansatz_energy() <= e_mps < workloads.bethe_ansatz_energy() + 1e-3
    # the pieces' site labels follow the iteration: the same bonds one iteration earlier, read with n - 1
    cur2, prev2 = _final_cell(res, n - 1, 2)
    bs2 = ob.bond_strengths(ob.pieces(cur2, prev2, cfg["lam_floor"]), n - 1, 4, [(1, 2), (2, 3), (3, 4), (4, 5)])
    for k in bs:
        assert abs(bs[k] - bs2[k]) < 1e-3


def test_bond_spread():
    av, dp, dm = ob.bond_spread([-0.2, -0.2, -0.2, -0.2])
    assert av == -0.2 and dp == 0.0 and dm == 0.0
    av, dp, dm = ob.bond_spread([-0.1, -0.3, -0.2, -0.2])
    assert abs(av + 0.2) < 1e-15 and abs(dp - 0.1) < 1e-15 and abs(dm + 0.1) < 1e-15
