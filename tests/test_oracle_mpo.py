"""Pins of the oracle's MPO builder (CPU only).

The MPO of Eq. (1)/(7), contracted over a finite open segment with the left
boundary = last row and right boundary = first column, must equal the
Hamiltonian summed directly from the bond list.
"""
import numpy as np
import pytest

import workloads
from oracle import mpo


@pytest.mark.parametrize("name,first,last", [
    ("chain", 1, 8), ("chain", 3, 10), ("random_chain", 5, 14), ("yc4", 1, 10), ("yc4", 4, 12),
    ("yc8", 1, 10), ("yc8", 8, 17), ("dimer", 1, 8)])
def test_mpo_contracts_to_bond_sum(name, first, last):
    cfg = workloads.workload(name)
    Ws, _ = mpo.build_mpo(cfg["ell"], cfg["bonds"])
    Hm = mpo.mpo_segment_matrix(Ws, cfg["ell"], first, last)
    bonds = workloads.segment_bonds(cfg["bonds"], cfg["ell"], first, last)
    Hb = mpo.bond_sum_matrix(bonds, first, last)
    assert np.abs(Hm - Hb).max() <= 1e-13
    assert np.abs(Hb).max() > 0.1


@pytest.mark.parametrize("name", ["chain", "random_chain", "yc4", "yc8", "dimer"])
def test_mpo_structure(name):
    """Lower triangular, identity corners, charge conservation, periodic cut charges."""
    cfg = workloads.workload(name)
    Ws, dq = mpo.build_mpo(cfg["ell"], cfg["bonds"])
    assert np.array_equal(dq[0], dq[cfg["ell"]])
    for c, W in enumerate(Ws, start=1):
        din, dout = W.shape[:2]
        assert din == len(dq[c - 1]) and dout == len(dq[c])
        assert np.array_equal(W[0, 0], np.eye(2)) and np.array_equal(W[din - 1, dout - 1], np.eye(2))
        for w in range(din):
            for v in range(dout):
                for s in range(2):
                    for t in range(2):
                        if W[w, v, s, t] != 0:
                            assert mpo.QP[s] - mpo.QP[t] == dq[c][v] - dq[c - 1][w]
        # lower triangular in the channel order complete < pending < identity
        for w in range(din):
            for v in range(dout):
                if np.any(W[w, v]) and not (w == din - 1 or v == 0):
                    # pending -> pending only (carry)
                    assert 0 < w < din - 1 and 0 < v < dout - 1


def test_channel_counts():
    """Channel counts at the cuts: chain 5, YC4 14 everywhere, YC8 between 14 and 20."""
    D = {}
    for name in ["chain", "yc4", "yc8"]:
        cfg = workloads.workload(name)
        Ws, _ = mpo.build_mpo(cfg["ell"], cfg["bonds"])
        D[name] = [W.shape[1] for W in Ws]
    assert set(D["chain"]) == {5}
    assert set(D["yc4"]) == {14}
    assert min(D["yc8"]) == 14 and max(D["yc8"]) == 20


def test_lattice_inputs():
    """Coordination numbers of the lattice inputs (4 for the square and kagome cylinders)."""
    for name, ell, z in [("yc4", 8, 4), ("yc8", 12, 4)]:
        cfg = workloads.workload(name)
        bonds = workloads.segment_bonds(cfg["bonds"], ell, 1, 5 * ell)
        deg = {}
        for (i, j, _) in bonds:
            deg[i] = deg.get(i, 0) + 1
            deg[j] = deg.get(j, 0) + 1
        interior = [deg[s] for s in range(2 * ell + 1, 3 * ell + 1)]
        assert set(interior) == {z}
        assert len(cfg["bonds"]) == 2 * ell
