"""The stored oracle trajectories are the oracle's (CPU only).

tests/golden/traj_*.json hold the FP64 oracle runs that the GPU trajectory
tests compare against.  Here a prefix of each is recomputed with the oracle
and must agree record by record, and the stored runs must satisfy what the
method fixes independently of any implementation: untruncated iterations
equal exact diagonalisation of their open segments (pin P1), and e_g is the
Step 5' difference quotient of the stored superblock energies.
"""
import pytest

import workloads
from oracle import ed, idmrg

from golden.make_trajectories import FIXTURES, load

# iterations recomputed per fixture (a few seconds of oracle time each)
PREFIX = {"yc8_m128": 8, "yc4_m128": 10, "random_chain_m256": 9, "yc8_m128_tight": 8, "yc4_m128_tight": 8,
          "random_chain_m256_tight": 8}


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_stored_trajectory_is_the_oracle(name):
    ref = load(name)
    wl, m, n_max, over = FIXTURES[name]
    assert (ref["workload"], ref["m"], ref["n_max"], ref["overrides"]) == (wl, m, n_max, over)
    cfg = workloads.workload(wl, m=m, **over)
    r = idmrg.run(cfg, mode="u1", n_max=PREFIX[name])
    stored = [s for s in ref["steps"] if s["n"] <= PREFIX[name]]
    assert len(stored) == len(r["steps"])
    for a, b in zip(r["steps"], stored):
        assert (a["n"], a["i"], a["m_kept"]) == (b["n"], b["i"], b["m_kept"])
        assert abs(a["energy"] - b["energy"]) <= 1e-12 * max(1.0, abs(b["energy"]))


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_stored_trajectory_invariants(name):
    ref = load(name)
    wl, m, n_max, over = FIXTURES[name]
    cfg = workloads.workload(wl, m=m, **over)
    ell = cfg["ell"]
    E = {(s["n"], s["i"]): s["energy"] for s in ref["steps"]}
    # the stored runs cover every superblock of every iteration and a full period of truncation
    assert sorted(E) == [(n, i) for n in range(1, n_max + 1) for i in range(1, ell // 2 + 1)]
    assert any(s["eps"] > 0 for s in ref["steps"])
    truncated = sorted({s["n"] for s in ref["steps"] if 2 ** s["n"] > m})
    assert len(truncated) >= ell
    # Step 5': e_g = (e^(n)_1 - e^(n-l)_1) / (2l) at (n + 1) mod l = 0, with e^(-1)_1 = 0
    assert sorted(int(n) for n in ref["e_g"]) == [n for n in range(1, n_max + 1) if (n + 1) % ell == 0]
    for n, e in ref["e_g"].items():
        n = int(n)
        e_old = E[(n - ell, 1)] if n - ell >= 1 else 0.0
        assert abs(e - (E[(n, 1)] - e_old) / (2 * ell)) <= 1e-15
    # P1: the last untruncated iteration, superblock 1, equals exact diagonalisation
    n = max(k for k in range(1, n_max + 1) if 2 ** k <= m and 2 * k + 2 <= 18)
    e0 = ed.ground_energy(workloads.segment_bonds(cfg["bonds"], ell, 1, 2 * n + 2), 1, 2 * n + 2)
    assert abs(E[(n, 1)] - e0) <= 1e-11
