"""The seeded input recipe (CPU): the matvec microbenchmark's sector profile and
the random-bond chain's couplings, as the recipe states them."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("m", [256, 512, 1024, 2048])
def test_sector_profile(m):
    """Charges -10..10 in steps of 2 with dims proportional to exp(-(q/2)^2 / 8), rounded by largest remainder
    to sum exactly m (so each dim is within 1 of its share)."""
    qs, ds = workloads.sector_dims(m)
    assert list(qs) == list(range(-10, 11, 2))
    assert sum(ds) == m
    w = np.exp(-((np.array(qs) / 2.0) ** 2) / 8.0)
    share = m * w / w.sum()
    assert np.all(np.abs(np.array(ds) - share) < 1.0)
    assert np.all(np.array(ds) >= np.floor(share))


def test_sector_profile_m1024():
    """The profile the recipe quotes for m = 1024: about 205, 181, 125, 67, 28, 9 for |q|/2 = 0..5."""
    qs, ds = workloads.sector_dims(1024)
    d = dict(zip(qs, ds))
    for q, want in zip(range(0, 11, 2), (205, 181, 125, 67, 28, 9)):
        assert abs(d[q] - want) <= 1 and abs(d[-q] - want) <= 1


def test_random_chain_couplings():
    """J_k = default_rng([SEED, 3]).uniform(0.5, 1.5, 16)[k - 1] couples sites (k, k + 1); J_16 couples the last
    site of the cell to the first site of the next one."""
    J = np.random.default_rng([workloads.SEED, 3]).uniform(0.5, 1.5, 16)
    bonds = workloads.random_chain_bonds(16)
    assert len(bonds) == 16
    for k, (i, j, c) in enumerate(sorted(bonds)):
        assert (i, j) == (k + 1, k + 2)
        assert c == J[k]
        assert 0.5 <= c <= 1.5


def test_seeded_draws_are_reproducible():
    assert np.array_equal(workloads.gaussian(7, 2, 256, 1, 3), workloads.gaussian(7, 2, 256, 1, 3))
    assert not np.array_equal(workloads.gaussian(7, 2, 256, 1, 3), workloads.gaussian(7, 2, 256, 0, 3))
    assert np.array_equal(workloads.start_vector(5, 1, 2), np.random.default_rng([workloads.SEED, 1, 2]).standard_normal(5))


def test_yc8_axis_sweep():
    """The reconstructed YC8 embedding gives the sweep of sites that Sec. 4 lists for the correlation function
    (i = 2, 14, 35, 47, ...), every site on it has the start's sublattice, and consecutive sites are joined by the
    bonds of the lattice's two-step paths (distances 2 and 2 sqrt(3) alternate with the parity of the ring)."""
    sweep = workloads.yc8_axis_sweep(8, 2)
    assert [s for s, _ in sweep[:4]] == [2, 14, 35, 47]
    assert all((s - 1) % 3 == 1 for s, _ in sweep)           # sublattice of label 2
    assert [s // 12 if s % 12 else s // 12 - 1 for s, _ in sweep] == list(range(9))   # one site per ring
    for R, (_, d) in enumerate(sweep):
        assert abs(d - np.sqrt(3 * R * R + R % 2)) <= 1e-12
    # the even rings lie exactly on the axis: distances R sqrt(3)
    assert abs(sweep[2][1] - 2 * np.sqrt(3)) <= 1e-12 and abs(sweep[8][1] - 8 * np.sqrt(3)) <= 1e-12
    # site 14 is a nearest-neighbour two-step path away from 2: 2 - 3 - 14 are both bonds of the cell
    bonds = {(i, j) for i, j, _ in workloads.yc8_kagome_bonds()}
    assert (2, 3) in bonds and (3, 14) in bonds
