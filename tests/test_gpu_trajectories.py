"""GPU trajectories of the full parallel iDMRG against the FP64 oracle (needs an MI355X).

The driver runs every iteration through the C-ABI (prediction, batched
Lanczos, truncation, both environment updates, hand-off) on reduced-m
versions of the YC8 kagome cylinder (l = 12, six superblocks, MPO channel
counts 14/17/20 by cut), the YC4 square cylinder (l = 8) and the random-bond
chain (l = 16, eight superblocks, its configured m = 256).  Each run covers
the untruncated iterations and more than one unit-cell period of truncated
ones, so every (W_f(c1), W_f(c2)) alignment and the wrap R_{l+2} = R_2 of
Step 2' occur.  The oracle trajectories are stored in tests/golden/ by
tests/golden/make_trajectories.py (oracle only; a CPU test re-derives a
prefix of each).

Per-site energies e^(n)_i / (2n + 2) and every Step 5' estimate e_g must
match within 1e-10 in FP64 and within 1e-9 with a low-precision matvec after
FP64 refinement; kept counts must be equal.  While nothing is discarded the
superblock energies must also equal exact diagonalisation of the open
segment 2i-1 .. 2i+2n, computed here from the bond list.
"""
import pytest

import workloads
from oracle import ed

from golden.make_trajectories import FIXTURES, load

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")

TOL = {"f64": 1e-10, "f32": 1e-9, "bf16x3": 1e-9}
# (fixture, matvec policy): FP64 at the production tolerance, and the low-precision policy of
# each workload's benchmark configuration (the random chain's configuration is FP64; split-bf16
# is run on it as well) against the runs converged to a residual of 1e-10 (see make_trajectories)
CASES = [("yc8_m128", "f64"), ("yc8_m128_tight", "bf16x3"), ("yc4_m128", "f64"), ("yc4_m128_tight", "f32"),
         ("random_chain_m256", "f64"), ("random_chain_m256_tight", "bf16x3")]
# untruncated iterations checked against exact diagonalisation (segments of at most 16 sites)
ED_ITERS = {"yc8_m128": (3, 5, 7), "yc4_m128": (3, 5, 7), "random_chain_m256": (3, 5, 7)}


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,prec", CASES)
def test_trajectory_against_oracle(gpu, name, prec):
    from paper_1606_06790_amd.driver import IDMRG
    ref = load(name)
    wl, m, n_max, over = FIXTURES[name]
    cfg = workloads.workload(wl, m=m, **over)
    print(f"[trajectory] {name} prec={prec} n_max={n_max}", flush=True)
    d = IDMRG(cfg, prec=prec)
    d.run(n_max)
    tol = TOL[prec]
    assert [(s["n"], s["i"]) for s in d.steps] == [(s["n"], s["i"]) for s in ref["steps"]]
    for g, o in zip(d.steps, ref["steps"]):
        assert g["converged"] and g["svd_converged"], g
        assert g["m_kept"] == o["m_kept"], (g, o)
    diff = sorted(((abs(g["e_site"] - o["e_site"]), g["n"], g["i"], g["residual"]) for g, o in zip(d.steps, ref["steps"])),
                  reverse=True)
    dg = max(abs(d.e_g[int(n)] - e) for n, e in ref["e_g"].items())
    print(f"[trajectory] {name} prec={prec}: max |e_site - oracle| = {diff[0][0]:.2e}, |e_g - oracle| = {dg:.2e}; "
          f"largest (diff, n, i, residual): {[(f'{a:.1e}', n, i, f'{r:.1e}') for a, n, i, r in diff[:5]]}", flush=True)
    assert diff[0][0] <= tol
    assert sorted(int(n) for n in ref["e_g"]) == sorted(d.e_g)
    assert dg <= tol


@pytest.mark.parametrize("name", sorted(ED_ITERS))
def test_untruncated_iterations_equal_ed(gpu, name):
    """The GPU path's superblock energies of untruncated iterations are exact ground energies."""
    from paper_1606_06790_amd.driver import IDMRG
    wl, m, _, _ = FIXTURES[name]
    cfg = workloads.workload(wl, m=m)
    d = IDMRG(cfg, prec="f64")
    nmax = max(ED_ITERS[name])
    assert 2 ** nmax <= m
    d.run(nmax)
    for s in d.steps:
        if s["n"] in ED_ITERS[name]:
            first, last = 2 * s["i"] - 1, 2 * s["i"] + 2 * s["n"]
            e0 = ed.ground_energy(workloads.segment_bonds(cfg["bonds"], cfg["ell"], first, last), first, last)
            assert abs(s["energy"] - e0) <= 1e-10, (s, e0)
