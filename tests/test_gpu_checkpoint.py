"""Resume from a checkpoint on the GPU (needs an MI355X): a run interrupted after iteration n_save and
resumed in a new driver (new library context, so a fresh tile tuner) reproduces the uninterrupted run
bit for bit: every superblock energy, every record (apart from its timings) and the final environments.

Cases: the Heisenberg chain (l = 4, m = 32) in FP64, saved before truncation starts, and the YC8 kagome
cylinder (l = 12, m = 64) with the split-bf16 matvec and FP64 refinement, saved after one unit-cell period,
so that the resumed run starts with the prediction of Eq. (10) from the restored decompositions.
"""
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

pytest.importorskip("paper_1606_06790_amd.lib")

CASES = [("chain", 32, "f64", 3, 9), ("yc8", 64, "bf16x3", 12, 16)]


@pytest.mark.parametrize("wl,m,prec,n_save,n_max", CASES)
def test_resume_matches_uninterrupted_run(tmp_path, wl, m, prec, n_save, n_max):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06790_amd.driver import IDMRG
    print(f"[checkpoint] {wl} m={m} prec={prec} save at n={n_save}, run to n={n_max}", flush=True)
    cfg = workloads.workload(wl, m=m)
    a = IDMRG(cfg, prec=prec)
    a.run(n_save)
    path = str(tmp_path / "state.npz")
    a.save(path)
    a.run(n_max)
    b = IDMRG.resume(path)
    assert b.n == n_save and b.prec == prec
    b.run(n_max)
    assert b.energies == a.energies
    assert b.e_g == a.e_g
    # the records match except for their wall-clock timings
    strip = lambda steps: [{k: v for k, v in r.items() if k != "step_seconds"} for r in steps]
    assert strip(b.steps) == strip(a.steps)
    assert all(s["converged"] and s["svd_converged"] for s in b.steps)
    for i in a.L:
        assert a.L[i][0] == b.L[i][0] and torch.equal(a.L[i][1], b.L[i][1])
        assert a.R[i][0] == b.R[i][0] and torch.equal(a.R[i][1], b.R[i][1])
    for i in a.prev:
        for k in ("U", "V", "lam"):
            assert torch.equal(a.prev[i][k], b.prev[i][k])
