"""A run configuration read from JSON drives the GPU path as it drives the oracle (needs an MI355X).

The configuration of the Heisenberg chain (l = 4, m = 32) with its own seed goes through save_config /
load_config and then to both the driver and the oracle: per-site energies agree within 1e-10 and kept
counts exactly (Sec. 3, Steps 2'-6). The fidelity error of iteration 1 (Eq. (12): the overlap of the
converged state with the random start vector of Step 3') agrees with the oracle's for that seed and
differs from a run with the default seed, so the seed really reached the start vectors. Only iteration 1
compares: its legs come from Step 1 alone, while from iteration 2 on each side expresses the two-site
state in its own singular vectors, which are fixed only up to sign (and rotation among equal singular
values), so the same random entries describe different states there.
"""
import pytest
import torch

import workloads
from oracle import idmrg

pytestmark = pytest.mark.gpu

pytest.importorskip("paper_1606_06790_amd.lib")


def test_seeded_json_config_matches_the_oracle(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06790_amd.driver import IDMRG
    path = str(tmp_path / "chain_seed7.json")
    workloads.save_config(dict(workloads.workload("chain"), seed=7), path)
    cfg = workloads.load_config(path)
    print(f"[config] chain seed={cfg['seed']} n_max=6", flush=True)
    ref = idmrg.run(cfg, n_max=6)
    d = IDMRG(cfg)
    d.run(6)
    assert [(s["n"], s["i"]) for s in d.steps] == [(s["n"], s["i"]) for s in ref["steps"]]
    # the log records carry the stage timings of their step and, on superblock 1, the Step 5' energy
    assert all(set(s["step_seconds"]) == {"predict", "lanczos", "truncate", "env"} for s in d.steps)
    assert [s["n"] for s in d.steps if "e_g" in s] == [3]
    assert d.steps[4]["e_g"] == d.e_g[3]
    for g, o in zip(d.steps, ref["steps"]):
        assert abs(g["e_site"] - o["e_site"]) <= 1e-10, (g["n"], g["i"])
        assert g["m_kept"] == o["m_kept"]
    first = [(g, o) for g, o in zip(d.steps, ref["steps"]) if g["n"] == 1]
    for g, o in first:
        assert abs(g["fidelity"] - o["fidelity"]) <= 1e-6, (g["n"], g["i"], g["fidelity"], o["fidelity"])
    d0 = IDMRG(workloads.workload("chain"))
    d0.run(1)
    assert max(abs(g["fidelity"] - h["fidelity"]) for (g, _), h in zip(first, d0.steps)) > 1e-3
