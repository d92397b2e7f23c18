"""Write the oracle trajectories that the GPU trajectory tests compare against.

Runs the FP64 oracle (``oracle.idmrg.run`` in U(1) mode, Sec. 3 of the paper:
Steps 1-7 with the parallel Steps 2', 3', 5') on reduced-m versions of the
cylinder and random-chain workloads and stores, per superblock (n, i), the
energy, the per-site energy, the kept count, the Lanczos iterations, the
fidelity error of Eq. (12) and the discarded weight of Eq. (14), plus every
Step 5' estimate e_g.  Nothing here comes from the GPU path.

    python tests/golden/make_trajectories.py            # all fixtures
    python tests/golden/make_trajectories.py yc4_m128   # one fixture
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import idmrg  # noqa: E402

# name: (workload, m, n_max, run-parameter overrides).  n_max covers the untruncated iterations
# (2^n <= m, where the oracle equals exact diagonalisation) and more than one full unit-cell
# period of truncated iterations, so every (W_f(c1), W_f(c2)) alignment and the wrap
# R_{l+2} = R_2 occur.  The "_tight" runs stop each Lanczos solve at a residual of 1e-10
# instead of 1e-8: the GPU's mixed-precision solves end at a different point of the residual
# ball than the oracle's FP64 Krylov sequence, and a truncated iteration's energy depends to
# first order on the previous state, so their comparison at 1e-9 per site needs both sides to
# converge further than the production tolerance.
FIXTURES = {
    "yc8_m128": ("yc8", 128, 24, {}),
    "yc4_m128": ("yc4", 128, 20, {}),
    "random_chain_m256": ("random_chain", 256, 24, {}),
    "yc8_m128_tight": ("yc8", 128, 24, {"tol_res": 1e-10}),
    "yc4_m128_tight": ("yc4", 128, 20, {"tol_res": 1e-10}),
    "random_chain_m256_tight": ("random_chain", 256, 24, {"tol_res": 1e-10}),
}


def path(name):
    return os.path.join(HERE, f"traj_{name}.json")


def make(name):
    wl, m, n_max, over = FIXTURES[name]
    cfg = workloads.workload(wl, m=m, **over)
    t0 = time.perf_counter()
    r = idmrg.run(cfg, mode="u1", n_max=n_max)
    keys = ("n", "i", "energy", "e_site", "m_kept", "iters", "fidelity", "eps")
    out = dict(workload=wl, m=m, n_max=n_max, overrides=over, mode="u1",
               generator="tests/golden/make_trajectories.py (oracle.idmrg.run, FP64)",
               steps=[{k: s[k] for k in keys} for s in r["steps"]],
               e_g={str(n): e for n, e in r["e_g"].items()})
    with open(path(name), "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"{name}: {len(out['steps'])} superblock records, e_g at n = {sorted(r['e_g'])}, "
          f"{time.perf_counter() - t0:.1f} s", flush=True)


def load(name):
    with open(path(name)) as f:
        return json.load(f)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(FIXTURES)):
        make(name)
