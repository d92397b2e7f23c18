"""Store the oracle's ground energies of the full-size superblock operators.

For each operator of tests/fullsize_ops.py (YC8 kagome at m = 2048 and 4096,
YC4 square at m = 1024) the FP64 oracle Lanczos (full re-orthogonalisation,
the stop rule of the iteration: |dtheta| <= 1e-12 and residual <= 1e-8) is
run from the seeded Gaussian start that the GPU test uses, and its energy,
iteration count and final residual are written to fullsize_energies.json.
The operators have N = 0.58M to 9.2M, which is minutes of oracle time, so the
GPU test reads the stored value instead of recomputing it.  Nothing here comes
from the GPU path.

    python tests/golden/make_fullsize_energies.py [yc4 yc8 yc8_m4096]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)

import workloads  # noqa: E402
from oracle.lanczos import lanczos  # noqa: E402

import fullsize_ops  # noqa: E402

PATH = os.path.join(HERE, "fullsize_energies.json")
START_KEY = 80   # workloads.gaussian(N, 80): the start vector of the GPU test


def load():
    with open(PATH) as f:
        return json.load(f)


def main(names):
    out = load() if os.path.exists(PATH) else {}
    for name in names:
        t0 = time.perf_counter()
        s = fullsize_ops.operator(name)
        sol = lanczos(s["mv"], workloads.gaussian(s["N"], START_KEY), 1e-12, 1e-8, 300)
        out[name] = dict(energy=sol["energy"], iters=sol["iters"], residual=sol["residual"], N=s["N"],
                         generator="tests/golden/make_fullsize_energies.py (oracle.lanczos, FP64)")
        with open(PATH, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")
        print(f"{name}: N = {s['N']}, E0 = {sol['energy']!r}, {sol['iters']} iterations, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(fullsize_ops.CONFIGS))
