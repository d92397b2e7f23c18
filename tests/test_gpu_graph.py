"""Lanczos iterations replayed from captured HIP graphs against the same
iterations launched directly (needs an MI355X).

Graph mode captures whole chunks of iterations (matvec and vector kernels) once
per pass shape and replays them many times per solve, with the host's stop-flag
reads and the direct launches of partial chunks in between.  The kernels and
their order are the same in both modes and every reduction is deterministic, so
energies, states and counters must agree bit for bit, on every replay.
"""
import numpy as np
import pytest

import workloads

from gpu_common import H, T

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


@pytest.fixture(scope="module")
def batch():
    """Three superblocks of different sizes (uneven U(1) blocks), as one batch."""
    from test_gpu_configs import _grown
    out = [_grown("yc8", 256, 10, 9), _grown("yc8", 160, 9, 8), _grown("yc4", 128, 7, 6)]
    return [p for p, _, _ in out], [n for _, n, _ in out]


@pytest.mark.parametrize("prec,chunk", [("f64", 8), ("f32", 8), ("bf16x3", 8), ("bf16x3", 5)])
def test_graph_matches_direct(ctx, batch, prec, chunk):
    probs, sizes = batch
    starts = [workloads.gaussian(n, 95, k) for k, n in enumerate(sizes)]
    runs = []
    for graph in (False, True, True):   # the second graph call captures and replays again
        psis = [T(x) for x in starts]
        es, infos = lib.lanczos_solve_batch(ctx, probs, psis, 1e-12, 1e-8, 300, prec, chunk, graph=graph)
        runs.append((es, infos, [H(p) for p in psis]))
    e0, i0, p0 = runs[0]
    assert all(i["converged"] for i in i0)
    assert max(i["iters"] for i in i0) > 3 * chunk   # enough chunks to replay each graph several times
    for es, infos, ps in runs[1:]:
        assert es == e0
        for a, b in zip(infos, i0):
            assert {k: a[k] for k in ("iters", "fp64_matvecs", "reorth_passes", "converged", "flags")} == \
                   {k: b[k] for k in ("iters", "fp64_matvecs", "reorth_passes", "converged", "flags")}
            assert a["residual"] == b["residual"] and a["overlap0"] == b["overlap0"]
        for a, b in zip(ps, p0):
            assert np.array_equal(a, b)


def test_graph_ignored_while_profiling(ctx, batch):
    """With profiling on, every launch is bracketed by events, so graph mode falls back to direct
    launches: the profile then counts one Lanczos vector launch group per iteration."""
    probs, sizes = batch
    psis = [T(workloads.gaussian(n, 96, k)) for k, n in enumerate(sizes)]
    ctx.profile(True)
    try:
        _, infos = lib.lanczos_solve_batch(ctx, probs, psis, 1e-12, 1e-8, 300, "f64", 8, graph=True)
        prof = ctx.profile_get()
    finally:
        ctx.profile(False)
    # class 4 (Lanczos vector kernels): one record per iteration plus start, finish and residual
    assert prof["lanczos_vec"][0] >= max(i["iters"] for i in infos)
