"""Checkpoint file of the driver (CPU): every piece of state survives a save / resume round trip bit for bit.

The driver's state after iteration n is what the next iteration reads (Sec. 3): L^(n)_{2i-1}, R^(n)_{2i},
the decomposition of iteration n and Lambda^(n-1) for the prediction of Eq. (10), and the energy history
of Step 5'.  A driver subclass that holds host tensors and opens no device context stands in for the GPU
driver; the GPU test of the same path (resumed run against an uninterrupted one) is in
test_gpu_checkpoint.py.
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads
from paper_1606_06790_amd.driver import CHECKPOINT_VERSION, IDMRG


class HostDriver(IDMRG):
    """The driver's state and file handling without a device context (no kernel is ever called)."""

    def __init__(self, cfg, device=0, prec=None, dense=False, predict=True, chunk=8, log=None, graph=False,
                 batched=True):
        self.torch = torch
        self.cfg = cfg
        self.ell = cfg["ell"]
        self.half = self.ell // 2
        self.dev = torch.device("cpu")
        self.prec = prec or cfg.get("prec", "f64")
        self.predict, self.dense, self.chunk, self.graph, self.batched = predict, dense, chunk, graph, batched
        self.fp32_basis = True
        self.log = log
        self.n = 0
        self.energies, self.steps, self.e_g = {}, [], {}
        self.L, self.R, self.prev, self.lam2 = {}, {}, {}, {}


def _leg(rng, k):
    return [(int(q), int(rng.integers(1, 5))) for q in range(-k, k + 1, 2)]


def _state(seed=3):
    """A driver after iteration n = 14 of the YC8 cylinder with random tensors and legs."""
    rng = np.random.default_rng(seed)
    d = HostDriver(workloads.workload("yc8", m=64), prec="bf16x3", predict=True, chunk=4, batched=False)
    d.fp32_basis = False
    d.n = 14
    T = lambda k: torch.from_numpy(rng.standard_normal(k))
    for i in range(1, d.half + 1):
        d.L[i] = (_leg(rng, 3), T(int(rng.integers(10, 50))))
        d.R[i] = (_leg(rng, 4), T(int(rng.integers(10, 50))))
        C = _leg(rng, 2)
        d.prev[i] = dict(C=C, U=T(30), V=T(31), lam=T(sum(x for _, x in C)), eps=float(rng.random()) * 1e-6,
                         eps_prime=1e-7, m_kept=64, cut_gap=None if i == 2 else 0.25, svd_sweeps=9,
                         svd_converged=True, null_completed=i == 3, warn=0)
        d.lam2[i] = (_leg(rng, 1), T(7))
    for n in range(1, 15):
        for i in range(1, d.half + 1):
            e = float(rng.standard_normal()) * n
            d.energies[(n, i)] = e
            d.steps.append(dict(n=n, i=i, energy=e, e_site=e / (2 * n + 2), iters=int(rng.integers(10, 200)),
                                residual=1e-9, converged=True, cut_gap=None, N=123))
    d.e_g[11] = -0.4379602
    return d


def _same(a, b):
    assert a.n == b.n and a.cfg == b.cfg and a.prec == b.prec
    assert (a.dense, a.predict, a.chunk, a.batched, a.fp32_basis) == (b.dense, b.predict, b.chunk, b.batched,
                                                                      b.fp32_basis)
    for name in ("L", "R", "lam2"):
        x, y = getattr(a, name), getattr(b, name)
        assert sorted(x) == sorted(y)
        for i in x:
            assert x[i][0] == y[i][0]
            assert x[i][1].dtype == y[i][1].dtype == torch.float64
            assert torch.equal(x[i][1], y[i][1])
    assert sorted(a.prev) == sorted(b.prev)
    for i in a.prev:
        p, q = a.prev[i], b.prev[i]
        assert sorted(p) == sorted(q)
        for k in p:
            if isinstance(p[k], torch.Tensor):
                assert torch.equal(p[k], q[k])
            else:
                assert p[k] == q[k], k
    # energies and records are exact: JSON writes the shortest decimal that reads back as the same double
    assert a.energies == b.energies and a.e_g == b.e_g and a.steps == b.steps


def test_checkpoint_round_trip_is_exact(tmp_path):
    d = _state()
    path = str(tmp_path / "state.npz")
    d.save(path)
    r = HostDriver.resume(path)
    _same(d, r)
    # the prediction's inputs come back with their legs and sizes intact
    assert [r.prev[i]["lam"].numel() for i in r.prev] == [sum(x for _, x in r.prev[i]["C"]) for i in r.prev]


def test_checkpoint_file_needs_no_unpickling(tmp_path):
    d = _state()
    path = str(tmp_path / "state.npz")
    d.save(path)
    with np.load(path, allow_pickle=False) as z:
        assert all(z[k].dtype == np.float64 for k in z.files if k != "header")
        h = json.loads(str(z["header"]))
    assert h["version"] == CHECKPOINT_VERSION and h["n"] == 14
    assert not (tmp_path / "state.npz.partial").exists()


def test_checkpoint_before_the_first_iteration(tmp_path):
    """n = 0: only the Step 1 environments exist (no decomposition yet)."""
    d = _state()
    d.n, d.prev, d.lam2, d.energies, d.steps, d.e_g = 0, {}, {}, {}, [], {}
    path = str(tmp_path / "s0.npz")
    d.save(path)
    _same(d, HostDriver.resume(path))


def test_checkpoint_rejects_another_version(tmp_path):
    d = _state()
    path = str(tmp_path / "state.npz")
    d.save(path)
    with np.load(path, allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    h = json.loads(str(arrays["header"]))
    h["version"] = CHECKPOINT_VERSION + 1
    arrays["header"] = np.array(json.dumps(h))
    np.savez(path, **arrays)
    with pytest.raises(ValueError, match="version"):
        HostDriver.resume(path)
