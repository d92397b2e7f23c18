"""Shared helpers of the GPU parity tests (inputs and conversions only)."""
import numpy as np
import pytest

import workloads
from oracle import mpo as omp

torch = pytest.importorskip("torch")

QP = [1, -1]


def dev():
    return torch.device("cuda", 0)


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev())


def H(t):
    return t.detach().cpu().numpy()


def mpo_pair(name, c1):
    """Oracle MPO tensors W_{c1}, W_{c1+1} of a workload, with their channel charges, as
    (oracle arrays, library Mpo objects)."""
    from paper_1606_06790_amd.lib import Mpo
    cfg = workloads.workload(name)
    Ws, dq = omp.build_mpo(cfg["ell"], cfg["bonds"])
    ell = cfg["ell"]
    f = lambda k: (k - 1) % ell + 1
    W1, W2 = Ws[f(c1) - 1], Ws[f(c1 + 1) - 1]
    dl, dm, dr = dq[f(c1) - 1], dq[f(c1)], dq[f(c1 + 1)]
    return (W1, W2, dl, dm, dr), (Mpo(W1, dl, dm, QP), Mpo(W2, dm, dr, QP))


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
