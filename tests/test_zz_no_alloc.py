"""heff_apply_static, the allocation-free variant of heff_apply (needs an MI355X).

Its scratch is the library's static device array instead of a workspace.  It
must give the same results as heff_apply (same plan and kernels: bitwise),
on two calls in a row with the second smaller, allocate nothing (no
workspace attached and no device allocation by the library), and reject a call
whose scratch exceeds the array with IDMRG_EINVAL before launching anything.
"""
import numpy as np
import pytest

import workloads
from oracle import layout, u1

from gpu_common import QP, H, T, mpo_pair, rel_err

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")
torch = pytest.importorskip("torch")

CASES = [  # (legs A, B), MPO workload: the second call is smaller
    (([(-3, 20), (-1, 70), (1, 65), (3, 15)], [(-3, 12), (-1, 67), (1, 80), (3, 30)]), "yc8"),
    (([(-1, 3), (1, 2)], [(-1, 2), (1, 3)]), "chain"),
]


def _case(legs, name, key):
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair(name, 3)
    A, B = legs
    Lf = workloads.gaussian(layout.envL_size(A, dl), 95, key, 1)
    Rf = workloads.gaussian(layout.envR_size(B, dr), 95, key, 2)
    x = workloads.gaussian(layout.psi_size(A, B, QP), 95, key, 3)
    y = layout.psi_to_flat(u1.heff_apply(layout.flat_to_envL(Lf, A, dl), W1, W2, layout.flat_to_envR(Rf, B, dr),
                                         layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr), A, B, QP)
    return dict(left=A, right=B, w1=M1, w2=M2, L=T(Lf), R=T(Rf)), x, y


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_static_scratch_matches_heff_apply(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx_s = lib.Context(0, workspace=False)     # no workspace: any scratch would have to be allocated
    ctx_w = lib.Context(0)
    for key, (legs, name) in enumerate(CASES):
        prob, x, yref = _case(legs, name, key)
        y_s = T(np.full(len(yref), np.nan))
        y_w = T(np.full(len(yref), np.nan))
        lib.heff_apply_static(ctx_s, [prob], [T(x)], [y_s], prec)
        lib.heff_apply(ctx_w, [prob], [T(x)], [y_w], prec)
        torch.cuda.synchronize()
        assert np.array_equal(H(y_s), H(y_w)), (prec, key)
        assert rel_err(H(y_s), yref) <= (1e-13 if prec == "f64" else 5e-5)
    assert ctx_s.stats()["device_allocs"] == 0


def test_static_scratch_rejects_large_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = lib.Context(0, workspace=False)
    m = 1024
    qs, ds = workloads.sector_dims(m)
    A = B = list(zip(qs, ds))
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair("yc8", 3)
    prob = dict(left=A, right=B, w1=M1, w2=M2, L=T(np.zeros(layout.envL_size(A, dl))),
                R=T(np.zeros(layout.envR_size(B, dr))))
    n = layout.psi_size(A, B, QP)
    y = T(np.full(n, 3.0))
    with pytest.raises(lib.IdmrgError) as e:
        lib.heff_apply_static(ctx, [prob], [T(np.ones(n))], [y], "f64")
    assert e.value.code == lib.EINVAL and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert np.all(H(y) == 3.0)
    assert ctx.stats()["device_allocs"] == 0
