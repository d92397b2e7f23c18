"""GPU parity on the matvec microbenchmark configuration and on the two
orthogonalisation modes of the Lanczos solver (needs an MI355X).

Matvec microbenchmark: the Heisenberg chain MPO (D = 5, d = 2), Gaussian FP64
environments (non-identity channels; the identity channels are implied) and a
Gaussian state, m = 256, 512, 1024, dense (one sector) and U(1)-blocked (the
benchmark's Gaussian sector profile), in every matvec precision.  Every output
element is compared with the oracle.
"""
import numpy as np
import pytest

import workloads
from oracle import dense as odense
from oracle import layout, u1

from gpu_common import QP, H, T, mpo_pair, rel_err

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")

TOL = {"f64": 1e-13, "f32": 5e-6, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _u1_problem(m, key):
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair("chain", 1)
    qs, ds = workloads.sector_dims(m)
    A = B = list(zip(qs, ds))
    nL, nR, nx = layout.envL_size(A, dl), layout.envR_size(B, dr), layout.psi_size(A, B, QP)
    Lf, Rf, x = workloads.gaussian(nL, key, 1), workloads.gaussian(nR, key, 2), workloads.gaussian(nx, key, 3)
    y = layout.psi_to_flat(u1.heff_apply(layout.flat_to_envL(Lf, A, dl), W1, W2, layout.flat_to_envR(Rf, B, dr),
                                         layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr), A, B, QP)
    prob = dict(left=A, right=B, w1=M1, w2=M2, L=T(Lf), R=T(Rf))
    return prob, x, y, (Lf, Rf, A, B, W1, W2, dl, dr)


@pytest.mark.parametrize("m", [256, 512, 1024])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_microbench_u1(ctx, m, prec):
    prob, x, y, _ = _u1_problem(m, 90 + m)
    yg = T(np.full(len(y), np.nan))
    lib.heff_apply(ctx, [prob], [T(x)], [yg], prec)
    err = rel_err(H(yg), y)
    assert err <= TOL[prec], err


@pytest.mark.parametrize("m", [512, 1024])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_microbench_dense(ctx, m, prec):
    """No symmetry blocks (all charges 0): one block per (s1, s2)."""
    from paper_1606_06790_amd.lib import Mpo
    (W1, W2, _, _, _), _ = mpo_pair("chain", 1)
    D = W1.shape[0]
    z = lambda k: [0] * k
    M1, M2 = Mpo(W1, z(D), z(D), [0, 0]), Mpo(W2, z(D), z(D), [0, 0])
    Lf = workloads.gaussian((D - 1) * m * m, 91, m, 1)
    Rf = workloads.gaussian(m * (D - 1) * m, 91, m, 2)
    x = workloads.gaussian(4 * m * m, 91, m, 3)
    L = np.zeros((m, D, m))
    L[:, :D - 1, :] = Lf.reshape(D - 1, m, m).transpose(1, 0, 2)
    L[:, D - 1, :] = np.eye(m)
    R = np.zeros((m, D, m))
    R[:, 1:, :] = Rf.reshape(m, D - 1, m)
    R[:, 0, :] = np.eye(m)
    y = odense.psi_to_flat(odense.heff_apply(L, W1, W2, R, odense.psi_from_flat(x, m, 2, m)))
    yg = T(np.full(4 * m * m, np.nan))
    lib.heff_apply(ctx, [dict(left=[(0, m)], right=[(0, m)], w1=M1, w2=M2, L=T(Lf), R=T(Rf))], [T(x)], [yg], prec)
    err = rel_err(H(yg), y)
    assert err <= TOL[prec], err


def _grown(name, m, c, nright):
    """A symmetric H_eff (oracle-grown environments, see fullsize_ops) as a library
    problem plus the oracle's matvec on it."""
    from fullsize_ops import grow as _grow
    from paper_1606_06790_amd.lib import Mpo
    s = _grow(name, m, c, nright)
    A, B = s["A"], s["B"]
    prob = dict(left=A, right=B, w1=Mpo(s["W1"], s["dl"], s["dm"], QP), w2=Mpo(s["W2"], s["dm"], s["dr"], QP),
                L=T(layout.envL_to_flat(s["L"], A, s["dl"])), R=T(layout.envR_to_flat(s["R"], B, s["dr"])))

    def apply(v):
        return layout.psi_to_flat(u1.heff_apply(s["L"], s["W1"], s["W2"], s["R"], layout.flat_to_psi(v, A, B, QP),
                                                A, B, QP, s["dl"], s["dr"]), A, B, QP)
    return prob, layout.psi_size(A, B, QP), apply


def test_lanczos_cgs2_modes(ctx):
    """The selective second Gram-Schmidt pass against CGS2 in every iteration, from the same
    start: both converge to the same energy, each energy is the oracle's Rayleigh quotient of
    the returned state, and the selective mode runs the second pass only rarely."""
    prob, N, apply = _grown("yc8", 256, 10, 9)
    x0 = workloads.gaussian(N, 92)
    out = {}
    for cgs2 in (False, True):
        psi = T(x0)
        es, infos = lib.lanczos_solve_batch(ctx, [prob], [psi], 1e-12, 1e-9, 300, "f64", cgs2=cgs2)
        p = H(psi)
        hp = apply(p)
        e_orc = float(p @ hp)
        assert infos[0]["converged"] == 1
        assert abs(es[0] - e_orc) <= 1e-12 * abs(e_orc)
        assert float(np.linalg.norm(hp - es[0] * p)) <= 1e-9 * 1.01
        out[cgs2] = (es[0], infos[0])
    (e1, i1), (e2, i2) = out[False], out[True]
    assert abs(e1 - e2) <= 1e-12 * abs(e2)
    assert i2["reorth_passes"] == i2["iters"] - 1 or i2["reorth_passes"] == i2["iters"]
    assert 1 <= i1["reorth_passes"] <= max(2, i1["iters"] // 10)


def test_lanczos_exhausts_space(ctx):
    """A two-site space smaller than k_max: the iteration runs into the invariant subspace
    (beta -> 0, where the projection removes almost all of w and the second pass must run)
    and still returns the lowest eigenvalue of the dense matrix."""
    prob, N, apply = _grown("chain", 6, 3, 2)
    assert N < 200
    Hd = np.stack([apply(np.eye(N)[k]) for k in range(N)], axis=1)
    assert np.abs(Hd - Hd.T).max() <= 1e-12 * np.abs(Hd).max()
    e_exact = float(np.linalg.eigvalsh(0.5 * (Hd + Hd.T))[0])
    psi = T(workloads.gaussian(N, 93))
    es, infos = lib.lanczos_solve_batch(ctx, [prob], [psi], 0.0, 0.0, 300, "f64")
    assert abs(es[0] - e_exact) <= 1e-12 * max(1.0, abs(e_exact))
    assert infos[0]["iters"] <= N
    p = H(psi)
    assert abs(np.linalg.norm(p) - 1.0) <= 1e-12
    assert float(np.linalg.norm(Hd @ p - es[0] * p)) <= 1e-10 * max(1.0, abs(e_exact))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_low_precision_energy_shift(ctx, prec):
    """The environments carry the block energies H_L, H_R as large diagonal-heavy blocks.
    Adding c I to H_L and c I to H_R adds 2c I to H_eff; the low-precision copies hold the
    blocks shifted by their mean diagonal and the shift comes back in FP64, so the absolute
    error of the matvec must stay at the level it has without the offset (unshifted copies
    would round the 2c |x| term at the low precision's relative error)."""
    from fullsize_ops import grow as _grow
    from paper_1606_06790_amd.lib import Mpo
    s = _grow("yc8", 256, 10, 9)
    A, B, dl, dr = s["A"], s["B"], s["dl"], s["dr"]
    x = workloads.gaussian(layout.psi_size(A, B, QP), 94)
    errs = []
    for c in (0.0, 40.0):
        L = {k: (v + c * np.eye(v.shape[0]) if k[0] == 0 and k[1] == k[2] else v) for k, v in s["L"].items()}
        R = {k: (v + c * np.eye(v.shape[0]) if k[0] == len(dr) - 1 and k[1] == k[2] else v) for k, v in s["R"].items()}
        y = layout.psi_to_flat(u1.heff_apply(L, s["W1"], s["W2"], R, layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr),
                               A, B, QP)
        prob = dict(left=A, right=B, w1=Mpo(s["W1"], dl, s["dm"], QP), w2=Mpo(s["W2"], s["dm"], dr, QP),
                    L=T(layout.envL_to_flat(L, A, dl)), R=T(layout.envR_to_flat(R, B, dr)))
        yg = T(np.full(len(y), np.nan))
        lib.heff_apply(ctx, [prob], [T(x)], [yg], prec)
        errs.append(float(np.abs(H(yg) - y).max()))
        if c > 0:   # the oracle's result does include the offset
            assert np.abs(y - layout.psi_to_flat(u1.heff_apply(s["L"], s["W1"], s["W2"], s["R"],
                                                                layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr),
                                                  A, B, QP) - 2 * c * x).max() <= 1e-11 * np.abs(y).max()
    ulp = {"f32": 2.0 ** -24, "bf16x3": 2.0 ** -16}[prec]
    xm = float(np.abs(x).max())
    assert errs[1] <= 3 * errs[0] + 0.1 * ulp * 80 * xm, errs
