"""GPU parity at the full sizes of the cylinder workloads: YC8 kagome at m = 2048
and m = 4096 (D up to 20, split-bf16 matvec) and YC4 square at m = 1024 (D = 14,
FP32 matvec).

The superblock is built without the GPU path: the MPO from the oracle's
finite-state construction, environments grown by the oracle's own Eqs. (4)
and (5) from the boundary vectors through twelve sites on each side, with
seeded random block isometries (QR of Gaussian draws) in place of the
optimised ones.  H_eff is then the projection of the segment Hamiltonian onto
an orthonormal basis, symmetric like the real one, with legs of about a dozen
U(1) sectors summing to m states.  The oracle computes every output at these
sizes in seconds, so the comparisons are elementwise.
"""
import numpy as np
import pytest

import workloads
from oracle import layout, u1
from oracle import mpo as omp

from gpu_common import QP, H, T, rel_err

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")

MIXED_TOL = {"f32": 5e-6, "bf16x3": 5e-5}
# (workload, m, matvec policy of its benchmark configuration, smallest MPO channel count at the centre,
#  left sites c of the superblock, sites grown on the right)
CONFIGS = {"yc8": ("yc8", 2048, "bf16x3", 14, 13, 12), "yc8_m4096": ("yc8", 4096, "bf16x3", 14, 15, 14),
           "yc4": ("yc4", 1024, "f32", 14, 13, 12)}


def _grow(name, m, c, nright):
    """Environments of superblock (sites c, c+1) of a cylinder workload with legs of about m states."""
    cfg = workloads.workload(name)
    ell = cfg["ell"]
    Ws, dq = omp.build_mpo(ell, cfg["bonds"])
    f = lambda k: (k - 1) % ell + 1
    W = lambda k: Ws[f(k) - 1]
    cut = lambda k: dq[f(k)]

    def new_leg(rows_of, charges):
        # min(m, rows) states shared over the charges in proportion to a Gaussian profile
        # (one state at a time to the sector of largest weight per state), within each
        # sector's number of rows
        qs = sorted(charges)
        w = [np.exp(-((q / 2.0) ** 2) / 8.0) for q in qs]
        cap = [rows_of(q) for q in qs]
        k = [0] * len(qs)
        for _ in range(min(m, sum(cap))):
            i = max((i for i in range(len(qs)) if k[i] < cap[i]), key=lambda i: w[i] / (k[i] + 1))
            k[i] += 1
        return [(q, kq) for q, kq in zip(qs, k) if kq > 0]

    def isometry(rows_of_sector, C, key):
        out = {}
        for qc, kc in C:
            rows = rows_of_sector(qc)
            r = sum(x[2] for x in rows)
            Q = np.linalg.qr(workloads.gaussian(r * kc, 77, key, qc + 1000).reshape(r, kc))[0]
            r0 = 0
            for row in rows:
                out[(row[0], row[1], qc)] = Q[r0:r0 + row[2]]
                r0 += row[2]
        return out

    L, A = u1.init_left(W(1), cut(1), QP)
    for j in range(2, c):
        Ad = dict(A)
        C = new_leg(lambda q: sum(Ad.get(q - s, 0) for s in QP), {qa + s for qa, _ in A for s in QP})
        L = u1.update_env_left(L, W(j), isometry(lambda q: layout.U_rows(A, QP, q), C, j), A, QP, C, cut(j - 1),
                               cut(j))
        A = C
    K = c + 1 + nright
    R, B = u1.init_right(W(K), cut(K - 1), QP)
    for j in range(K - 1, c + 1, -1):
        Bd = dict(B)
        C = new_leg(lambda q: sum(Bd.get(q + s, 0) for s in QP), {qb - s for qb, _ in B for s in QP})
        R = u1.update_env_right(R, W(j), isometry(lambda q: layout.V_rows(B, QP, q), C, 1000 + j), B, QP, C,
                                cut(j - 1), cut(j))
        B = C
    return dict(L=L, A=A, R=R, B=B, W1=W(c), W2=W(c + 1), dl=cut(c - 1), dm=cut(c), dr=cut(c + 1))


@pytest.fixture(scope="module", params=sorted(CONFIGS))
def full(request):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06790_amd.lib import Mpo
    name, m, prec, dmin, c, nright = CONFIGS[request.param]
    s = _grow(name, m, c, nright)
    s.update(name=name, m=m, prec=prec, dmin=dmin)
    A, B = s["A"], s["B"]
    s["prob"] = dict(left=A, right=B, w1=Mpo(s["W1"], s["dl"], s["dm"], QP), w2=Mpo(s["W2"], s["dm"], s["dr"], QP),
                     L=T(layout.envL_to_flat(s["L"], A, s["dl"])), R=T(layout.envR_to_flat(s["R"], B, s["dr"])))
    s["N"] = layout.psi_size(A, B, QP)
    s["x"] = workloads.gaussian(s["N"], 78)
    s["y"] = layout.psi_to_flat(u1.heff_apply(s["L"], s["W1"], s["W2"], s["R"], layout.flat_to_psi(s["x"], A, B, QP),
                                              A, B, QP, s["dl"], s["dr"]), A, B, QP)
    s["ctx"] = lib.Context(0)
    return s


def test_fullsize_shape(full):
    m = full["m"]
    assert sum(d for _, d in full["A"]) == m and sum(d for _, d in full["B"]) == m
    assert len(full["dl"]) >= full["dmin"] and len(full["dr"]) >= full["dmin"] and full["N"] > m * m // 4


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_fullsize_heff_apply(full, prec):
    """Every element of H_eff x at the full size against the oracle."""
    y = T(np.zeros(full["N"]))
    lib.heff_apply(full["ctx"], [full["prob"]], [T(full["x"])], [y], prec)
    err = rel_err(H(y), full["y"])
    assert err <= (1e-13 if prec == "f64" else MIXED_TOL[prec]), err


def test_fullsize_truncate(full):
    """Schmidt decomposition of a Gaussian two-site state at the full m: kept legs, every kept
    singular value, eps, isometries and kept subspaces against the oracle (LAPACK SVD)."""
    A, B, m = full["A"], full["B"], full["m"]
    x = workloads.gaussian(full["N"], 79)
    x /= np.linalg.norm(x)
    tr = u1.truncate_twosite(layout.flat_to_psi(x, A, B, QP), A, B, QP, m, 1e-14, 1e-5)
    o = lib.truncate_twosite(full["ctx"], [dict(left=A, right=B, psi=T(x))], QP, m, 1e-14, 1e-5)[0]
    assert o["svd_converged"]
    assert o["C"] == tr["C"] and o["m_kept"] == tr["m_kept"] == m
    assert abs(o["eps"] - tr["eps"]) <= 1e-12
    lam = layout.flat_to_lam(H(o["lam"]), o["C"])
    U = layout.flat_to_U(H(o["U"]), A, QP, o["C"])
    V = layout.flat_to_V(H(o["V"]), B, QP, o["C"])
    # Orthonormality: the accumulated Jacobi transform of a row is the product of
    # about (sweeps x blocks) ~ 10^3 orthogonal 64 x 64 updates, each orthogonal to
    # ~1e-14, so deviations of order 1e-12 are expected at n ~ 800 (LAPACK's own
    # bound is O(n eps)); 1e-11 leaves energies untouched at the 1e-10 level.
    for q, k in o["C"]:
        assert np.abs(lam[q] - tr["lam"][q]).max() <= 1e-13
        Ug = np.concatenate([U[(a, s, q)] for (a, s, _) in layout.U_rows(A, QP, q)])
        Vg = np.concatenate([V[(s, b, q)] for (s, b, _) in layout.V_rows(B, QP, q)])
        assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-11
        assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-11
        if tr["cut_gap"] is None or tr["cut_gap"] > 1e-6:
            Uo = np.concatenate([tr["U"][(a, s, q)] for (a, s, _) in layout.U_rows(A, QP, q)])
            assert np.abs(Ug @ Ug.T - Uo @ Uo.T).max() <= 1e-9


@pytest.mark.parametrize("prec", ["f64", "policy"])
def test_fullsize_lanczos(full, prec):
    """Lanczos at the full size from a Gaussian start, in FP64 and in the configuration's mixed
    policy.  The returned energy must be the oracle's Rayleigh quotient of the returned state,
    and the reported residual the oracle's |H psi - E psi| (so the stop decision was taken on
    the true residual)."""
    A, B = full["A"], full["B"]
    if prec == "policy":
        prec = full["prec"]
    psi = T(workloads.gaussian(full["N"], 80))
    es, infos = lib.lanczos_solve_batch(full["ctx"], [full["prob"]], [psi], 1e-12, 1e-8, 300, prec)
    p = H(psi)
    assert abs(np.linalg.norm(p) - 1.0) <= 1e-12
    hp = layout.psi_to_flat(u1.heff_apply(full["L"], full["W1"], full["W2"], full["R"], layout.flat_to_psi(p, A, B, QP),
                                          A, B, QP, full["dl"], full["dr"]), A, B, QP)
    e_orc = float(p @ hp)
    res_orc = float(np.linalg.norm(hp - es[0] * p))
    assert abs(es[0] - e_orc) <= 1e-11 * abs(e_orc)
    assert abs(res_orc - infos[0]["residual"]) <= 1e-10 + 1e-6 * res_orc
    if infos[0]["converged"]:
        assert res_orc <= 1e-8 * 1.01
