"""GPU parity at the full sizes of the cylinder workloads: YC8 kagome at m = 2048
and m = 4096 (D up to 20, split-bf16 matvec) and YC4 square at m = 1024 (D = 14,
FP32 matvec).

The superblock operators come from tests/fullsize_ops.py (oracle MPO and
oracle-grown environments with seeded isometries).  The oracle computes every
output of heff_apply, truncate_twosite, update_env and predict_wavefunction
at these sizes in seconds, so those comparisons are elementwise; the Lanczos
ground energy is compared with the oracle's own Lanczos on the same operator
(live for YC4, stored by tests/golden/make_fullsize_energies.py for YC8).
"""
import numpy as np
import pytest

import workloads
from oracle import layout, u1
from oracle.lanczos import lanczos

import fullsize_ops
from fullsize_ops import QP, CONFIGS
from gpu_common import H, T, rel_err

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")

MIXED_TOL = {"f32": 5e-6, "bf16x3": 5e-5}


@pytest.fixture(scope="module", params=sorted(CONFIGS))
def full(request):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06790_amd.lib import Mpo
    print(f"[fullsize] building {request.param}", flush=True)
    s = fullsize_ops.operator(request.param)
    s["key"] = request.param
    A, B = s["A"], s["B"]
    s["prob"] = dict(left=A, right=B, w1=Mpo(s["W1"], s["dl"], s["dm"], QP), w2=Mpo(s["W2"], s["dm"], s["dr"], QP),
                     L=T(layout.envL_to_flat(s["L"], A, s["dl"])), R=T(layout.envR_to_flat(s["R"], B, s["dr"])))
    s["x"] = workloads.gaussian(s["N"], 78)
    s["y"] = s["mv"](s["x"])
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
    # Kept subspaces (projectors) to 1e-10.  Orthonormality to 5e-12 rather than 1e-13: the
    # accumulated Jacobi transform of a row is a product of about (sweeps x block pairs) ~ 10^3
    # orthogonal 64 x 64 updates, each orthogonal to ~1e-15 .. 1e-14, so deviations grow to
    # ~1e-12 for blocks of 2000-2600 rows (measured: 5.8e-13 at m = 2048, 1.4e-12 at m = 4096;
    # LAPACK's own bound is O(n eps), ~5e-13 at n = 2600).
    worst_orth = worst_proj = 0.0
    for q, k in o["C"]:
        assert np.abs(lam[q] - tr["lam"][q]).max() <= 1e-13
        Ug = np.concatenate([U[(a, s, q)] for (a, s, _) in layout.U_rows(A, QP, q)])
        Vg = np.concatenate([V[(s, b, q)] for (s, b, _) in layout.V_rows(B, QP, q)])
        worst_orth = max(worst_orth, np.abs(Ug.T @ Ug - np.eye(k)).max(), np.abs(Vg.T @ Vg - np.eye(k)).max())
        if tr["cut_gap"] is None or tr["cut_gap"] > 1e-6:
            Uo = np.concatenate([tr["U"][(a, s, q)] for (a, s, _) in layout.U_rows(A, QP, q)])
            worst_proj = max(worst_proj, np.abs(Ug @ Ug.T - Uo @ Uo.T).max())
    print(f"[fullsize] {full['key']} truncate: orthonormality {worst_orth:.2e}, projectors {worst_proj:.2e}, "
          f"sweeps {o['svd_sweeps']}", flush=True)
    assert worst_orth <= 5e-12
    assert worst_proj <= 1e-10


def _lam(leg, key, zero_every=0):
    lam = np.abs(workloads.gaussian(sum(k for _, k in leg), 81, key)) + 1e-3
    if zero_every:
        lam[::zero_every] = 0.0
    return lam


@pytest.mark.parametrize("side", ["left", "right"])
def test_fullsize_update_env(full, side):
    """Eqs. (4), (5) at the full size: the environment of the next iteration from the
    superblock's environment, its MPO tensor and a full-size isometry (m new states), every
    element against the oracle."""
    m = full["m"]
    if side == "left":
        A, W, dl, dm = full["A"], full["W1"], full["dl"], full["dm"]
        Cl = fullsize_ops.u_leg(A, m)
        iso = fullsize_ops.isometry(lambda q: layout.U_rows(A, QP, q), Cl, 5001)
        ref = layout.envL_to_flat(u1.update_env_left(full["L"], W, iso, A, QP, Cl, dl, dm), Cl, dm)
        item = dict(old_leg=A, new_leg=Cl, w=full["prob"]["w1"], env_old=full["prob"]["L"],
                    iso=T(layout.U_to_flat(iso, A, QP, Cl)))
        out = lib.update_env(full["ctx"], lib.LEFT, [item])[0]
    else:
        B, W, dm, dr = full["B"], full["W2"], full["dm"], full["dr"]
        Cl = fullsize_ops.v_leg(B, m)
        iso = fullsize_ops.isometry(lambda q: layout.V_rows(B, QP, q), Cl, 5002)
        ref = layout.envR_to_flat(u1.update_env_right(full["R"], W, iso, B, QP, Cl, dm, dr), Cl, dm)
        item = dict(old_leg=B, new_leg=Cl, w=full["prob"]["w2"], env_old=full["prob"]["R"],
                    iso=T(layout.V_to_flat(iso, B, QP, Cl)))
        out = lib.update_env(full["ctx"], lib.RIGHT, [item])[0]
    assert sum(k for _, k in Cl) == m
    err = rel_err(H(out), ref)
    print(f"[fullsize] {full['key']} update_env {side}: {len(ref)} elements, max rel err {err:.2e}", flush=True)
    assert err <= 1e-13


def test_fullsize_predict(full):
    """Eq. (10) at the full size: legs of m states around the contracted leg (the superblock's
    left leg), Schmidt values with every seventh of the contracted leg's values zero (the
    lambda = 0 branch), every element of the predicted state against the oracle."""
    m = full["m"]
    Bt = full["A"]
    Aa = fullsize_ops.v_leg(Bt, m)
    Bb = fullsize_ops.u_leg(Bt, m)
    V = fullsize_ops.isometry(lambda q: layout.V_rows(Bt, QP, q), Aa, 6001)
    U = fullsize_ops.isometry(lambda q: layout.U_rows(Bt, QP, q), Bb, 6002)
    la, lt, lb = _lam(Aa, 1), _lam(Bt, 2, zero_every=7), _lam(Bb, 3)
    ref = u1.predict_wavefunction(layout.flat_to_lam(la, Aa), V, layout.flat_to_lam(lt, Bt), U,
                                  layout.flat_to_lam(lb, Bb), Aa, Bb, QP, 1e-14)
    out = lib.predict_wavefunction(full["ctx"], [dict(leg_a=Aa, leg_beta=Bt, leg_b=Bb, lam_i=T(la),
                                                      V_i=T(layout.V_to_flat(V, Bt, QP, Aa)), lam_prev=T(lt),
                                                      U_ip1=T(layout.U_to_flat(U, Bt, QP, Bb)), lam_ip1=T(lb))],
                                   QP, 1e-14)[0]
    ref_flat = layout.psi_to_flat(ref, Aa, Bb, QP)
    err = rel_err(H(out), ref_flat)
    print(f"[fullsize] {full['key']} predict: N = {len(ref_flat)}, max rel err {err:.2e}", flush=True)
    assert err <= 1e-13


def _oracle_ground_energy(full):
    """The oracle Lanczos energy of the operator: live for the smallest operator, else the value
    stored by tests/golden/make_fullsize_energies.py from the same construction."""
    if full["N"] <= 1_000_000:
        return lanczos(full["mv"], workloads.gaussian(full["N"], 80), 1e-12, 1e-8, 300)["energy"]
    from golden.make_fullsize_energies import load
    rec = load()[full["key"]]
    assert rec["N"] == full["N"]
    return rec["energy"]


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
    assert infos[0]["converged"] and res_orc <= 1e-8 * 1.01
    # the ground state, not an excited eigenpair: the oracle's own Lanczos energy of this operator
    e0 = _oracle_ground_energy(full)
    print(f"[fullsize] {full['key']} lanczos {prec}: E = {es[0]!r}, oracle E0 = {e0!r}, "
          f"|dE| = {abs(es[0] - e0):.2e}, {infos[0]['iters']} iterations", flush=True)
    assert abs(es[0] - e0) <= 1e-12
