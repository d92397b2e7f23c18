"""Observables of the uniform MPS (Eq. (11); Sec. 4) on the GPU against the oracle (needs an MI355X).

* twosite_to_right_iso is an exact permutation: compared element by element with the oracle's layouts read by
  hand (every block of the two-site state transposed into the fused site's V layout).
* env_overlap against the blockwise sum of products of the oracle's environment dictionaries.
* UniformMPS: the library's pieces, fixed points and operator chains against oracle.observables on the same
  decompositions (the driver's last iteration, copied to the host and laid out densely), for the Heisenberg
  chain and the YC8 kagome cylinder at small m: bond strengths, the correlation function along the cylinder,
  and the Step 5' energy per site as the sum of the cell's bond energies.
"""
import numpy as np
import pytest

import workloads
from oracle import layout
from oracle import observables as ob

from gpu_common import QP, H, T

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")
torch = pytest.importorskip("torch")

A = [(-3, 20), (-1, 70), (1, 65), (3, 15)]
B = [(-3, 12), (-1, 67), (1, 80), (3, 30)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def test_twosite_to_right_iso_is_a_transpose(ctx):
    x = workloads.gaussian(layout.psi_size(A, B, QP), 70, 1)
    out = lib.twosite_to_right_iso(ctx, [dict(left=A, right=B, psi=T(x))], QP)[0]
    psi = layout.flat_to_psi(x, A, B, QP)
    qf = lib.fused_qp(QP)
    V = {}
    for (qa, s1, s2), blk in psi.items():
        qb = qa + QP[s1] + QP[s2]
        V[(2 * s1 + s2, qb, qa)] = blk.T
    ref = layout.V_to_flat(V, B, qf, A)
    assert np.array_equal(H(out), ref)


def test_env_overlap(ctx):
    leg = [(-2, 7), (0, 11), (2, 5), (4, 3)]
    ql = [0, 2, 0, 0]              # L channels 0..2 stored, 3 the identity
    qr = [0, 2, 0, 0]              # R channels 1..3 stored, 0 the identity
    Lf = workloads.gaussian(layout.envL_size(leg, ql), 71, 1)
    Rf = workloads.gaussian(layout.envR_size(leg, qr), 71, 2)
    L = layout.flat_to_envL(Lf, leg, ql)
    R = layout.flat_to_envR(Rf, leg, qr)
    items, ref = [], []
    for wl, wr in ((0, 2), (1, 1), (2, 3), (0, 3)):
        s = 0.0
        for (w, qa, qa2), blk in L.items():
            if w == wl and (wr, qa, qa2) in R:
                s += float(np.sum(blk * R[(wr, qa, qa2)]))
        ref.append(s)
        items.append(dict(leg=leg, ql=ql, L=T(Lf), qr=qr, R=T(Rf), wl=wl, wr=wr))
    out = lib.env_overlap(ctx, items)
    for a, b in zip(out, ref):
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b))
    with pytest.raises(lib.IdmrgError):
        lib.env_overlap(ctx, [dict(leg=leg, ql=ql, L=T(Lf), qr=qr, R=T(Rf), wl=1, wr=2)])   # charges differ


def _dense_leg(leg):
    """{charge: (offset, dim)} of a leg laid out densely in sector order."""
    out, off = {}, 0
    for q, k in leg:
        out[q] = (off, k)
        off += k
    return out, off


def _dense_decomposition(tr, A_leg, B_leg, C_leg):
    """U[a,s,c], V[s,b,c], lam[c] of a library truncation (legs A, B of the two-site state, kept leg C), densely."""
    dA, mA = _dense_leg(A_leg)
    dB, mB = _dense_leg(B_leg)
    dC, mC = _dense_leg(C_leg)
    U = np.zeros((mA, 2, mC))
    V = np.zeros((2, mB, mC))
    for (qa, s, qc), blk in layout.flat_to_U(H(tr["U"]), A_leg, QP, C_leg).items():
        U[dA[qa][0]:dA[qa][0] + dA[qa][1], s, dC[qc][0]:dC[qc][0] + dC[qc][1]] = blk
    for (s, qb, qc), blk in layout.flat_to_V(H(tr["V"]), B_leg, QP, C_leg).items():
        V[s, dB[qb][0]:dB[qb][0] + dB[qb][1], dC[qc][0]:dC[qc][0] + dC[qc][1]] = blk
    return dict(U=U, V=V, lam=H(tr["lam"]))


def _oracle_cell(d):
    """The oracle's Eq. (11) pieces from the driver's last two iterations (host copies, dense)."""
    half = d.half
    cur, prev_lam = {}, {}
    for i in range(1, half + 1):
        # superblock i at iteration n: left leg = kept leg of superblock i at n-1, right leg = that of i+1
        ip1 = i % half + 1
        A_leg, B_leg = d.lam2[i][0], d.lam2[ip1][0]
        cur[i] = _dense_decomposition(d.prev[i], A_leg, B_leg, d.prev[i]["C"])
        prev_lam[i] = H(d.lam2[i][1])
    return ob.pieces(cur, prev_lam, d.cfg["lam_floor"])


@pytest.mark.parametrize("name, m, n", [("chain", 16, 39), ("yc8", 24, 23)])
def test_uniform_mps_matches_oracle(ctx, name, m, n):
    from paper_1606_06790_amd.driver import IDMRG
    from paper_1606_06790_amd.observables import UniformMPS
    cfg = workloads.workload(name, m=m)
    d = IDMRG(cfg, prec="f64")
    d.run(n)
    u = UniformMPS(d)
    Bs = _oracle_cell(d)
    fp = ob.fixed_points(Bs)
    assert abs(u.fixed_points() - fp[0]) <= 1e-11 * abs(fp[0])
    pairs = [(i, j) for (i, j, _) in cfg["bonds"]]
    got = u.bond_strengths(pairs)
    ref = ob.bond_strengths(Bs, n, cfg["ell"], pairs, fp)
    err = max(abs(got[k] - ref[k]) for k in pairs)
    print(f"[observables] {name} m={m}: {len(pairs)} bonds, max |GPU - oracle| {err:.2e}, "
          f"cells to converge L/R {u.cells_L}/{u.cells_R}")
    assert err <= 1e-10
    # the cell's bond energies add up to the Step 5' energy per site (the same invariant as the oracle's pin)
    e_mps = sum(J * got[(i, j)] for (i, j, J) in cfg["bonds"]) / cfg["ell"]
    e_g = d.e_g[max(d.e_g)]
    print(f"[observables] {name}: energy per site from bonds {e_mps:.8f}, Step 5' e_g {e_g:.8f}")
    assert abs(e_mps - e_g) < (5e-5 if name == "chain" else 5e-3)
    # correlation function along the axis
    label = 2
    corr = u.correlation_function(label, 4)
    a = ob.position(label, n + 2, cfg["ell"])
    ref_c = [ob.spin_correlation(Bs, a, a + cfg["ell"] * r, fp) for r in range(1, 5)]
    for x, y in zip(corr, ref_c):
        assert abs(x - y) <= 1e-10 * max(1.0, abs(y)) + 1e-13
    if name == "yc8":
        # the sweep along the cylinder's axis: pairs of different labels several cells apart
        sweep = workloads.yc8_axis_sweep(3, label)
        got_ax = u.correlations([(a, a + s - label) for s, _ in sweep[1:]])
        for (s, _), x in zip(sweep[1:], got_ax):
            y = ob.spin_correlation(Bs, a, a + s - label, fp)
            assert abs(x - y) <= 1e-10 * max(1.0, abs(y)) + 1e-13, (s, x, y)
