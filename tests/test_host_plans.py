"""Host-side checks of the library (CPU only, no GPU needed).

* libidmrg.so loads and exports every symbol that include/idmrg.h declares;
* the flat-layout size functions agree with the oracle's reading of the
  storage order;
* the work plans of heff_apply and update_env, executed by a plain host
  interpreter (tests/hostplan/plan_exec.cpp, built here with g++), reproduce
  the oracle's contractions.  This checks every block offset and every MPO
  mixing coefficient of the plans without a GPU.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import workloads
from oracle import layout, mpo as omp, u1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
QP = [1, -1]


@pytest.fixture(scope="module")
def lib():
    from paper_1606_06790_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libidmrg.so not built")
    return L


def test_exports_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "idmrg.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(\w+)\(", hdr, re.M))
    assert {"heff_apply", "lanczos_solve_batch", "truncate_twosite", "update_env", "predict_wavefunction"} <= names
    L = C.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert names == set(lib.EXPORTS)


def test_layout_sizes(lib):
    A = [(-5, 3), (-3, 11), (-1, 20), (1, 17), (3, 9)]
    B = [(-3, 7), (-1, 19), (1, 21), (3, 4), (5, 2)]
    Cl = [(-2, 12), (0, 30), (2, 9)]
    cfg = workloads.workload("yc8")
    _, dq = omp.build_mpo(cfg["ell"], cfg["bonds"])
    for d in dq:
        assert lib.envL_size(A, list(d)) == layout.envL_size(A, d)
        assert lib.envR_size(B, list(d)) == layout.envR_size(B, d)
    assert lib.psi_size(A, B, QP) == layout.psi_size(A, B, QP)
    assert lib.U_size(A, QP, Cl) == sum(sum(r[2] for r in layout.U_rows(A, QP, q)) * k for q, k in Cl)
    assert lib.V_size(B, QP, Cl) == sum(sum(r[2] for r in layout.V_rows(B, QP, q)) * k for q, k in Cl)


@pytest.fixture(scope="module")
def hostplan(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hostplan") / "libhostplan.so")
    src = os.path.join(ROOT, "tests", "hostplan", "plan_exec.cpp")
    plan = os.path.join(ROOT, "paper_1606_06790_amd", "csrc", "plan.cpp")
    cmd = ["g++", "-O2", "-shared", "-fPIC", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1606_06790_amd", "csrc"),
           src, plan, "-o", out]
    try:
        subprocess.check_call(cmd)
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("g++ or HIP headers unavailable")
    return C.CDLL(out)


def _mpo_pair(name, c1):
    from paper_1606_06790_amd.lib import Mpo
    cfg = workloads.workload(name)
    Ws, dq = omp.build_mpo(cfg["ell"], cfg["bonds"])
    ell = cfg["ell"]
    f = lambda k: (k - 1) % ell + 1
    W1, W2 = Ws[f(c1) - 1], Ws[f(c1 + 1) - 1]
    dl, dm, dr = dq[f(c1) - 1], dq[f(c1)], dq[f(c1 + 1)]
    return (W1, W2, dl, dm, dr), (Mpo(W1, dl, dm, QP), Mpo(W2, dm, dr, QP))


LEGS = [([(-1, 3), (1, 2)], [(-1, 2), (1, 3)]),
        ([(-3, 5), (-1, 9), (1, 8), (3, 2)], [(-3, 3), (-1, 7), (1, 10), (3, 4)]),
        ([(-5, 1), (-3, 6), (-1, 7), (1, 9), (3, 4), (5, 2)], [(-5, 2), (-3, 5), (-1, 8), (1, 6), (3, 3), (5, 1)]),
        # several 16-row and 32-k fragments per block, with ragged edges
        ([(-3, 23), (-1, 37), (1, 41), (3, 19)], [(-3, 17), (-1, 45), (1, 33), (3, 21)])]


@pytest.mark.parametrize("name,c1", [("chain", 1), ("yc4", 3), ("yc8", 4), ("yc8", 9), ("dimer", 2)])
@pytest.mark.parametrize("li", [0, 1, 2, 3])
def test_heff_plan_on_host(lib, hostplan, name, c1, li):
    (W1, W2, dl, dm, dr), (M1, M2) = _mpo_pair(name, c1)
    A, B = LEGS[li]
    nL, nR, nx = layout.envL_size(A, dl), layout.envR_size(B, dr), layout.psi_size(A, B, QP)
    Lf, Rf, x = workloads.gaussian(nL, 60, li, 1), workloads.gaussian(nR, 60, li, 2), workloads.gaussian(nx, 60, li, 3)
    ref = layout.psi_to_flat(u1.heff_apply(layout.flat_to_envL(Lf, A, dl), W1, W2, layout.flat_to_envR(Rf, B, dr),
                                           layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr), A, B, QP)
    k = lib._Keep()
    h = lib.Heff_t(k.leg(A), k.leg(B), k.mpo(M1), k.mpo(M2), C.c_void_p(Lf.ctypes.data), C.c_void_p(Rf.ctypes.data))
    y = np.full(nx, np.nan)
    assert hostplan.hostplan_heff(C.byref(h), C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data)) == 0
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # the split-bf16 form of the plan (fragment-layout operands), executed in FP64, with the H_L / H_R
    # diagonals of the packed environments shifted and the shift added back
    y = np.full(nx, np.nan)
    flags = (C.c_int * 2)()
    assert hostplan.hostplan_heff_frag(C.byref(h), C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data),
                                       C.c_double(1.75), C.c_double(-2.5), flags) == 0
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # every MPO here (finite-state Heisenberg form) has the structure, so the shift path is exercised
    assert flags[0] == 1 and flags[1] == 1, list(flags)


@pytest.mark.parametrize("name,c1", [("chain", 2), ("yc8", 4), ("dimer", 1)])
@pytest.mark.parametrize("side", ["left", "right"])
def test_env_plan_on_host(lib, hostplan, name, c1, side):
    (W1, W2, dl, dm, dr), (M1, M2) = _mpo_pair(name, c1)
    A, B = LEGS[2]
    Cl = [(-4, 2), (-2, 5), (0, 7), (2, 4), (4, 1)]
    if side == "left":
        n_iso = sum(sum(r[2] for r in layout.U_rows(A, QP, q)) * kk for q, kk in Cl)
        Ef, If = workloads.gaussian(layout.envL_size(A, dl), 61, 1), workloads.gaussian(n_iso, 61, 2)
        ref = layout.envL_to_flat(u1.update_env_left(layout.flat_to_envL(Ef, A, dl), W1,
                                                     layout.flat_to_U(If, A, QP, Cl), A, QP, Cl, dl, dm), Cl, dm)
        old, W, sd = A, M1, 0
    else:
        n_iso = sum(sum(r[2] for r in layout.V_rows(B, QP, q)) * kk for q, kk in Cl)
        Ef, If = workloads.gaussian(layout.envR_size(B, dr), 62, 1), workloads.gaussian(n_iso, 62, 2)
        ref = layout.envR_to_flat(u1.update_env_right(layout.flat_to_envR(Ef, B, dr), W2,
                                                      layout.flat_to_V(If, B, QP, Cl), B, QP, Cl, dm, dr), Cl, dm)
        old, W, sd = B, M2, 1
    k = lib._Keep()
    out = np.full(len(ref), np.nan)
    u = lib.EnvUpdate_t(k.leg(old), k.leg(Cl), k.mpo(W), C.c_void_p(Ef.ctypes.data), C.c_void_p(If.ctypes.data),
                        C.c_void_p(out.ctypes.data))
    assert hostplan.hostplan_env(sd, C.byref(u)) == 0
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


# ---- the uniform MPS (Eq. (11)): a two-site piece as the fused site's isometries, and environment overlaps

A_OBS = [(-3, 4), (-1, 7), (1, 6), (3, 2)]
B_OBS = [(-3, 3), (-1, 6), (1, 8), (3, 3)]


def test_twosite_V_plan_on_host(lib, hostplan):
    x = workloads.gaussian(layout.psi_size(A_OBS, B_OBS, QP), 63, 1)
    psi = layout.flat_to_psi(x, A_OBS, B_OBS, QP)
    V = {}
    for (qa, s1, s2), blk in psi.items():
        V[(2 * s1 + s2, qa + QP[s1] + QP[s2], qa)] = blk.T
    qf = lib.fused_qp(QP)
    ref = layout.V_to_flat(V, B_OBS, qf, A_OBS)
    out = np.full(len(ref), np.nan)
    k = lib._Keep()
    assert hostplan.hostplan_twosite_V(C.byref(k.leg(A_OBS)), C.byref(k.leg(B_OBS)), 2, k.ints(QP),
                                       C.c_void_p(x.ctypes.data), C.c_void_p(out.ctypes.data)) == 0
    assert np.array_equal(out, ref)


def test_overlap_plan_on_host(lib, hostplan):
    leg = [(-2, 3), (0, 5), (2, 4), (4, 2)]
    ql, qr = [0, 2, 0, 0], [0, 2, 0, 0]
    Lf, Rf = workloads.gaussian(layout.envL_size(leg, ql), 64, 1), workloads.gaussian(layout.envR_size(leg, qr), 64, 2)
    L, R = layout.flat_to_envL(Lf, leg, ql), layout.flat_to_envR(Rf, leg, qr)
    k = lib._Keep()
    for wl, wr in ((0, 2), (1, 1), (2, 3)):
        ref = sum(float(np.sum(b * R[(wr, qa, qa2)])) for (w, qa, qa2), b in L.items()
                  if w == wl and (wr, qa, qa2) in R)
        it = lib.Overlap_t(k.leg(leg), 4, k.ints(ql), C.c_void_p(Lf.ctypes.data), 4, k.ints(qr),
                           C.c_void_p(Rf.ctypes.data), wl, wr)
        out = C.c_double()
        assert hostplan.hostplan_overlap(C.byref(it), C.byref(out)) == 0
        assert abs(out.value - ref) <= 1e-13 * max(1.0, abs(ref))
    it = lib.Overlap_t(k.leg(leg), 4, k.ints(ql), C.c_void_p(Lf.ctypes.data), 4, k.ints(qr),
                       C.c_void_p(Rf.ctypes.data), 1, 2)
    assert hostplan.hostplan_overlap(C.byref(it), C.byref(C.c_double())) == -1    # channel charges differ


def _dense(blocks, rows_leg, cols_leg, key):
    """Dense matrix of the blocks blocks[key(qa, qb)] over two legs (sectors in order)."""
    ro, co = {}, {}
    off = 0
    for q, k in rows_leg:
        ro[q] = off
        off += k
    M = np.zeros((off, sum(k for _, k in cols_leg)))
    off = 0
    for q, k in cols_leg:
        co[q] = off
        off += k
    for qa, da in rows_leg:
        for qb, db in cols_leg:
            b = blocks.get(key(qa, qb))
            if b is not None:
                M[ro[qa]:ro[qa] + da, co[qb]:co[qb] + db] = b
    return M


@pytest.mark.parametrize("ops", [("1", "1"), ("+", "1"), ("1", "-"), ("z", "z")])
def test_fused_piece_transfer_on_host(lib, hostplan, ops):
    """update_env(LEFT)'s plan with the piece as the fused site's left isometry and the observables' three-channel
    MPO equals the oracle's piece transfer with the operators inserted (channel 1) and without (channel 0)."""
    from oracle import observables as ob
    from paper_1606_06790_amd.observables import fused_mpo
    x = workloads.gaussian(layout.psi_size(A_OBS, B_OBS, QP), 65, 1)
    psi = layout.flat_to_psi(x, A_OBS, B_OBS, QP)
    W = fused_mpo(ops[0], ops[1], 0, lib.LEFT, QP)
    # L: channels 0 and 1 the same charge-0 block-diagonal matrix
    X = {(w, q, q): np.asarray(workloads.gaussian(d * d, 65, 2, q + 100).reshape(d, d)) for q, d in A_OBS
         for w in (0, 1)}
    Lf = layout.envL_to_flat(X, A_OBS, W.ql)
    out = np.full(layout.envL_size(B_OBS, W.qr), np.nan)
    k = lib._Keep()
    u = lib.EnvUpdate_t(k.leg(A_OBS), k.leg(B_OBS), k.mpo(W), C.c_void_p(Lf.ctypes.data), C.c_void_p(x.ctypes.data),
                        C.c_void_p(out.ctypes.data))
    assert hostplan.hostplan_env(0, C.byref(u)) == 0
    Lnew = layout.flat_to_envL(out, B_OBS, W.qr)
    # oracle: dense piece and dense X
    ma, mb = sum(d for _, d in A_OBS), sum(d for _, d in B_OBS)
    Bd = np.zeros((ma, 2, 2, mb))
    ao, bo = {}, {}
    o = 0
    for q, d in A_OBS:
        ao[q] = o
        o += d
    o = 0
    for q, d in B_OBS:
        bo[q] = o
        o += d
    for (qa, s1, s2), blk in psi.items():
        qb = qa + QP[s1] + QP[s2]
        Bd[ao[qa]:ao[qa] + blk.shape[0], s1, s2, bo[qb]:bo[qb] + blk.shape[1]] = blk
    Xd = _dense({(q, q): X[(0, q, q)] for q, _ in A_OBS}, A_OBS, A_OBS, lambda a, b: (a, b))
    opm = {"1": None, "+": ob.SP, "-": ob.SM, "z": ob.SZ}
    for ch, (o1, o2) in ((0, (None, None)), (1, (opm[ops[0]], opm[ops[1]]))):
        ref = ob.apply_piece(Xd, Bd, o1, o2)
        got = _dense({(qa, qb): v for (w, qa, qb), v in Lnew.items() if w == ch}, B_OBS, B_OBS, lambda a, b: (a, b))
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), ch


def test_fused_piece_right_transfer_on_host(lib, hostplan):
    """update_env(RIGHT)'s plan with the piece rewritten as the fused site's right isometry (twosite plan) and the
    observables' right MPO equals the right transfer Y'[a, a'] = sum B[a,s,t,b] Y[b,b'] B[a',s,t,b'] in channels 1, 2."""
    from paper_1606_06790_amd.observables import fused_mpo
    x = workloads.gaussian(layout.psi_size(A_OBS, B_OBS, QP), 66, 1)
    qf = lib.fused_qp(QP)
    Vf = np.full(sum(sum(r[2] for r in layout.V_rows(B_OBS, qf, q)) * d for q, d in A_OBS), np.nan)
    k = lib._Keep()
    assert hostplan.hostplan_twosite_V(C.byref(k.leg(A_OBS)), C.byref(k.leg(B_OBS)), 2, k.ints(QP),
                                       C.c_void_p(x.ctypes.data), C.c_void_p(Vf.ctypes.data)) == 0
    W = fused_mpo("1", "1", 0, lib.RIGHT, QP)
    Y = {(w, q, q): np.asarray(workloads.gaussian(d * d, 66, 2, q + 100).reshape(d, d)) for q, d in B_OBS
         for w in (1, 2)}
    Rf = layout.envR_to_flat(Y, B_OBS, W.qr)
    out = np.full(layout.envR_size(A_OBS, W.ql), np.nan)
    u = lib.EnvUpdate_t(k.leg(B_OBS), k.leg(A_OBS), k.mpo(W), C.c_void_p(Rf.ctypes.data), C.c_void_p(Vf.ctypes.data),
                        C.c_void_p(out.ctypes.data))
    assert hostplan.hostplan_env(1, C.byref(u)) == 0
    Rnew = layout.flat_to_envR(out, A_OBS, W.ql)
    psi = layout.flat_to_psi(x, A_OBS, B_OBS, QP)
    ma, mb = sum(d for _, d in A_OBS), sum(d for _, d in B_OBS)
    ao, bo, o = {}, {}, 0
    for q, d in A_OBS:
        ao[q], o = o, o + d
    o = 0
    for q, d in B_OBS:
        bo[q], o = o, o + d
    Bd = np.zeros((ma, 2, 2, mb))
    for (qa, s1, s2), blk in psi.items():
        qb = qa + QP[s1] + QP[s2]
        Bd[ao[qa]:ao[qa] + blk.shape[0], s1, s2, bo[qb]:bo[qb] + blk.shape[1]] = blk
    Yd = _dense({(q, q): Y[(2, q, q)] for q, _ in B_OBS}, B_OBS, B_OBS, lambda a, b: (a, b))
    ref = np.einsum("astb,bB,AstB->aA", Bd, Yd, Bd)
    for ch in (1, 2):
        got = _dense({(qa, qb): v for (w, qa, qb), v in Rnew.items() if w == ch}, A_OBS, A_OBS, lambda a, b: (a, b))
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), ch


@pytest.mark.parametrize("stage", [1, 2])
def test_gemm_xcd_ranges(lib, hostplan, stage):
    """The per-XCD tile ranges after a GEMM task table cover every tile once, in order, and split the work (K + 64 per
    tile) so that no XCD's share exceeds the mean by more than one tile: three YC8 superblocks on the legs of the
    host tests, in the split-bf16 plan."""
    k = lib._Keep()
    hs = []
    for li, c1 in ((3, 4), (2, 9), (3, 7)):
        (_, _, _, _, _), (M1, M2) = _mpo_pair("yc8", c1)
        A, B = LEGS[li]
        hs.append(lib.Heff_t(k.leg(A), k.leg(B), k.mpo(M1), k.mpo(M2), None, None))
    arr = (lib.Heff_t * len(hs))(*hs)
    out = (C.c_double * 19)()
    assert hostplan.hostplan_xcd_ranges(arr, len(hs), stage, out) == 0
    s = [int(v) for v in out[:9]]
    xmax, tiles = int(out[9]), int(out[10])
    work = list(out[11:19])
    assert s[0] == 0 and s[8] == tiles and all(a <= b for a, b in zip(s, s[1:]))
    assert xmax == max(b - a for a, b in zip(s, s[1:]))
    mean = sum(work) / 8
    assert max(work) <= mean + 1.0 + 1e-9
