"""GPU parity of the five C-ABI calls against the FP64 oracle (needs an MI355X).

Every call is fed the same seeded inputs as the oracle.  FP64 results must
agree elementwise to 1e-13 relative to the largest output magnitude (the
rounding of FP64 sums of at most a few thousand terms), energies to 1e-12,
trajectories (per-site energies) to 1e-10.
"""
import numpy as np
import pytest

import workloads
from oracle import dense as odense
from oracle import idmrg as oidmrg
from oracle import layout, u1

from gpu_common import QP, H, T, mpo_pair, rel_err

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


LEGS = {
    "small": ([(-1, 3), (1, 2)], [(-1, 2), (1, 3)]),
    "ragged": ([(-3, 20), (-1, 70), (1, 65), (3, 15)], [(-3, 12), (-1, 67), (1, 80), (3, 30)]),
    "wide": ([(-5, 8), (-3, 33), (-1, 66), (1, 70), (3, 40), (5, 9)],
             [(-5, 5), (-3, 41), (-1, 72), (1, 61), (3, 30), (5, 11)]),
    # sectors of several 256-row tiles and up to 14 K-slabs of 32, none a multiple of a tile
    "big": ([(-3, 150), (-1, 421), (1, 389), (3, 131)], [(-3, 141), (-1, 397), (1, 410), (3, 127)]),
}


def _heff_case(name, legs, key):
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair(name, 4)
    A, B = LEGS[legs]
    nL, nR, nx = layout.envL_size(A, dl), layout.envR_size(B, dr), layout.psi_size(A, B, QP)
    Lf, Rf, x = workloads.gaussian(nL, key, 1), workloads.gaussian(nR, key, 2), workloads.gaussian(nx, key, 3)
    y = layout.psi_to_flat(u1.heff_apply(layout.flat_to_envL(Lf, A, dl), W1, W2, layout.flat_to_envR(Rf, B, dr),
                                         layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr), A, B, QP)
    prob = dict(left=A, right=B, w1=M1, w2=M2, L=T(Lf), R=T(Rf))
    return prob, x, y


def test_heff_apply_batched_u1(ctx):
    cases = [_heff_case("chain", "small", 11), _heff_case("chain", "ragged", 12), _heff_case("yc8", "wide", 13),
             _heff_case("yc4", "ragged", 14)]
    probs = [c[0] for c in cases]
    xs = [T(c[1]) for c in cases]
    ys = [T(np.full(len(c[2]), np.nan)) for c in cases]
    lib.heff_apply(ctx, probs, xs, ys, "f64")
    for (p, x, y), yg in zip(cases, ys):
        assert rel_err(H(yg), y) <= 1e-13


@pytest.mark.parametrize("m", [40, 96, 256])
def test_heff_apply_dense(ctx, m):
    """No symmetry blocks (all charges 0): one block per (s1, s2)."""
    from paper_1606_06790_amd.lib import Mpo
    (W1, W2, dl, dm, dr), _ = mpo_pair("chain", 1)
    D = W1.shape[0]
    z = lambda k: [0] * k
    M1, M2 = Mpo(W1, z(D), z(D), [0, 0]), Mpo(W2, z(D), z(D), [0, 0])
    Lf = workloads.gaussian((D - 1) * m * m, 20, m, 1)
    Rf = workloads.gaussian(m * (D - 1) * m, 20, m, 2)
    x = workloads.gaussian(4 * m * m, 20, m, 3)
    L = np.zeros((m, D, m))
    L[:, :D - 1, :] = Lf.reshape(D - 1, m, m).transpose(1, 0, 2)
    L[:, D - 1, :] = np.eye(m)
    R = np.zeros((m, D, m))
    R[:, 1:, :] = Rf.reshape(m, D - 1, m)
    R[:, 0, :] = np.eye(m)
    y = odense.psi_to_flat(odense.heff_apply(L, W1, W2, R, odense.psi_from_flat(x, m, 2, m)))
    yg = T(np.zeros(4 * m * m))
    lib.heff_apply(ctx, [dict(left=[(0, m)], right=[(0, m)], w1=M1, w2=M2, L=T(Lf), R=T(Rf))], [T(x)], [yg], "f64")
    assert rel_err(H(yg), y) <= 1e-13


def _iso_size(rows_fn, leg, Cl):
    return sum(sum(r[2] for r in rows_fn(leg, QP, q)) * k for q, k in Cl)


@pytest.mark.parametrize("side", ["left", "right"])
def test_update_env(ctx, side):
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair("yc8", 3)
    A = LEGS["wide"][0]
    Cl = [(-4, 17), (-2, 60), (0, 90), (2, 55), (4, 21)]
    if side == "left":
        Lf = workloads.gaussian(layout.envL_size(A, dl), 30, 1)
        Uf = workloads.gaussian(_iso_size(layout.U_rows, A, Cl), 30, 2)
        L = layout.flat_to_envL(Lf, A, dl)
        U = layout.flat_to_U(Uf, A, QP, Cl)
        ref = u1.update_env_left(L, W1, U, A, QP, Cl, dl, dm)
        out = lib.update_env(ctx, lib.LEFT, [dict(old_leg=A, new_leg=Cl, w=M1, env_old=T(Lf), iso=T(Uf))])[0]
        ref_flat = layout.envL_to_flat(ref, Cl, dm)
    else:
        B = LEGS["wide"][1]
        Rf = workloads.gaussian(layout.envR_size(B, dr), 31, 1)
        Vf = workloads.gaussian(_iso_size(layout.V_rows, B, Cl), 31, 2)
        R = layout.flat_to_envR(Rf, B, dr)
        V = layout.flat_to_V(Vf, B, QP, Cl)
        ref = u1.update_env_right(R, W2, V, B, QP, Cl, dm, dr)
        out = lib.update_env(ctx, lib.RIGHT, [dict(old_leg=B, new_leg=Cl, w=M2, env_old=T(Rf), iso=T(Vf))])[0]
        ref_flat = layout.envR_to_flat(ref, Cl, dm)
    assert rel_err(H(out), ref_flat) <= 1e-13


def test_predict_wavefunction(ctx):
    Aa = [(-2, 30), (0, 70), (2, 33)]
    Bt = [(-3, 20), (-1, 66), (1, 64), (3, 18)]
    Bb = [(-2, 25), (0, 81), (2, 28)]
    Vf = workloads.gaussian(_iso_size(layout.V_rows, Bt, Aa), 40, 1)
    Uf = workloads.gaussian(_iso_size(layout.U_rows, Bt, Bb), 40, 2)
    la = np.abs(workloads.gaussian(sum(k for _, k in Aa), 40, 3))
    lt = np.abs(workloads.gaussian(sum(k for _, k in Bt), 40, 4))
    lt[::7] = 0.0                       # zero Schmidt values take the 0 branch of Eq. (10)
    lb = np.abs(workloads.gaussian(sum(k for _, k in Bb), 40, 5))
    ref = u1.predict_wavefunction(layout.flat_to_lam(la, Aa), layout.flat_to_V(Vf, Bt, QP, Aa),
                                  layout.flat_to_lam(lt, Bt), layout.flat_to_U(Uf, Bt, QP, Bb),
                                  layout.flat_to_lam(lb, Bb), Aa, Bb, QP, 1e-14)
    out = lib.predict_wavefunction(ctx, [dict(leg_a=Aa, leg_beta=Bt, leg_b=Bb, lam_i=T(la), V_i=T(Vf), lam_prev=T(lt),
                                              U_ip1=T(Uf), lam_ip1=T(lb))], QP, 1e-14)[0]
    assert rel_err(H(out), layout.psi_to_flat(ref, Aa, Bb, QP)) <= 1e-13


def _oracle_states(name, m, n_max, **over):
    cfg = workloads.workload(name, m=m, **over)
    return cfg, oidmrg.run(cfg, mode="u1", n_max=n_max, keep_states=True)


def test_truncate_twosite(ctx):
    """Singular values, kept legs, eps and eps' equal the oracle's; the kept
    subspaces agree (projectors) and the isometries are orthonormal."""
    cfg, r = _oracle_states("random_chain", 24, 7)
    sts = [st for st in r["states"] if st["n"] in (3, 5, 6, 7)][:8]
    items = [dict(left=st["A"], right=st["B"], psi=T(st["psi"])) for st in sts]
    out = lib.truncate_twosite(ctx, items, QP, cfg["m"], cfg["lam_floor"], cfg["deg_rel"])
    for st, o in zip(sts, out):
        tr = st["tr"]
        assert o["C"] == tr["C"]
        assert o["m_kept"] == tr["m_kept"]
        assert abs(o["eps"] - tr["eps"]) <= 1e-14 + 1e-10 * tr["eps"]
        assert abs(o["eps_prime"] - tr["eps_prime"]) <= 1e-14 + 1e-10 * tr["eps_prime"]
        lam = layout.flat_to_lam(H(o["lam"]), o["C"])
        for q, _ in o["C"]:
            assert np.abs(lam[q] - tr["lam"][q]).max() <= 1e-13
        U = layout.flat_to_U(H(o["U"]), st["A"], QP, o["C"])
        V = layout.flat_to_V(H(o["V"]), st["B"], QP, o["C"])
        for q, k in o["C"]:
            rows = layout.U_rows(st["A"], QP, q)
            Ug = np.concatenate([U[(a, s, q)] for (a, s, _) in rows])
            Uo = np.concatenate([tr["U"][(a, s, q)] for (a, s, _) in rows])
            assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-13
            if tr["cut_gap"] is None or tr["cut_gap"] > 1e-6:
                assert np.abs(Ug @ Ug.T - Uo @ Uo.T).max() <= 1e-10
            vrows = layout.V_rows(st["B"], QP, q)
            Vg = np.concatenate([V[(s, b, q)] for (s, b, _) in vrows])
            assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-13


def _graded_psi(seed, ns=9):
    """Two-site state of ns+ns spins (legs C(ns,k)) whose centre blocks have low
    rank k (values in [1e-3, 1]) and only k nonzero columns (as when the right
    leg carries zero-weight states): each block is U diag(sigma) V^T with U
    dense and V supported on k random columns.  The one-sided Jacobi iteration then has many more rows
    than the dimension of their span, and the surplus rows decay to rounding
    residue instead of reaching zero."""
    from math import comb
    A = [(2 * k - ns, comb(ns, k)) for k in range(ns + 1)]
    B = list(A)
    psi = {}
    for q, (rows, cols) in u1.center_sectors(A, B, QP).items():
        r, c = sum(x[2] for x in rows), sum(x[2] for x in cols)
        g = np.random.default_rng([seed, q + 100])
        k = max(1, min(r, c) // 4)
        Ur = np.linalg.qr(g.standard_normal((r, k)))[0]
        Vr = np.zeros((c, k))
        Vr[np.sort(g.choice(c, k, replace=False))] = np.linalg.qr(g.standard_normal((k, k)))[0]
        sig = 10.0 ** g.uniform(-3, 0, k)
        M = (Ur * sig) @ Vr.T
        r0 = 0
        for (qa, s1, da) in rows:
            c0 = 0
            for (s2, qb, db) in cols:
                psi[(qa, s1, s2)] = M[r0:r0 + da, c0:c0 + db]
                c0 += db
            r0 += da
    x = layout.psi_to_flat(psi, A, B, QP)
    return A, B, x / np.linalg.norm(x)


def _check_graded(o, A, B, tr):
    assert o["svd_converged"] and o["warn"] == 0
    assert o["C"] == tr["C"] and o["m_kept"] == tr["m_kept"]
    assert abs(o["eps"] - tr["eps"]) <= 1e-14
    lam = layout.flat_to_lam(H(o["lam"]), o["C"])
    U = layout.flat_to_U(H(o["U"]), A, QP, o["C"])
    V = layout.flat_to_V(H(o["V"]), B, QP, o["C"])
    for q, k in o["C"]:
        assert np.abs(lam[q] - tr["lam"][q]).max() <= 1e-13
        Ug = np.concatenate([U[(a, s, q)] for (a, s, _) in layout.U_rows(A, QP, q)])
        Vg = np.concatenate([V[(s, b, q)] for (s, b, _) in layout.V_rows(B, QP, q)])
        assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-12
        assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-12
        real = lam[q] > 0
        Uo = np.concatenate([tr["U"][(a, s, q)] for (a, s, _) in layout.U_rows(A, QP, q)])[:, tr["lam"][q] > 0]
        assert np.abs(Ug[:, real] @ Ug[:, real].T - Uo @ Uo.T).max() <= 1e-10


def test_truncate_completion_per_problem(ctx):
    """One call, m = 64: the 9+9-spin state has 255 values above the floor and 1024
    candidates, so no zero-weight state is kept and its null rows are left uncompleted; the
    5+5-spin state has 64 candidates, all kept, fewer of them nonzero, so its zero-weight
    states are kept and completed.  Both must match the oracle and return isometries."""
    items, refs = [], []
    for seed, ns in ((11, 9), (13, 5)):
        A, B, x = _graded_psi(seed, ns)
        items.append(dict(left=A, right=B, psi=T(x)))
        refs.append((A, B, u1.truncate_twosite(layout.flat_to_psi(x, A, B, QP), A, B, QP, 64, 1e-14, 1e-5)))
    out = lib.truncate_twosite(ctx, items, QP, 64, 1e-14, 1e-5)
    assert [o["null_completed"] for o in out] == [False, True]
    assert refs[1][2]["m_kept"] > sum(1 for v in refs[1][2]["lam"].values() for l in v if l > 0)
    for (A, B, tr), o in zip(refs, out):
        _check_graded(o, A, B, tr)


def test_truncate_no_partial_null_space(ctx):
    """m = 512 lies between the ~255 nonzero values and the 1024 candidates of the graded
    9+9-spin state: only the nonzero values are kept (no arbitrary part of the null space),
    m_kept < m, exactly as in the oracle, and no completion is needed."""
    A, B, x = _graded_psi(11)
    tr = u1.truncate_twosite(layout.flat_to_psi(x, A, B, QP), A, B, QP, 512, 1e-14, 1e-5)
    o = lib.truncate_twosite(ctx, [dict(left=A, right=B, psi=T(x))], QP, 512, 1e-14, 1e-5)[0]
    npos = sum(1 for v in tr["lam"].values() for lam in v if lam > 0)
    assert tr["m_kept"] == npos < 512
    assert not o["null_completed"]
    _check_graded(o, A, B, tr)


def test_truncate_graded_spectrum(ctx):
    """Rows of the Jacobi iteration whose singular values are far below the
    floor have no reliable direction; the returned U and V must still be
    isometries, and the kept spectrum, kept legs and eps must equal the
    oracle's (regression: such rows once came back non-orthogonal).  m = 1024
    keeps every candidate, zero-weight states included, so the completion runs."""
    items, refs = [], []
    for seed in (11, 12):
        A, B, x = _graded_psi(seed)
        items.append(dict(left=A, right=B, psi=T(x)))
        refs.append((A, B, u1.truncate_twosite(layout.flat_to_psi(x, A, B, QP), A, B, QP, 1024, 1e-14, 1e-5)))
    out = lib.truncate_twosite(ctx, items, QP, 1024, 1e-14, 1e-5)
    for (A, B, tr), o in zip(refs, out):
        assert o["null_completed"]
        _check_graded(o, A, B, tr)


def _flat_problem(st):
    from paper_1606_06790_amd.lib import Mpo
    A, B = st["A"], st["B"]
    return dict(left=A, right=B, w1=Mpo(st["W1"], st["dl"], st["dm"], QP), w2=Mpo(st["W2"], st["dm"], st["dr"], QP),
                L=T(layout.envL_to_flat(st["L"], A, st["dl"])), R=T(layout.envR_to_flat(st["R"], B, st["dr"])))


def test_lanczos_solve_batch(ctx):
    """Same H, same start vector: energy within 1e-12, |<psi_gpu|psi_orc>| >= 1 - 1e-12."""
    cfg, r = _oracle_states("random_chain", 32, 7, tol_res=1e-10)
    sts = [st for st in r["states"] if st["n"] in (2, 6, 7)]
    probs = [_flat_problem(st) for st in sts]
    psis = [T(st["v0"]) for st in sts]
    es, infos = lib.lanczos_solve_batch(ctx, probs, psis, cfg["tol_E"], cfg["tol_res"], cfg["k_max"], "f64")
    steps = {(s["n"], s["i"]): s for s in r["steps"]}
    for st, e, inf, p in zip(sts, es, infos, psis):
        ref = steps[(st["n"], st["i"])]
        assert abs(e - ref["energy"]) <= 1e-12
        assert abs(abs(float(H(p) @ st["psi"])) - 1.0) <= 1e-12
        assert inf["converged"] == 1
        assert inf["residual"] <= 1e-8
        assert abs(inf["iters"] - ref["iters"]) <= 2
        assert abs((1 - inf["overlap0"]) - ref["fidelity"]) <= 1e-10


def _run_gpu(cfg, n_max, **kw):
    from paper_1606_06790_amd.driver import IDMRG
    d = IDMRG(cfg, **kw)
    d.run(n_max)
    return d


def test_trajectory_chain():
    """Uniform chain, l = 4, m = 32, 20 iterations: per-site energies and e_g of the
    GPU path equal the oracle's within 1e-10; untruncated steps equal ED."""
    cfg = workloads.workload("chain")
    g = _run_gpu(cfg, 20)
    o = oidmrg.run(cfg, mode="u1", n_max=20)
    for a, b in zip(g.steps, o["steps"]):
        assert (a["n"], a["i"]) == (b["n"], b["i"])
        assert abs(a["e_site"] - b["e_site"]) <= 1e-10, (a, b)
        assert a["m_kept"] == b["m_kept"]
    for n, e in o["e_g"].items():
        assert abs(g.e_g[n] - e) <= 1e-10
    assert abs(g.e_g[19] - workloads.bethe_ansatz_energy()) <= 5e-4


def test_trajectory_dimer():
    """Dimerised limit: exact energies -3(n+1)/4, exact prediction (fidelity error 0,
    one Lanczos step) on the GPU path too."""
    cfg = workloads.workload("dimer", m=8, n_max=8)
    g = _run_gpu(cfg, 8)
    for s in g.steps:
        assert abs(s["energy"] + 0.75 * (s["n"] + 1)) <= 1e-12
        if s["n"] >= 3:
            assert s["fidelity"] <= 1e-12 and s["iters"] == 1


def test_trajectory_random_chain():
    """Random-bond chain, l = 16 (8 superblocks per batched call), m = 48, 12 iterations."""
    cfg = workloads.workload("random_chain", m=48)
    g = _run_gpu(cfg, 12)
    o = oidmrg.run(cfg, mode="u1", n_max=12)
    for a, b in zip(g.steps, o["steps"]):
        assert abs(a["e_site"] - b["e_site"]) <= 1e-10, (a, b)
        assert a["m_kept"] == b["m_kept"]


def test_errors_are_reported(ctx):
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair("chain", 1)
    A, B = LEGS["small"]
    bad = dict(left=[(1, 2), (-1, 3)], right=B, w1=M1, w2=M2, L=T(np.zeros(100)), R=T(np.zeros(100)))
    with pytest.raises(lib.IdmrgError) as e:
        lib.heff_apply(ctx, [bad], [T(np.zeros(10))], [T(np.zeros(10))])
    assert e.value.code == lib.EINVAL
    # start vector of zero norm
    good = _heff_case("chain", "small", 50)[0]
    n = layout.psi_size(A, B, QP)
    with pytest.raises(lib.IdmrgError) as e:
        lib.lanczos_solve_batch(ctx, [good], [T(np.zeros(n))])
    assert e.value.code == lib.EINVAL
    # k_max = 2 cannot converge: a warning, with the best Ritz pair returned
    es, infos = lib.lanczos_solve_batch(ctx, [good], [T(workloads.gaussian(n, 50, 9))], k_max=2)
    assert infos[0]["warn"] == lib.WARN_NOCONV and infos[0]["iters"] == 2 and np.isfinite(es[0])


# ----------------------------------------------------------------- mixed precision

MIXED_TOL = {"f32": 5e-6, "bf16x3": 5e-5}   # max |y - y_64| / max |y_64| of one matvec


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_lanczos_repeatable_across_tuning(prec):
    """A fresh context tunes the GEMM tiling during its first solve (the first
    matvecs try every tile variant); the second solve uses the chosen variant
    throughout.  Tile shapes do not change the summation order, so both solves
    must agree bitwise."""
    c2 = lib.Context(0)
    cfg, r = _oracle_states("random_chain", 32, 7, tol_res=1e-10)
    # (split-bf16 tries six tilings, among them the eight-wave and the persistent kernels)
    sts = [st for st in r["states"] if st["n"] in (6, 7)]
    probs = [_flat_problem(st) for st in sts]
    runs = []
    for _ in range(2):
        psis = [T(st["v0"]) for st in sts]
        es, infos = lib.lanczos_solve_batch(c2, probs, psis, cfg["tol_E"], cfg["tol_res"], cfg["k_max"], prec)
        assert min(i["iters"] for i in infos) >= 5
        runs.append((es, [H(p) for p in psis]))
    assert runs[0][0] == runs[1][0]
    for a, b in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(a, b)


TILINGS = {"f64": range(4), "f32": range(4), "bf16x3": range(6)}


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_heff_apply_every_tiling(prec):
    """Every GEMM tiling of the policy, forced through the tuner table, gives bitwise the same matvec (a tile shape
    changes no summation order), and that matvec is within the policy's tolerance of the oracle.  The tuner keys of
    these shapes come from a short solve on the same problems."""
    cases = [_heff_case("chain", "ragged", 81), _heff_case("yc8", "wide", 82), _heff_case("chain", "big", 83)]
    probs = [c[0] for c in cases]
    c2 = lib.Context(0)
    psis = [T(c[1] / np.linalg.norm(c[1])) for c in cases]
    lib.lanczos_solve_batch(c2, probs, psis, k_max=12, prec=prec)
    table = [e for e in c2.tuning() if e["prec"] == {"f64": 0, "f32": 1, "bf16x3": 2}[prec]]
    assert {e["stage"] for e in table} == {0, 1}
    outs = []
    for tiling in TILINGS[prec]:
        c2.set_tuning([dict(e, tiling=tiling) for e in table])
        ys = [T(np.full(len(c[2]), np.nan)) for c in cases]
        lib.heff_apply(c2, probs, [T(c[1]) for c in cases], ys, prec)
        outs.append([H(y) for y in ys])
        print(f"[tiling] {prec} tiling {tiling}: max rel err "
              f"{max(rel_err(o, c[2]) for o, c in zip(outs[-1], cases)):.2e}")
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    for o, c in zip(outs[0], cases):
        assert rel_err(o, c[2]) <= (1e-13 if prec == "f64" else MIXED_TOL[prec])


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_heff_apply_mixed(ctx, prec):
    """Low-precision matvec policies against the FP64 oracle, relative to the output's magnitude."""
    cases = [_heff_case("chain", "ragged", 71), _heff_case("yc8", "wide", 72)]
    ys = [T(np.zeros(len(c[2]))) for c in cases]
    lib.heff_apply(ctx, [c[0] for c in cases], [T(c[1]) for c in cases], ys, prec)
    for (p, x, y), yg in zip(cases, ys):
        err = rel_err(H(yg), y)
        assert err <= MIXED_TOL[prec], err
        assert err >= 1e-9          # the policy really computed in low precision


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("fp32_basis", [True, False])
def test_lanczos_mixed_refined(ctx, prec, fp32_basis):
    """Mixed-precision Lanczos with FP64-anchored refinement: the energy is an FP64
    Rayleigh quotient with FP64 residual <= tol_res, so it matches the oracle to 1e-12,
    with the first pass's Krylov vectors stored in FP32 or in FP64."""
    cfg, r = _oracle_states("random_chain", 32, 7, tol_res=1e-10)
    sts = [st for st in r["states"] if st["n"] in (6, 7)]
    probs = [_flat_problem(st) for st in sts]
    psis = [T(st["v0"]) for st in sts]
    es, infos = lib.lanczos_solve_batch(ctx, probs, psis, cfg["tol_E"], cfg["tol_res"], cfg["k_max"], prec,
                                        fp32_basis=fp32_basis)
    print(f"[lanczos mixed] {prec} fp32_basis={fp32_basis}: iterations {[i['iters'] for i in infos]}, "
          f"FP64 matvecs {[i['fp64_matvecs'] for i in infos]}")
    steps = {(s["n"], s["i"]): s for s in r["steps"]}
    for st, e, inf, p in zip(sts, es, infos, psis):
        assert abs(e - steps[(st["n"], st["i"])]["energy"]) <= 1e-12
        assert abs(abs(float(H(p) @ st["psi"])) - 1.0) <= 1e-11
        assert inf["converged"] == 1 and inf["residual"] <= cfg["tol_res"]
        assert inf["fp64_matvecs"] >= 2


def test_trajectory_chain_mixed():
    """Uniform chain with the split-bf16 matvec and FP64 refinement: per-site energies
    within 1e-9 of the FP64 oracle."""
    cfg = workloads.workload("chain")
    g = _run_gpu(cfg, 20, prec="bf16x3")
    o = oidmrg.run(cfg, mode="u1", n_max=20)
    for a, b in zip(g.steps, o["steps"]):
        assert abs(a["e_site"] - b["e_site"]) <= 1e-9, (a, b)
