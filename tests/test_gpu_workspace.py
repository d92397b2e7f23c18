"""The workspace contract of the C-ABI and its error paths (needs an MI355X).

* With a workspace attached (the binding's default: each call is sized with
  idmrg_workspace_size and one PyTorch-allocated buffer grows to fit), no call
  allocates device memory, and a size query followed by its call builds the
  plan once.
* heff_apply, update_env and predict_wavefunction are asynchronous: issued
  behind ~0.2 s of matrix products on the same stream they return at once, with no
  stream synchronisation by the library, and their results are right once the
  stream has run.
* A workspace smaller than the call needs gives IDMRG_ENOMEM and launches
  nothing; a NaN in the inputs gives IDMRG_ENUMERIC from the calls that return
  host scalars.  (Every loop of the kernels is bounded, so NaN data only makes
  them run to their caps.)
* The library-owned scratch mode gives bitwise the same results.
"""
import time

import numpy as np
import pytest

import workloads
from oracle import layout, u1

from gpu_common import QP, H, T, mpo_pair, rel_err

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_1606_06790_amd.lib")
torch = pytest.importorskip("torch")

A = [(-3, 20), (-1, 70), (1, 65), (3, 15)]
B = [(-3, 12), (-1, 67), (1, 80), (3, 30)]
Cl = [(-4, 17), (-2, 60), (0, 90), (2, 55), (4, 21)]


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    (W1, W2, dl, dm, dr), (M1, M2) = mpo_pair("yc8", 3)
    Lf = workloads.gaussian(layout.envL_size(A, dl), 90, 1)
    Rf = workloads.gaussian(layout.envR_size(B, dr), 90, 2)
    x = workloads.gaussian(layout.psi_size(A, B, QP), 90, 3)
    y = layout.psi_to_flat(u1.heff_apply(layout.flat_to_envL(Lf, A, dl), W1, W2, layout.flat_to_envR(Rf, B, dr),
                                         layout.flat_to_psi(x, A, B, QP), A, B, QP, dl, dr), A, B, QP)
    n_iso = sum(sum(r[2] for r in layout.U_rows(A, QP, q)) * k for q, k in Cl)
    Uf = workloads.gaussian(n_iso, 90, 4)
    env_ref = layout.envL_to_flat(u1.update_env_left(layout.flat_to_envL(Lf, A, dl), W1,
                                                     layout.flat_to_U(Uf, A, QP, Cl), A, QP, Cl, dl, dm), Cl, dm)
    prob = dict(left=A, right=B, w1=M1, w2=M2, L=T(Lf), R=T(Rf))
    return dict(prob=prob, x=x, y=y, Uf=Uf, env_ref=env_ref, M1=M1, Lf=Lf)


def _env_item(case):
    return dict(old_leg=A, new_leg=Cl, w=case["M1"], env_old=case["prob"]["L"], iso=T(case["Uf"]))


def test_no_device_allocation_with_workspace(case):
    ctx = lib.Context(0)
    yg = T(np.zeros(len(case["y"])))
    lib.heff_apply(ctx, [case["prob"]], [T(case["x"])], [yg], "f64")
    lib.heff_apply(ctx, [case["prob"]], [T(case["x"])], [yg], "bf16x3")
    lib.update_env(ctx, lib.LEFT, [_env_item(case)])
    psi = T(case["x"] / np.linalg.norm(case["x"]))
    lib.lanczos_solve_batch(ctx, [case["prob"]], [psi], k_max=30, prec="bf16x3")
    lib.truncate_twosite(ctx, [dict(left=A, right=B, psi=psi)], QP, 64)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["device_allocs"] == 0, st
    assert ctx.ws_bytes > 0
    # a size query followed by the call of the same shapes builds the plan once
    before = ctx.stats()["plan_builds"]
    lib.update_env(ctx, lib.RIGHT, [dict(old_leg=B, new_leg=Cl, w=mpo_pair("yc8", 3)[1][1], env_old=case["prob"]["R"],
                                         iso=T(workloads.gaussian(sum(sum(r[2] for r in layout.V_rows(B, QP, q)) * k
                                                                          for q, k in Cl), 90, 5)))])
    assert ctx.stats()["plan_builds"] == before + 1


def test_calls_are_asynchronous(case):
    ctx = lib.Context(0)
    x = T(case["x"])
    ys = [T(np.zeros(len(case["y"]))) for _ in range(3)]
    env = _env_item(case)
    lib.heff_apply(ctx, [case["prob"]], [x], [ys[0]], "f64")     # plans and workspace in place
    lib.update_env(ctx, lib.LEFT, [env])
    busy = torch.randn(8192, 8192, device="cuda")
    torch.cuda.synchronize()
    s0 = ctx.stats()
    for _ in range(30):                                           # ~0.1-0.3 s of work queued on the stream
        busy = busy @ busy * 1e-4
    t0 = time.perf_counter()
    for y in ys:
        lib.heff_apply(ctx, [case["prob"]], [x], [y], "f64")
    out = lib.update_env(ctx, lib.LEFT, [env])[0]
    t_host = time.perf_counter() - t0
    s1 = ctx.stats()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    print(f"[workspace] host time of 4 queued calls {t_host * 1e3:.2f} ms, stream done after {t_all * 1e3:.1f} ms")
    assert s1["stream_syncs"] == s0["stream_syncs"] and s1["device_allocs"] == s0["device_allocs"]
    assert t_all > 0.02 and t_host < 0.25 * t_all
    for y in ys:
        assert rel_err(H(y), case["y"]) <= 1e-13
    assert rel_err(H(out), case["env_ref"]) <= 1e-13


def test_workspace_too_small_is_enomem(case):
    ctx = lib.Context(0, workspace=False)
    small = torch.empty(4096, dtype=torch.uint8, device="cuda")
    assert ctx.lib.idmrg_set_workspace(ctx.handle, lib.C.c_void_p(small.data_ptr()), 4096) == lib.OK
    y = T(np.full(len(case["y"]), 7.0))
    with pytest.raises(lib.IdmrgError) as e:
        lib.heff_apply(ctx, [case["prob"]], [T(case["x"])], [y], "f64")
    assert e.value.code == lib.ENOMEM and "workspace" in str(e.value)
    torch.cuda.synchronize()
    assert np.all(H(y) == 7.0)                                  # nothing was launched
    assert ctx.stats()["device_allocs"] == 0
    # detached again, the library allocates its own scratch and the call succeeds
    assert ctx.lib.idmrg_set_workspace(ctx.handle, None, 0) == lib.OK
    lib.heff_apply(ctx, [case["prob"]], [T(case["x"])], [y], "f64")
    assert ctx.stats()["device_allocs"] >= 1
    assert rel_err(H(y), case["y"]) <= 1e-13


def test_library_scratch_gives_the_same_results(case):
    out = []
    for managed in (True, False):
        ctx = lib.Context(0, workspace=managed)
        psi = T(case["x"] / np.linalg.norm(case["x"]))
        es, _ = lib.lanczos_solve_batch(ctx, [case["prob"]], [psi], k_max=40, prec="f64")
        out.append((es[0], H(psi)))
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])


def test_nan_input_is_enumeric(case):
    ctx = lib.Context(0)
    Lbad = case["Lf"].copy()
    Lbad[len(Lbad) // 2] = np.nan
    prob = dict(case["prob"], L=T(Lbad))
    psi = T(case["x"])
    with pytest.raises(lib.IdmrgError) as e:
        lib.lanczos_solve_batch(ctx, [prob], [psi], k_max=4, prec="f64")
    assert e.value.code == lib.ENUMERIC
    xb = case["x"] / np.linalg.norm(case["x"])
    xb[3] = np.nan
    with pytest.raises(lib.IdmrgError) as e:
        lib.truncate_twosite(ctx, [dict(left=A, right=B, psi=T(xb))], QP, 64)
    assert e.value.code == lib.ENUMERIC


def test_tuning_cache_round_trip(case, tmp_path):
    """A tuner table saved as JSON and loaded into a fresh context gives the same tile choices and bitwise the same
    solve; a table stored for another build of the library is ignored."""
    path = str(tmp_path / "tune.json")
    out = []
    for k in range(2):
        ctx = lib.Context(0)
        if k == 1:
            assert ctx.load_tuning(path) > 0
            loaded = {(e["prec"], e["stage"], e["log2_flops"], e["log2_n"], e["log2_k"]): e["tiling"]
                      for e in ctx.tuning()}
        psi = T(case["x"] / np.linalg.norm(case["x"]))
        es, _ = lib.lanczos_solve_batch(ctx, [case["prob"]], [psi], k_max=40, prec="bf16x3")
        out.append((es[0], H(psi)))
        if k == 0:
            ctx.save_tuning(path)
            saved = {(e["prec"], e["stage"], e["log2_flops"], e["log2_n"], e["log2_k"]): e["tiling"]
                     for e in ctx.tuning()}
    assert saved and loaded == saved
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])
    import json
    with open(path) as f:
        doc = json.load(f)
    doc["key"]["library"] = "0" * 16
    with open(path, "w") as f:
        json.dump(doc, f)
    assert lib.Context(0).load_tuning(path) == 0
