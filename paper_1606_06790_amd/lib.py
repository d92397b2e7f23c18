"""Thin ctypes binding of libidmrg.so (the C-ABI in include/idmrg.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device memory comes from PyTorch tensors (float64, on the GPU);
the calls enqueue on the current PyTorch stream of the tensors' device.

The library must be built (``python -m paper_1606_06790_amd.build`` or
``__graft_entry__.build()``); importing this module on a machine without it
raises an error instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libidmrg.so")

OK, WARN_NOCONV, EINVAL, ENOMEM, EHIP, ENUMERIC, EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
PREC = {"f64": 0, "f32": 1, "bf16x3": 2}
LEFT, RIGHT = 0, 1

OP_HEFF, OP_LANCZOS, OP_TRUNCATE, OP_ENV_LEFT, OP_ENV_RIGHT, OP_PREDICT, OP_TWOSITE_V, OP_OVERLAP = range(8)

EXPORTS = ["idmrg_create", "idmrg_destroy", "idmrg_set_stream", "idmrg_last_error", "idmrg_psi_size",
           "idmrg_envL_size", "idmrg_envR_size", "idmrg_U_size", "idmrg_V_size", "idmrg_heff_work",
           "heff_apply", "lanczos_solve_batch", "truncate_twosite", "update_env", "predict_wavefunction",
           "idmrg_profile", "idmrg_profile_get", "idmrg_workspace_size", "idmrg_set_workspace", "idmrg_get_stats",
           "heff_apply_static", "idmrg_tune_get", "idmrg_tune_set", "twosite_to_right_iso", "env_overlap"]
PROF_CLASSES = ["heff_gemm1", "heff_gemm2", "heff_mix", "convert", "lanczos_vec", "svd", "trunc_other", "env",
                "predict", "heff_gemm1_lo", "heff_gemm2_lo", "heff_mix_lo"]


class IdmrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"idmrg error {code}: {msg}")
        self.code = code


# ---------------------------------------------------------------- C structs

class Leg_t(C.Structure):
    _fields_ = [("nsec", C.c_int32), ("q", C.POINTER(C.c_int32)), ("dim", C.POINTER(C.c_int32))]


class Mpo_t(C.Structure):
    _fields_ = [("dl", C.c_int32), ("dr", C.c_int32), ("d", C.c_int32), ("w", C.POINTER(C.c_double)),
                ("ql", C.POINTER(C.c_int32)), ("qr", C.POINTER(C.c_int32)), ("qp", C.POINTER(C.c_int32))]


class Heff_t(C.Structure):
    _fields_ = [("left", Leg_t), ("right", Leg_t), ("w1", C.POINTER(Mpo_t)), ("w2", C.POINTER(Mpo_t)),
                ("L", C.c_void_p), ("R", C.c_void_p)]


class LanczosOpts_t(C.Structure):
    _fields_ = [("tol_E", C.c_double), ("tol_res", C.c_double), ("k_max", C.c_int32), ("prec", C.c_int32),
                ("chunk", C.c_int32), ("fp32_basis", C.c_int32), ("cgs2", C.c_int32), ("graph", C.c_int32)]


class LanczosInfo_t(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("fp64_matvecs", C.c_int32), ("flags", C.c_int32),
                ("reorth_passes", C.c_int32), ("reserved", C.c_int32), ("residual", C.c_double),
                ("overlap0", C.c_double)]


class Trunc_t(C.Structure):
    _fields_ = [("left", Leg_t), ("right", Leg_t), ("psi", C.c_void_p), ("cap_sec", C.c_int32),
                ("q_out", C.POINTER(C.c_int32)), ("dim_out", C.POINTER(C.c_int32)), ("U", C.c_void_p),
                ("V", C.c_void_p), ("lambda_", C.c_void_p), ("cap_U", C.c_int64), ("cap_V", C.c_int64),
                ("cap_lam", C.c_int64), ("nsec_out", C.c_int32), ("m_kept", C.c_int32), ("eps", C.c_double),
                ("eps_prime", C.c_double), ("cut_gap", C.c_double), ("svd_sweeps", C.c_int32),
                ("svd_converged", C.c_int32), ("null_completed", C.c_int32), ("reserved", C.c_int32)]


class EnvUpdate_t(C.Structure):
    _fields_ = [("old_leg", Leg_t), ("new_leg", Leg_t), ("w", C.POINTER(Mpo_t)), ("env_old", C.c_void_p),
                ("iso", C.c_void_p), ("env_new", C.c_void_p)]


class Predict_t(C.Structure):
    _fields_ = [("leg_a", Leg_t), ("leg_beta", Leg_t), ("leg_b", Leg_t), ("lam_i", C.c_void_p), ("V_i", C.c_void_p),
                ("lam_prev", C.c_void_p), ("U_ip1", C.c_void_p), ("lam_ip1", C.c_void_p), ("psi", C.c_void_p)]


class Twosite_t(C.Structure):
    _fields_ = [("left", Leg_t), ("right", Leg_t), ("psi", C.c_void_p), ("out", C.c_void_p)]


class Overlap_t(C.Structure):
    _fields_ = [("leg", Leg_t), ("nl", C.c_int32), ("ql", C.POINTER(C.c_int32)), ("L", C.c_void_p),
                ("nr", C.c_int32), ("qr", C.POINTER(C.c_int32)), ("R", C.c_void_p), ("wl", C.c_int32),
                ("wr", C.c_int32)]


class WsQuery_t(C.Structure):
    _fields_ = [("prec", C.c_int32), ("m_max", C.c_int32), ("d", C.c_int32), ("pad", C.c_int32),
                ("qp", C.POINTER(C.c_int32)), ("opts", C.POINTER(LanczosOpts_t))]


class TuneEntry_t(C.Structure):
    _fields_ = [("prec", C.c_int32), ("stage", C.c_int32), ("log2_flops", C.c_int32), ("log2_n", C.c_int32),
                ("log2_k", C.c_int32), ("tiling", C.c_int32), ("trial_ms", C.c_float * 8)]


class Stats_t(C.Structure):
    _fields_ = [("device_allocs", C.c_int64), ("stream_syncs", C.c_int64), ("staged_bytes", C.c_int64),
                ("plan_builds", C.c_int64)]


_lib = None


def load():
    """Load libidmrg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    lib.idmrg_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]
    lib.idmrg_destroy.argtypes = [C.c_void_p]
    lib.idmrg_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    lib.idmrg_last_error.argtypes = [C.c_void_p]
    lib.idmrg_last_error.restype = C.c_char_p
    lib.idmrg_psi_size.argtypes = [Leg_t, Leg_t, C.c_int32, C.POINTER(C.c_int32)]
    lib.idmrg_psi_size.restype = C.c_int64
    lib.idmrg_envL_size.argtypes = [Leg_t, C.c_int32, C.POINTER(C.c_int32)]
    lib.idmrg_envL_size.restype = C.c_int64
    lib.idmrg_envR_size.argtypes = [Leg_t, C.c_int32, C.POINTER(C.c_int32)]
    lib.idmrg_envR_size.restype = C.c_int64
    lib.idmrg_U_size.argtypes = [Leg_t, C.c_int32, C.POINTER(C.c_int32), Leg_t]
    lib.idmrg_U_size.restype = C.c_int64
    lib.idmrg_V_size.argtypes = [Leg_t, C.c_int32, C.POINTER(C.c_int32), Leg_t]
    lib.idmrg_V_size.restype = C.c_int64
    lib.idmrg_heff_work.argtypes = [C.POINTER(Heff_t), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.heff_apply.argtypes = [C.c_void_p, C.c_int, C.POINTER(Heff_t), C.POINTER(C.c_void_p),
                               C.POINTER(C.c_void_p), C.c_int]
    lib.heff_apply_static.argtypes = lib.heff_apply.argtypes
    lib.lanczos_solve_batch.argtypes = [C.c_void_p, C.c_int, C.POINTER(Heff_t), C.POINTER(C.c_void_p),
                                        C.POINTER(LanczosOpts_t), C.POINTER(C.c_double),
                                        C.POINTER(LanczosInfo_t)]
    lib.truncate_twosite.argtypes = [C.c_void_p, C.c_int, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                     C.c_double, C.c_double, C.POINTER(Trunc_t)]
    lib.update_env.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(EnvUpdate_t)]
    lib.predict_wavefunction.argtypes = [C.c_void_p, C.c_int, C.c_int32, C.POINTER(C.c_int32), C.c_double,
                                         C.POINTER(Predict_t)]
    lib.twosite_to_right_iso.argtypes = [C.c_void_p, C.c_int, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Twosite_t)]
    lib.env_overlap.argtypes = [C.c_void_p, C.c_int, C.POINTER(Overlap_t), C.POINTER(C.c_double)]
    lib.idmrg_workspace_size.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(WsQuery_t),
                                         C.POINTER(C.c_size_t)]
    lib.idmrg_set_workspace.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.idmrg_get_stats.argtypes = [C.c_void_p, C.POINTER(Stats_t)]
    lib.idmrg_tune_get.argtypes = [C.c_void_p, C.POINTER(TuneEntry_t), C.c_int, C.POINTER(C.c_int)]
    lib.idmrg_tune_set.argtypes = [C.c_void_p, C.POINTER(TuneEntry_t), C.c_int]
    lib.idmrg_profile.argtypes = [C.c_void_p, C.c_int]
    lib.idmrg_profile_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
    for name in ["idmrg_profile", "idmrg_profile_get", "idmrg_create", "idmrg_destroy", "idmrg_set_stream",
                 "idmrg_heff_work", "heff_apply", "idmrg_workspace_size", "idmrg_set_workspace", "idmrg_get_stats",
                 "heff_apply_static", "idmrg_tune_get", "idmrg_tune_set",
                 "lanczos_solve_batch", "truncate_twosite", "update_env", "predict_wavefunction"]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


# ---------------------------------------------------------------- marshalling helpers

class _Keep:
    """Holds ctypes arrays alive for the duration of one call."""

    def __init__(self):
        self.items = []

    def ints(self, seq):
        a = (C.c_int32 * max(1, len(seq)))(*[int(x) for x in seq])
        self.items.append(a)
        return a

    def doubles(self, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        self.items.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def leg(self, leg):
        q = [int(x) for x, _ in leg]
        d = [int(x) for _, x in leg]
        return Leg_t(len(q), self.ints(q), self.ints(d))

    def mpo(self, W):
        m = Mpo_t(W.dl, W.dr, W.d, self.doubles(W.w), self.ints(W.ql), self.ints(W.qr), self.ints(W.qp))
        self.items.append(m)
        return C.pointer(m)


class Mpo:
    """One MPO tensor W[w, w', s, s'] with channel and local charges."""

    def __init__(self, w, ql, qr, qp):
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.dl, self.dr, self.d, _ = self.w.shape
        self.ql, self.qr, self.qp = [int(x) for x in ql], [int(x) for x in qr], [int(x) for x in qp]


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != _torch().float64 or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous float64 CUDA tensors")
    return C.c_void_p(t.data_ptr())


def _torch():
    import torch
    return torch


def _check(ctx, rc):
    if rc < 0:
        raise IdmrgError(rc, load().idmrg_last_error(ctx.handle).decode())
    return rc


class Context:
    """Library context bound to a device and PyTorch's current stream on it.

    The device scratch of every call comes from one workspace that PyTorch
    allocates: each call is sized first (idmrg_workspace_size) and the
    workspace grows when a call needs more, so the library itself never
    allocates device memory.  workspace=False leaves the scratch to the library
    (its own block, grown with hipMalloc)."""

    def __init__(self, device=0, workspace=True):
        torch = _torch()
        self.device = device
        self.lib = load()
        self.managed = workspace
        self.ws, self.ws_bytes = None, 0
        h = C.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        rc = self.lib.idmrg_create(C.byref(h), device, C.c_void_p(stream))
        if rc != 0:
            raise IdmrgError(rc, "idmrg_create failed")
        self.handle = h

    def workspace_size(self, op, nprob, desc, query):
        """Bytes of device workspace the call needs (builds and keeps its plan)."""
        b = C.c_size_t()
        _check(self, self.lib.idmrg_workspace_size(self.handle, op, nprob, desc, C.byref(query), C.byref(b)))
        return int(b.value)

    def reserve(self, op, nprob, desc, query):
        """Size the call and grow the attached workspace if it needs more."""
        if not self.managed:
            return
        need = self.workspace_size(op, nprob, desc, query)
        if need <= self.ws_bytes:
            return
        torch = _torch()
        new = max(need, self.ws_bytes + self.ws_bytes // 4)
        new = (new + (1 << 20) - 1) >> 20 << 20
        if self.ws is not None:
            # work queued on the stream may still use the old block: PyTorch reuses freed memory only in
            # stream order, and empty_cache (a hipFree) waits for the device before releasing it
            self.ws = None
            self.ws_bytes = 0
            _check(self, self.lib.idmrg_set_workspace(self.handle, None, 0))
            torch.cuda.empty_cache()
        t = torch.empty(new, dtype=torch.uint8, device=torch.device("cuda", self.device))
        _check(self, self.lib.idmrg_set_workspace(self.handle, C.c_void_p(t.data_ptr()), new))
        self.ws, self.ws_bytes = t, new

    def tuning(self):
        """The autotuner's table: [{prec, stage, log2_flops, log2_n, log2_k, tiling, trial_ms}]."""
        n = C.c_int()
        _check(self, self.lib.idmrg_tune_get(self.handle, None, 0, C.byref(n)))
        arr = (TuneEntry_t * max(n.value, 1))()
        _check(self, self.lib.idmrg_tune_get(self.handle, arr, n.value, C.byref(n)))
        out = []
        for e in arr[:n.value]:
            d = {k: int(getattr(e, k)) for k, _ in TuneEntry_t._fields_ if k != "trial_ms"}
            d["trial_ms"] = [round(float(x), 4) for x in e.trial_ms]
            out.append(d)
        return out

    def set_tuning(self, entries):
        """Install autotuner entries (from tuning(), e.g. a JSON cache of an earlier run)."""
        arr = (TuneEntry_t * max(len(entries), 1))()
        for i, d in enumerate(entries):
            ms = list(d.get("trial_ms", [])) + [-1.0] * 8
            arr[i] = TuneEntry_t(d["prec"], d["stage"], d["log2_flops"], d["log2_n"], d["log2_k"], d["tiling"],
                                 (C.c_float * 8)(*ms[:8]))
        _check(self, self.lib.idmrg_tune_set(self.handle, arr, len(entries)))

    def _tuning_key(self):
        """What a stored tuner table is valid for: the device and this exact build of the library."""
        import hashlib
        with open(LIB_PATH, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()[:16]
        return dict(device=_torch().cuda.get_device_name(self.device), library=digest)

    def load_tuning(self, path):
        """Install the tuner table of a JSON cache written by save_tuning.  A cache written for another device or
        another build of the library is ignored (its timings would not hold).  Returns the number of entries."""
        if not os.path.exists(path):
            return 0
        with open(path) as f:
            doc = json.load(f)
        if doc.get("key") != self._tuning_key():
            return 0
        self.set_tuning(doc["entries"])
        return len(doc["entries"])

    def save_tuning(self, path):
        """Write the tuner table, with the device and library it was measured on, as JSON."""
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(dict(key=self._tuning_key(), entries=self.tuning()), f, indent=1)
        os.replace(tmp, path)

    def stats(self):
        st = Stats_t()
        _check(self, self.lib.idmrg_get_stats(self.handle, C.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in Stats_t._fields_}

    def sync_stream(self):
        torch = _torch()
        self.lib.idmrg_set_stream(self.handle, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def profile(self, enable=True):
        """Bracket every library launch with HIP events (clears the counters when enabling)."""
        _check(self, self.lib.idmrg_profile(self.handle, 1 if enable else 0))

    def profile_get(self):
        """{class: (launches, ms, flops)} of the launches since profiling was enabled."""
        out = {}
        for k, name in enumerate(PROF_CLASSES):
            n, ms, fl = C.c_int64(), C.c_double(), C.c_double()
            _check(self, self.lib.idmrg_profile_get(self.handle, k, C.byref(n), C.byref(ms), C.byref(fl)))
            out[name] = (int(n.value), float(ms.value), float(fl.value))
        return out

    def close(self):
        if self.handle:
            self.lib.idmrg_destroy(self.handle)
            self.handle = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- sizes

def psi_size(A, B, qp):
    k = _Keep()
    return int(load().idmrg_psi_size(k.leg(A), k.leg(B), len(qp), k.ints(qp)))


def envL_size(A, ql):
    k = _Keep()
    return int(load().idmrg_envL_size(k.leg(A), len(ql), k.ints(ql)))


def envR_size(B, qr):
    k = _Keep()
    return int(load().idmrg_envR_size(k.leg(B), len(qr), k.ints(qr)))


def U_size(A, qp, Cleg):
    k = _Keep()
    return int(load().idmrg_U_size(k.leg(A), len(qp), k.ints(qp), k.leg(Cleg)))


def V_size(B, qp, Cleg):
    k = _Keep()
    return int(load().idmrg_V_size(k.leg(B), len(qp), k.ints(qp), k.leg(Cleg)))


def _heff_structs(k, problems):
    arr = (Heff_t * len(problems))()
    for j, h in enumerate(problems):
        arr[j] = Heff_t(k.leg(h["left"]), k.leg(h["right"]), k.mpo(h["w1"]), k.mpo(h["w2"]), _ptr(h["L"]),
                        _ptr(h["R"]))
    k.items.append(arr)
    return arr


def heff_work(h):
    """(flops, bytes) of one heff_apply of problem h."""
    k = _Keep()
    arr = _heff_structs(k, [h])
    f, b = C.c_double(), C.c_double()
    rc = load().idmrg_heff_work(arr, C.byref(f), C.byref(b))
    if rc != 0:
        raise IdmrgError(rc, "idmrg_heff_work failed")
    return f.value, b.value


# ---------------------------------------------------------------- the five calls

def heff_apply(ctx, problems, xs, ys, prec="f64"):
    """ys[p] = H_p xs[p] (Sec. 2, Step 3)."""
    k = _Keep()
    arr = _heff_structs(k, problems)
    xp = (C.c_void_p * len(xs))(*[_ptr(x) for x in xs])
    yp = (C.c_void_p * len(ys))(*[_ptr(y) for y in ys])
    ctx.reserve(OP_HEFF, len(problems), arr, WsQuery_t(prec=PREC[prec]))
    _check(ctx, ctx.lib.heff_apply(ctx.handle, len(problems), arr, xp, yp, PREC[prec]))


def heff_apply_static(ctx, problems, xs, ys, prec="f64"):
    """ys[p] = H_p xs[p] with the library's static scratch (no allocation by the call)."""
    k = _Keep()
    arr = _heff_structs(k, problems)
    xp = (C.c_void_p * len(xs))(*[_ptr(x) for x in xs])
    yp = (C.c_void_p * len(ys))(*[_ptr(y) for y in ys])
    _check(ctx, ctx.lib.heff_apply_static(ctx.handle, len(problems), arr, xp, yp, PREC[prec]))


def lanczos_solve_batch(ctx, problems, psis, tol_E=1e-12, tol_res=1e-8, k_max=300, prec="f64", chunk=8,
                        fp32_basis=True, cgs2=False, graph=False):
    """Lowest eigenpairs; psis are overwritten with the ground states.  Returns (energies, infos).
    graph=True replays full chunks of iterations as captured HIP graphs (bitwise the same results).
    fp32_basis (mixed precision only): the first pass's Krylov vectors after its start vector stored in FP32."""
    k = _Keep()
    arr = _heff_structs(k, problems)
    P = len(problems)
    pp = (C.c_void_p * P)(*[_ptr(x) for x in psis])
    opts = LanczosOpts_t(tol_E, tol_res, k_max, PREC[prec], chunk, 1 if fp32_basis else 0, 1 if cgs2 else 0, 1 if graph else 0)
    e = (C.c_double * P)()
    inf = (LanczosInfo_t * P)()
    ctx.reserve(OP_LANCZOS, P, arr, WsQuery_t(opts=C.pointer(opts)))
    rc = _check(ctx, ctx.lib.lanczos_solve_batch(ctx.handle, P, arr, pp, C.byref(opts), e, inf))
    infos = [dict(iters=x.iters, converged=x.converged, fp64_matvecs=x.fp64_matvecs, flags=x.flags,
                  reorth_passes=x.reorth_passes, residual=x.residual, overlap0=x.overlap0, warn=rc) for x in inf]
    return [float(x) for x in e], infos


def truncate_twosite(ctx, items, qp, m_max, lam_floor=1e-14, deg_rel=1e-5):
    """items: list of dict(left, right, psi).  Returns list of dict(C, U, V, lam, eps, eps_prime,
    m_kept, cut_gap, svd_sweeps, svd_converged, warn) with U, V, lam as new float64 device tensors."""
    torch = _torch()
    k = _Keep()
    P = len(items)
    arr = (Trunc_t * P)()
    bufs = []
    d = len(qp)
    for j, it in enumerate(items):
        A, B = it["left"], it["right"]
        rows = sum(x for _, x in A) * d
        cols = sum(x for _, x in B) * d
        cap_sec = len(A) * d + len(B) * d + 2
        kmax = min(m_max, rows, cols)
        dev = it["psi"].device
        U = torch.empty(rows * kmax + 1, dtype=torch.float64, device=dev)
        V = torch.empty(cols * kmax + 1, dtype=torch.float64, device=dev)
        lam = torch.empty(kmax + 1, dtype=torch.float64, device=dev)
        qo = (C.c_int32 * cap_sec)()
        do = (C.c_int32 * cap_sec)()
        bufs.append((U, V, lam, qo, do))
        arr[j] = Trunc_t(k.leg(A), k.leg(B), _ptr(it["psi"]), cap_sec, qo, do, C.c_void_p(U.data_ptr()),
                         C.c_void_p(V.data_ptr()), C.c_void_p(lam.data_ptr()), U.numel(), V.numel(),
                         lam.numel(), 0, 0, 0.0, 0.0, 0.0, 0, 0)
    qpa = k.ints(qp)
    ctx.reserve(OP_TRUNCATE, P, arr, WsQuery_t(m_max=m_max, d=d, qp=qpa))
    rc = _check(ctx, ctx.lib.truncate_twosite(ctx.handle, P, d, qpa, m_max, lam_floor, deg_rel, arr))
    out = []
    for j, it in enumerate(items):
        U, V, lam, qo, do = bufs[j]
        t = arr[j]
        Cleg = [(int(qo[s]), int(do[s])) for s in range(t.nsec_out)]
        nU, nV = U_size(it["left"], qp, Cleg), V_size(it["right"], qp, Cleg)
        m = sum(x for _, x in Cleg)
        out.append(dict(C=Cleg, U=U[:nU].clone(), V=V[:nV].clone(), lam=lam[:m].clone(), eps=t.eps,
                        eps_prime=t.eps_prime, m_kept=t.m_kept, cut_gap=(None if t.cut_gap < 0 else t.cut_gap),
                        svd_sweeps=t.svd_sweeps, svd_converged=bool(t.svd_converged),
                        null_completed=bool(t.null_completed), warn=rc))
    return out


def update_env(ctx, side, items):
    """items: list of dict(old_leg, new_leg, w (Mpo), env_old, iso).  Returns new env tensors."""
    torch = _torch()
    k = _Keep()
    P = len(items)
    arr = (EnvUpdate_t * P)()
    outs = []
    for j, it in enumerate(items):
        W = it["w"]
        n = envL_size(it["new_leg"], W.qr) if side == LEFT else envR_size(it["new_leg"], W.ql)
        o = torch.empty(max(n, 1), dtype=torch.float64, device=it["env_old"].device)
        outs.append(o[:n])
        arr[j] = EnvUpdate_t(k.leg(it["old_leg"]), k.leg(it["new_leg"]), k.mpo(W), _ptr(it["env_old"]),
                             _ptr(it["iso"]), C.c_void_p(o.data_ptr()))
    ctx.reserve(OP_ENV_LEFT if side == LEFT else OP_ENV_RIGHT, P, arr, WsQuery_t())
    _check(ctx, ctx.lib.update_env(ctx.handle, P, side, arr))
    return outs


def predict_wavefunction(ctx, items, qp, lam_floor=1e-14):
    """items: list of dict(leg_a, leg_beta, leg_b, lam_i, V_i, lam_prev, U_ip1, lam_ip1).  Returns psi tensors."""
    torch = _torch()
    k = _Keep()
    P = len(items)
    arr = (Predict_t * P)()
    outs = []
    for j, it in enumerate(items):
        n = psi_size(it["leg_a"], it["leg_b"], qp)
        o = torch.empty(n, dtype=torch.float64, device=it["V_i"].device)
        outs.append(o)
        arr[j] = Predict_t(k.leg(it["leg_a"]), k.leg(it["leg_beta"]), k.leg(it["leg_b"]), _ptr(it["lam_i"]),
                           _ptr(it["V_i"]), _ptr(it["lam_prev"]), _ptr(it["U_ip1"]), _ptr(it["lam_ip1"]),
                           C.c_void_p(o.data_ptr()))
    qpa = k.ints(qp)
    ctx.reserve(OP_PREDICT, P, arr, WsQuery_t(d=len(qp), qp=qpa))
    _check(ctx, ctx.lib.predict_wavefunction(ctx.handle, P, len(qp), qpa, lam_floor, arr))
    return outs


def fused_qp(qp):
    """Charges of the fused site of two sites: s = s1 d + s2 has qp[s1] + qp[s2]."""
    return [a + b for a in qp for b in qp]


def twosite_to_right_iso(ctx, items, qp):
    """items: list of dict(left, right, psi).  Returns each psi as the fused site's right isometry (V layout,
    new leg = left)."""
    torch = _torch()
    k = _Keep()
    P = len(items)
    arr = (Twosite_t * P)()
    outs = []
    for j, it in enumerate(items):
        o = torch.empty(V_size(it["right"], fused_qp(qp), it["left"]), dtype=torch.float64, device=it["psi"].device)
        outs.append(o)
        arr[j] = Twosite_t(k.leg(it["left"]), k.leg(it["right"]), _ptr(it["psi"]), C.c_void_p(o.data_ptr()))
    qpa = k.ints(qp)
    ctx.reserve(OP_TWOSITE_V, P, arr, WsQuery_t(d=len(qp), qp=qpa))
    _check(ctx, ctx.lib.twosite_to_right_iso(ctx.handle, P, len(qp), qpa, arr))
    return outs


def env_overlap(ctx, items):
    """items: list of dict(leg, ql, L, qr, R, wl, wr).  Returns [sum_{a,a'} L[a,wl,a'] R[a,wr,a']] as floats."""
    k = _Keep()
    P = len(items)
    arr = (Overlap_t * P)()
    for j, it in enumerate(items):
        arr[j] = Overlap_t(k.leg(it["leg"]), len(it["ql"]), k.ints(it["ql"]), _ptr(it["L"]), len(it["qr"]),
                           k.ints(it["qr"]), _ptr(it["R"]), it["wl"], it["wr"])
    out = (C.c_double * P)()
    ctx.reserve(OP_OVERLAP, P, arr, WsQuery_t())
    _check(ctx, ctx.lib.env_overlap(ctx.handle, P, arr, out))
    return [float(x) for x in out]
