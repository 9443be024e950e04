"""Thin ctypes binding of libufss (argument marshalling only).

Every function forwards to the C ABI entry point of the same name declared in
``include/ufss.h``; all computation happens in the HIP library.  Device
buffers are torch tensors (complex64, contiguous, on the GPU): the binding
passes their ``data_ptr()`` and the current HIP stream.  If the library is
missing or fails to load, every call raises -- there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libufss.so")

UFSS_OK = 0
ERRORS = {
    -1: "INVALID_ARG", -2: "BAND_TOO_SMALL", -3: "HIP", -4: "OOM",
    -5: "UNSUPPORTED", -6: "DIVERGED",
}
F32, BF16 = 0, 1
ALGO_AUTO, ALGO_GEMM, ALGO_PHASOR, ALGO_FFT = 0, 1, 2, 3
SAMPLE_RND, SAMPLE_RND_F, SAMPLE_MAX, SAMPLE_NRG, SAMPLE_NRG_F = 0, 1, 2, 3, 4

EXPORTED = [
    "ufss_last_error", "ufss_select_freqs", "ufss_sample_bins", "ufss_sigma_estimate", "ufss_crb", "ufss_crb_mixed",
    "ufss_plan_create", "ufss_plan_create_mixed", "ufss_plan_destroy",
    "ufss_plan_info_get", "ufss_forward", "ufss_adjoint", "ufss_lipschitz", "ufss_fista",
    "ufss_fista_backtracking",
    "ufss_shrink_update", "ufss_shrink_update_noalloc", "ufss_absmax", "ufss_time_kernel", "ufss_fista_batched",
    "ufss_batch_create", "ufss_batch_run", "ufss_batch_set_lambdas", "ufss_batch_destroy",
    "ufss_synth_scene", "ufss_synth_measure",
    "ufss_autotune", "ufss_plan_set_tiling", "ufss_plan_kernel_timing", "ufss_plan_kernel_times", "ufss_plan_set_phasor_tables", "ufss_unrolled_create", "ufss_unrolled_destroy", "ufss_unrolled_params",
    "ufss_unrolled_forward", "ufss_unrolled_grad", "ufss_unrolled_train_step",
    "ufss_unrolled_save", "ufss_unrolled_load",
]


class UfssError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = ERRORS.get(code, "?")


class Geom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("z_start", ctypes.c_double), ("t0", ctypes.c_double), ("c", ctypes.c_double),
        ("fs", ctypes.c_double), ("fc", ctypes.c_double), ("frac_bw", ctypes.c_double),
        ("band_db", ctypes.c_double),
        ("win_x", ctypes.c_int32), ("win_y", ctypes.c_int32),
        ("dtype", ctypes.c_int32), ("algo", ctypes.c_int32),
        ("theta", ctypes.c_double),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("t0", ctypes.c_double), ("lipschitz", ctypes.c_double),
        ("band_lo", ctypes.c_int32), ("band_hi", ctypes.c_int32), ("band_size", ctypes.c_int32),
        ("win_x", ctypes.c_int32), ("win_y", ctypes.c_int32),
        ("m", ctypes.c_int32), ("per_position", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("algo", ctypes.c_int32), ("union_size", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64),
        ("fwd_split", ctypes.c_int32), ("adj_split", ctypes.c_int32),
        ("fwd_waves", ctypes.c_int32), ("fwd_zsplit", ctypes.c_int32),
        ("fwd_tile", ctypes.c_int32), ("adj_tile", ctypes.c_int32),
        ("fwd_rows", ctypes.c_int32), ("adj_rows", ctypes.c_int32),
        ("fwd_chunk", ctypes.c_int32), ("adj_chunk", ctypes.c_int32),
        ("phasor_tables", ctypes.c_int32), ("adj_waves", ctypes.c_int32),
    ]


class Tiling(ctypes.Structure):
    """GEMM tiling (ufss_tiling); 0 keeps the plan's current value."""
    _fields_ = [(f, ctypes.c_int32) for f in (
        "fwd_split", "adj_split", "fwd_waves", "fwd_zsplit", "fwd_tile", "adj_tile",
        "fwd_rows", "adj_rows", "fwd_chunk", "adj_chunk", "adj_waves")]


class FistaStats(ctypes.Structure):
    _fields_ = [
        ("obj", ctypes.POINTER(ctypes.c_double)), ("res", ctypes.POINTER(ctypes.c_double)),
        ("rel_change", ctypes.POINTER(ctypes.c_double)),
        ("err_ref", ctypes.POINTER(ctypes.c_double)),
        ("iters_done", ctypes.c_int32), ("lambda_", ctypes.c_double),
    ]


class FistaState(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_void_p), ("k_done", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libufss (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libufss.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        # torch ships its own HIP runtime: loaded first, it also serves this
        # library (one runtime per process); loaded second, it finds the GPU
        # already taken by the other runtime
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        sig = {
            "ufss_last_error": ([], ctypes.c_char_p),
            "ufss_select_freqs": ([ctypes.POINTER(Geom), I32, I32, U64, P, P], ctypes.c_int),
            "ufss_sample_bins": ([ctypes.POINTER(Geom), I32, I32, U64, P, P], ctypes.c_int),
            "ufss_sigma_estimate": ([ctypes.POINTER(Geom), I32, I32, P,
                                     ctypes.POINTER(SigmaEst)], ctypes.c_int),
            "ufss_crb": ([ctypes.POINTER(Geom), I32, I32, I32, P, ctypes.POINTER(CrbPoint), P, P,
                          P], ctypes.c_int),
            "ufss_crb_mixed": ([ctypes.POINTER(Geom), I32, I32, I32, P, I32, P,
                                ctypes.POINTER(CrbPoint), P, P, P], ctypes.c_int),
            "ufss_plan_create_mixed": ([ctypes.POINTER(Geom), I32, I32, P, I32, P, P], ctypes.c_int),
            "ufss_plan_create": ([ctypes.POINTER(Geom), I32, I32, P, ctypes.POINTER(P)], ctypes.c_int),
            "ufss_plan_destroy": ([P], ctypes.c_int),
            "ufss_plan_info_get": ([P, ctypes.POINTER(PlanInfo)], ctypes.c_int),
            "ufss_forward": ([P, P, P, P], ctypes.c_int),
            "ufss_adjoint": ([P, P, P, P], ctypes.c_int),
            "ufss_lipschitz": ([P, I32, D, D, U64, ctypes.POINTER(D), P], ctypes.c_int),
            "ufss_fista_backtracking": ([P, P, D, D, D, I32, D, P, P,
                                         ctypes.POINTER(FistaStats), P, P, P], ctypes.c_int),
            "ufss_fista": ([P, P, D, D, I32, D, I32, P, P, ctypes.POINTER(FistaStats),
                            ctypes.POINTER(FistaState), P], ctypes.c_int),
            "ufss_shrink_update": ([I64, P, P, P, D, D, D, P, P, P], ctypes.c_int),
            "ufss_shrink_update_noalloc": ([I64, P, P, P, D, D, D, P, P, P], ctypes.c_int),
            "ufss_absmax": ([I64, P, ctypes.POINTER(D), P], ctypes.c_int),
            "ufss_time_kernel": ([P, I32, I32, ctypes.POINTER(D), P], ctypes.c_int),
            "ufss_fista_batched": ([I32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                    ctypes.POINTER(D), ctypes.POINTER(D), I32, ctypes.POINTER(D), P],
                                   ctypes.c_int),
            "ufss_synth_scene": ([ctypes.POINTER(Geom), I32, D, D, I32, I32, U64, P, P], ctypes.c_int),
            "ufss_synth_measure": ([P, P, D, U64, P, P], ctypes.c_int),
            "ufss_batch_create": ([I32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                   ctypes.POINTER(D), ctypes.POINTER(D), I32, P, ctypes.POINTER(P)],
                                  ctypes.c_int),
            "ufss_batch_run": ([P, ctypes.POINTER(D), ctypes.POINTER(D), P], ctypes.c_int),
            "ufss_batch_set_lambdas": ([P, ctypes.POINTER(D), P], ctypes.c_int),
            "ufss_batch_destroy": ([P], ctypes.c_int),
            "ufss_autotune": ([P, ctypes.c_char_p, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), P],
                              ctypes.c_int),
            "ufss_plan_set_tiling": ([P, ctypes.POINTER(Tiling)], ctypes.c_int),
            "ufss_plan_kernel_timing": ([P, I32], ctypes.c_int),
            "ufss_plan_kernel_times": ([P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I32),
                                        ctypes.POINTER(I32)], ctypes.c_int),
            "ufss_plan_set_phasor_tables": ([P, I32, ctypes.POINTER(I32)], ctypes.c_int),
            "ufss_unrolled_create": ([P, I32, I32, D, D, U64, ctypes.POINTER(P)], ctypes.c_int),
            "ufss_unrolled_destroy": ([P], ctypes.c_int),
            "ufss_unrolled_params": ([P, P, P, ctypes.POINTER(I64)], ctypes.c_int),
            "ufss_unrolled_forward": ([P, P, P, P], ctypes.c_int),
            "ufss_unrolled_grad": ([P, P, P, I32, ctypes.POINTER(D), P, P], ctypes.c_int),
            "ufss_unrolled_train_step": ([P, I32, ctypes.POINTER(P), ctypes.POINTER(P), D,
                                          ctypes.POINTER(D), P], ctypes.c_int),
            "ufss_unrolled_save": ([P, ctypes.c_char_p], ctypes.c_int),
            "ufss_unrolled_load": ([P, ctypes.c_char_p], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code):
    if code != UFSS_OK:
        raise UfssError(code, lib().ufss_last_error().decode())


def make_geom(g, dtype=F32, algo=ALGO_AUTO):
    """ctypes geometry from a geometry dict (see workloads.geometry)."""
    return Geom(int(g["nx"]), int(g["ny"]), int(g["nz"]), int(g["nt"]), g["dx"], g["dy"], g["dz"],
                g["z_start"], g["t0"], g["c"], g["fs"], g["fc"], g["frac_bw"], g["band_db"],
                int(g["win_x"]), int(g["win_y"]), int(dtype), int(algo),
                float(g.get("theta", 0.0)))


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, dtype="complex64"):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch." + dtype:
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


def _numel_check(t, n, name):
    if t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))


def ufss_select_freqs(g, m, per_position, seed):
    """Seeded bins (int32 [m] or [ny, nx, m]) and the band size."""
    geom = make_geom(g)
    shape = (g["ny"], g["nx"], m) if per_position else (m,)
    out = np.zeros(shape, dtype=np.int32)
    band = ctypes.c_int32(0)
    _check(lib().ufss_select_freqs(ctypes.byref(geom), int(m), int(bool(per_position)),
                                   ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                   out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(band)))
    return out, band.value


def ufss_sample_bins(g, m, strategy, seed):
    """Bins of one sampling strategy (SAMPLE_*) and whether they are per position."""
    geom = make_geom(g)
    per = strategy in (SAMPLE_RND_F, SAMPLE_NRG_F)
    shape = (g["ny"], g["nx"], m) if per else (m,)
    out = np.zeros(shape, dtype=np.int32)
    flag = ctypes.c_int32(-1)
    _check(lib().ufss_sample_bins(ctypes.byref(geom), int(m), int(strategy),
                                  ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                  out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(flag)))
    assert flag.value == int(per)
    return out, per


class SigmaEst(ctypes.Structure):
    _fields_ = [("fro_sq", ctypes.c_double), ("fro_sq_central", ctypes.c_double),
                ("n", ctypes.c_int64), ("sigma_hat", ctypes.c_double),
                ("sigma_hat_central", ctypes.c_double)]


def ufss_sigma_estimate(g, m, per_position, bins):
    """Sec. IV-C Frobenius estimate of sigma_max (dict of the struct's fields)."""
    geom = make_geom(g)
    b = np.ascontiguousarray(bins, dtype=np.int32)
    want = g["nx"] * g["ny"] * m if per_position else m
    if b.size != want:
        raise ValueError("bins has %d entries, expected %d" % (b.size, want))
    out = SigmaEst()
    _check(lib().ufss_sigma_estimate(ctypes.byref(geom), int(m), int(bool(per_position)),
                                     b.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)))
    return {f: getattr(out, f) for f, _ in SigmaEst._fields_}


class CrbPoint(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                ("amp", ctypes.c_double), ("phase", ctypes.c_double), ("sigma2", ctypes.c_double)]


def ufss_crb(g, m, per_position, bins, point, stream=None, signs=None):
    """Cramer-Rao bounds for a stack of bin selections (with ``signs``: of
    randomly mixed measurements, ufss_crb_mixed; signs int8 [trials, nt] or
    [trials, ny, nx, nt], or without the trial axis for one selection).

    bins: int array [trials, m] (shared) or [trials, ny, nx, m]; a single
    selection without the leading axis is accepted.  point: dict with x, y, z,
    amp, phase, sigma2.  Returns (crb [trials, 3], fim [trials, 5, 5])."""
    b = np.ascontiguousarray(bins, dtype=np.int32)
    one = b.ndim == (3 if per_position else 1)
    if one:
        b = b[None]
    trials = b.shape[0]
    want = g["nx"] * g["ny"] * m if per_position else m
    if b[0].size != want:
        raise ValueError("each selection has %d entries, expected %d" % (b[0].size, want))
    geom = make_geom(g)
    pt = CrbPoint(*(float(point[k]) for k in ("x", "y", "z", "amp", "phase", "sigma2")))
    crb = np.zeros((trials, 3))
    fim = np.zeros((trials, 5, 5))
    if signs is None:
        _check(lib().ufss_crb(ctypes.byref(geom), int(m), int(bool(per_position)), int(trials),
                              b.ctypes.data_as(ctypes.c_void_p), ctypes.byref(pt),
                              fim.ctypes.data_as(ctypes.c_void_p),
                              crb.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    else:
        sg = np.ascontiguousarray(signs, dtype=np.int8)
        if one:
            sg = sg[None]
        per_s = sg.ndim == 4
        if sg.shape[0] != trials or sg[0].size != (g["nx"] * g["ny"] if per_s else 1) * g["nt"]:
            raise ValueError("signs must be [trials, nt] or [trials, ny, nx, nt]")
        _check(lib().ufss_crb_mixed(ctypes.byref(geom), int(m), int(bool(per_position)), int(trials),
                                    b.ctypes.data_as(ctypes.c_void_p), int(per_s),
                                    sg.ctypes.data_as(ctypes.c_void_p), ctypes.byref(pt),
                                    fim.ctypes.data_as(ctypes.c_void_p),
                                    crb.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return (crb[0], fim[0]) if one else (crb, fim)


class Plan:
    """Owning handle of a ufss plan (ufss_plan_create / ufss_plan_destroy).

    ``signs`` (int8 +-1, [nt] or [ny, nx, nt]) makes a randomly mixed plan
    (ufss_plan_create_mixed); its bins may then lie anywhere in [0, nt)."""

    def __init__(self, g, m, per_position, bins, dtype=F32, algo=ALGO_AUTO, signs=None):
        self.g = dict(g)
        self.m = int(m)
        self.per_position = bool(per_position)
        geom = make_geom(g, dtype, algo)
        b = np.ascontiguousarray(bins, dtype=np.int32)
        want = g["nx"] * g["ny"] * m if per_position else m
        if b.size != want:
            raise ValueError("bins has %d entries, expected %d" % (b.size, want))
        h = ctypes.c_void_p()
        if signs is None:
            _check(lib().ufss_plan_create(ctypes.byref(geom), self.m, int(self.per_position),
                                          b.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        else:
            sg = np.ascontiguousarray(signs, dtype=np.int8)
            per_s = sg.ndim == 3
            if sg.size != (g["nx"] * g["ny"] if per_s else 1) * g["nt"]:
                raise ValueError("signs must be [nt] or [ny, nx, nt]")
            _check(lib().ufss_plan_create_mixed(ctypes.byref(geom), self.m, int(self.per_position),
                                                b.ctypes.data_as(ctypes.c_void_p), int(per_s),
                                                sg.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.handle = h
        self.nvox = g["nx"] * g["ny"] * g["nz"]
        self.nmeas = g["nx"] * g["ny"] * m

    def info(self):
        i = PlanInfo()
        _check(lib().ufss_plan_info_get(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().ufss_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ufss_forward(plan, x, y, stream=None):
    _numel_check(x, plan.nvox, "x")
    _numel_check(y, plan.nmeas, "y")
    _check(lib().ufss_forward(plan.handle, _ptr(x, "x"), _ptr(y, "y"), _stream(stream)))


def ufss_adjoint(plan, y, x, stream=None):
    _numel_check(x, plan.nvox, "x")
    _numel_check(y, plan.nmeas, "y")
    _check(lib().ufss_adjoint(plan.handle, _ptr(y, "y"), _ptr(x, "x"), _stream(stream)))


def ufss_lipschitz(plan, max_iters=200, rtol=1e-6, margin=0.01, seed=4, stream=None):
    L = ctypes.c_double(0.0)
    _check(lib().ufss_lipschitz(plan.handle, int(max_iters), float(rtol), float(margin),
                                ctypes.c_uint64(seed), ctypes.byref(L), _stream(stream)))
    return L.value


def ufss_fista(plan, y, lam, L, iters, x, tol=0.0, accel=True, a_ref=None, state=None,
               stream=None, real=False):
    """Run FISTA/ISTA; returns a dict of per-iteration FP64 statistics.

    ``state`` may be a dict {"gamma": tensor, "k_done": int}; it is updated.
    """
    _numel_check(x, plan.nvox, "x")
    _numel_check(y, plan.nmeas, "y")
    n = max(int(iters), 1)
    arrs = {k: np.zeros(n) for k in ("obj", "res", "rel_change", "err_ref")}
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st = FistaStats(dp(arrs["obj"]), dp(arrs["res"]), dp(arrs["rel_change"]),
                    dp(arrs["err_ref"]), 0, 0.0)
    cst = None
    if state is not None:
        _numel_check(state["gamma"], plan.nvox, "state gamma")
        cst = FistaState(_ptr(state["gamma"], "gamma"), int(state.get("k_done", 0)))
    code = lib().ufss_fista(plan.handle, _ptr(y, "y"), float(lam), float(L), int(iters),
                            float(tol), int(bool(accel)) | (2 if real else 0), _ptr(x, "x"),
                            _ptr(a_ref, "a_ref") if a_ref is not None else None,
                            ctypes.byref(st), ctypes.byref(cst) if cst is not None else None,
                            _stream(stream))
    if cst is not None:
        state["k_done"] = cst.k_done
    _check(code)
    k = st.iters_done
    out = {key: v[:k].copy() for key, v in arrs.items()}
    out["iters_done"] = k
    out["lambda"] = st.lambda_
    return out


def ufss_fista_backtracking(plan, y, lam, L0, eta, iters, x, tol=0.0, a_ref=None,
                            stream=None):
    """FISTA with backtracking; per-iteration FP64 statistics plus the accepted
    constants ("L") and trial counts ("trials")."""
    _numel_check(x, plan.nvox, "x")
    _numel_check(y, plan.nmeas, "y")
    n = max(int(iters), 1)
    arrs = {k: np.zeros(n) for k in ("obj", "res", "rel_change", "err_ref", "L")}
    trials = np.zeros(n, dtype=np.int32)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st = FistaStats(dp(arrs["obj"]), dp(arrs["res"]), dp(arrs["rel_change"]),
                    dp(arrs["err_ref"]), 0, 0.0)
    _check(lib().ufss_fista_backtracking(
        plan.handle, _ptr(y, "y"), float(lam), float(L0), float(eta), int(iters), float(tol),
        _ptr(x, "x"), _ptr(a_ref, "a_ref") if a_ref is not None else None, ctypes.byref(st),
        arrs["L"].ctypes.data_as(ctypes.c_void_p), trials.ctypes.data_as(ctypes.c_void_p),
        _stream(stream)))
    k = st.iters_done
    out = {key: v[:k].copy() for key, v in arrs.items()}
    out["trials"] = trials[:k].copy()
    out["iters_done"] = k
    out["lambda"] = st.lambda_
    return out


def ufss_shrink_update(gamma, g, a, step, thresh, beta, a_ref=None, stream=None):
    """Fused update in place; returns the 5 FP64 norms (see ufss.h)."""
    n = a.numel()
    for t, nm in ((gamma, "gamma"), (g, "g")):
        _numel_check(t, n, nm)
    out = np.zeros(5)
    _check(lib().ufss_shrink_update(n, _ptr(gamma, "gamma"), _ptr(g, "g"), _ptr(a, "a"),
                                    float(step), float(thresh), float(beta),
                                    _ptr(a_ref, "a_ref") if a_ref is not None else None,
                                    out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return out


def ufss_shrink_update_noalloc(gamma, g, a, step, thresh, beta, a_ref=None, stream=None,
                               want_norms=True):
    """ufss_shrink_update without device allocation; returns the 5 FP64 norms
    (None when ``want_norms`` is False: then nothing synchronises)."""
    n = a.numel()
    for t, nm in ((gamma, "gamma"), (g, "g")):
        _numel_check(t, n, nm)
    out = np.zeros(5) if want_norms else None
    _check(lib().ufss_shrink_update_noalloc(
        n, _ptr(gamma, "gamma"), _ptr(g, "g"), _ptr(a, "a"), float(step), float(thresh),
        float(beta), _ptr(a_ref, "a_ref") if a_ref is not None else None,
        out.ctypes.data_as(ctypes.c_void_p) if out is not None else None, _stream(stream)))
    return out


def ufss_absmax(x, stream=None):
    out = ctypes.c_double(0.0)
    _check(lib().ufss_absmax(x.numel(), _ptr(x, "x"), ctypes.byref(out), _stream(stream)))
    return out.value


def ufss_time_kernel(plan, which, reps=10, stream=None):
    """Average duration (ms) of the forward (0) or adjoint (1) core kernel."""
    ms = ctypes.c_double(0.0)
    _check(lib().ufss_time_kernel(plan.handle, int(which), int(reps), ctypes.byref(ms),
                                  _stream(stream)))
    return ms.value


def ufss_fista_batched(plans, ys, xs, lambdas, Ls, iters, stream=None):
    """Batched FISTA (one grouped launch per phase, one hipGraph); returns the
    final residual norm of every scan."""
    n = len(plans)
    if not (len(ys) == len(xs) == len(lambdas) == len(Ls) == n):
        raise ValueError("plans, ys, xs, lambdas and Ls must have the same length")
    for p, y, x in zip(plans, ys, xs):
        _numel_check(x, p.nvox, "x")
        _numel_check(y, p.nmeas, "y")
    PA = ctypes.c_void_p * n
    hp = PA(*[p.handle.value for p in plans])
    yp = PA(*[_ptr(y, "y").value for y in ys])
    xp = PA(*[_ptr(x, "x").value for x in xs])
    lam = (ctypes.c_double * n)(*[float(v) for v in lambdas])
    Lc = (ctypes.c_double * n)(*[float(v) for v in Ls])
    res = (ctypes.c_double * n)()
    _check(lib().ufss_fista_batched(n, hp, yp, xp, lam, Lc, int(iters), res, _stream(stream)))
    return np.array(list(res))


def ufss_synth_scene(g, n_scat, amp, max_depth, back_wall, seed, x, stream=None):
    """Point-scatterer scene drawn on the device into x (see ufss.h)."""
    _numel_check(x, g["nx"] * g["ny"] * g["nz"], "x")
    geom = make_geom(g)
    _check(lib().ufss_synth_scene(ctypes.byref(geom), int(n_scat), float(amp[0]), float(amp[1]),
                                  int(max_depth), int(-1 if back_wall is None else back_wall),
                                  ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(x, "x"), _stream(stream)))


def ufss_synth_measure(plan, x, snr_db, seed, y, stream=None):
    """y = A x + complex Gaussian noise at snr_db, on the device (see ufss.h)."""
    _numel_check(x, plan.nvox, "x")
    _numel_check(y, plan.nmeas, "y")
    _check(lib().ufss_synth_measure(plan.handle, _ptr(x, "x"), float(snr_db),
                                    ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(y, "y"), _stream(stream)))


class Batch:
    """Owning handle of a persistent batch (ufss_batch_create / _run /
    _set_lambdas / _destroy): the iterations are captured once and replayed by
    every run.  Keeps references to the plans and buffers it was built on."""

    def __init__(self, plans, ys, xs, lambdas, Ls, iters, stream=None):
        n = len(plans)
        if not (len(ys) == len(xs) == len(lambdas) == len(Ls) == n):
            raise ValueError("plans, ys, xs, lambdas and Ls must have the same length")
        for p, y, x in zip(plans, ys, xs):
            _numel_check(x, p.nvox, "x")
            _numel_check(y, p.nmeas, "y")
        PA = ctypes.c_void_p * n
        hp = PA(*[p.handle.value for p in plans])
        yp = PA(*[_ptr(y, "y").value for y in ys])
        xp = PA(*[_ptr(x, "x").value for x in xs])
        lam = (ctypes.c_double * n)(*[float(v) for v in lambdas])
        Lc = (ctypes.c_double * n)(*[float(v) for v in Ls])
        h = ctypes.c_void_p()
        _check(lib().ufss_batch_create(n, hp, yp, xp, lam, Lc, int(iters), _stream(stream),
                                       ctypes.byref(h)))
        self.handle = h
        self.n = n
        self.iters = int(iters)
        self._keep = (list(plans), list(ys), list(xs))

    def run(self, stream=None):
        """Replay; returns (final residual norms, lambdas used) per scan."""
        res = (ctypes.c_double * self.n)()
        lam = (ctypes.c_double * self.n)()
        _check(lib().ufss_batch_run(self.handle, res, lam, _stream(stream)))
        return np.array(list(res)), np.array(list(lam))

    def set_lambdas(self, lambdas, stream=None):
        if len(lambdas) != self.n:
            raise ValueError("expected %d lambdas" % self.n)
        lam = (ctypes.c_double * self.n)(*[float(v) for v in lambdas])
        _check(lib().ufss_batch_set_lambdas(self.handle, lam, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().ufss_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ufss_autotune(plan, cache_path=None, use_cache=True, write_cache=True, stream=None, quick=False):
    """Pick the tiling of the plan's GEMMs by timing; returns the (fwd, adj) d_y splits."""
    fs = ctypes.c_int32(0)
    asp = ctypes.c_int32(0)
    flags = (1 if use_cache else 0) | (2 if write_cache else 0) | (4 if quick else 0)
    path = cache_path.encode() if cache_path else None
    _check(lib().ufss_autotune(plan.handle, path, flags, ctypes.byref(fs), ctypes.byref(asp),
                               _stream(stream)))
    return fs.value, asp.value


def ufss_plan_set_tiling(plan, *values, **fields):
    """Manual GEMM tiling: values in ufss_tiling's field order and/or by name;
    0 (or absent) keeps the plan's current value.  See ufss_autotune."""
    names = [f for f, _ in Tiling._fields_]
    if len(values) > len(names):
        raise TypeError("at most %d tiling values" % len(names))
    t = Tiling()
    for f, v in list(zip(names, values)) + list(fields.items()):
        if f not in names:
            raise TypeError("unknown tiling field " + f)
        setattr(t, f, int(v))
    _check(lib().ufss_plan_set_tiling(plan.handle, ctypes.byref(t)))


def ufss_plan_kernel_timing(plan, enable):
    """Start (clearing earlier records) or stop timing the core kernel launches."""
    _check(lib().ufss_plan_kernel_timing(plan.handle, 1 if enable else 0))


def ufss_plan_kernel_times(plan):
    """(forward ms, adjoint ms, forward launches, adjoint launches) averaged over
    the launches timed since timing was enabled."""
    f, a = ctypes.c_double(0), ctypes.c_double(0)
    nf, na = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().ufss_plan_kernel_times(plan.handle, ctypes.byref(f), ctypes.byref(a), ctypes.byref(nf),
                                        ctypes.byref(na)))
    return f.value, a.value, nf.value, na.value


def ufss_plan_set_phasor_tables(plan, enable):
    """BF16 GEMM plans: build (True) or free (False) the phasor tables; returns
    whether they are in use afterwards."""
    act = ctypes.c_int32(0)
    _check(lib().ufss_plan_set_phasor_tables(plan.handle, 1 if enable else 0, ctypes.byref(act)))
    return bool(act.value)


class Net:
    """Owning handle of a learned unrolled network (ufss_unrolled_*)."""

    def __init__(self, plan, stages=16, channels=8, L=1.0, mu=0.1, seed=7):
        h = ctypes.c_void_p()
        _check(lib().ufss_unrolled_create(plan.handle, int(stages), int(channels), float(L),
                                          float(mu), ctypes.c_uint64(seed), ctypes.byref(h)))
        self.handle = h
        self.plan = plan
        self.stages, self.channels = int(stages), int(channels)
        n = ctypes.c_int64(0)
        _check(lib().ufss_unrolled_params(h, None, None, ctypes.byref(n)))
        self.nparams = n.value

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().ufss_unrolled_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ufss_unrolled_params(net, set_to=None):
    """Current parameters (float32 numpy); optionally set them first."""
    out = np.zeros(net.nparams, dtype=np.float32)
    src = None
    if set_to is not None:
        src = np.ascontiguousarray(set_to, dtype=np.float32)
        if src.size != net.nparams:
            raise ValueError("expected %d parameters" % net.nparams)
    _check(lib().ufss_unrolled_params(net.handle, out.ctypes.data_as(ctypes.c_void_p),
                                      src.ctypes.data_as(ctypes.c_void_p) if src is not None else None,
                                      None))
    return out


def ufss_unrolled_forward(net, y, x, stream=None):
    _numel_check(x, net.plan.nvox, "x")
    _numel_check(y, net.plan.nmeas, "y")
    _check(lib().ufss_unrolled_forward(net.handle, _ptr(y, "y"), _ptr(x, "x"), _stream(stream)))


def ufss_unrolled_grad(net, y, target, accumulate=False, stream=None):
    """(loss, gradient as float32 numpy)."""
    _numel_check(target, net.plan.nvox, "target")
    _numel_check(y, net.plan.nmeas, "y")
    g = np.zeros(net.nparams, dtype=np.float32)
    loss = ctypes.c_double(0.0)
    _check(lib().ufss_unrolled_grad(net.handle, _ptr(y, "y"), _ptr(target, "target"),
                                    int(bool(accumulate)), ctypes.byref(loss),
                                    g.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return loss.value, g


def ufss_unrolled_train_step(net, ys, targets, lr, stream=None):
    n = len(ys)
    PA = ctypes.c_void_p * n
    yp = PA(*[_ptr(y, "y").value for y in ys])
    tp = PA(*[_ptr(t, "target").value for t in targets])
    loss = ctypes.c_double(0.0)
    _check(lib().ufss_unrolled_train_step(net.handle, n, yp, tp, float(lr), ctypes.byref(loss),
                                          _stream(stream)))
    return loss.value


def ufss_unrolled_save(net, path):
    _check(lib().ufss_unrolled_save(net.handle, str(path).encode()))


def ufss_unrolled_load(net, path):
    _check(lib().ufss_unrolled_load(net.handle, str(path).encode()))


def lambda_from_mu(mu):
    """ufss_fista's lambda argument asking for lambda = mu * max|A^H y|."""
    if not (mu > 0) or math.isnan(mu):
        raise ValueError("mu must be positive")
    return -float(mu)
