"""ctypes binding of libppl (include/ppl.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
arguments (ints, floats, torch tensors) into the C ABI's plain pointers and
sizes. torch is imported before the library is loaded so that the process
holds exactly one HIP runtime (the one torch ships), which libppl then shares.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime libppl binds to)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libppl.so")

PPL_OK = 0
PPL_E_ARG = -1
PPL_E_NOMEM = -2
PPL_E_HIP = -3
PPL_E_NONFINITE = -4
PPL_E_NOCONV = -5
PPL_E_DIVERGED = -6
PPL_E_STATE = -7
PPL_E_UNSUPPORTED = -8
ERROR_NAMES = {0: "PPL_OK", -1: "PPL_E_ARG", -2: "PPL_E_NOMEM", -3: "PPL_E_HIP", -4: "PPL_E_NONFINITE",
               -5: "PPL_E_NOCONV", -6: "PPL_E_DIVERGED", -7: "PPL_E_STATE", -8: "PPL_E_UNSUPPORTED"}

PPL_FP64, PPL_FP32, PPL_BF16X3, PPL_BF16X6 = 0, 1, 2, 3
PREC = {"fp64": PPL_FP64, "fp32": PPL_FP32, "bf16x3": PPL_BF16X3, "bf16x6": PPL_BF16X6}
PPL_START_MP2, PPL_START_GIVEN, PPL_START_GIVEN_CHECKED = 0, 1, 2


class ppl_desc_t(ctypes.Structure):
    _fields_ = [("o", ctypes.c_int32), ("v", ctypes.c_int32), ("naux", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("keep_fp64", ctypes.c_int32),
                ("tile_contract", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("build_scratch", ctypes.c_uint64), ("diis_max", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


class ppl_plan_info_t(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("vpm_bytes", ctypes.c_uint64),
                ("n_batches", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("a_per_batch", ctypes.c_int32), ("tile_build", ctypes.c_int32),
                ("tile_contract", ctypes.c_int32), ("n_plus", ctypes.c_int32),
                ("n_minus", ctypes.c_int32), ("p_plus", ctypes.c_int32), ("p_minus", ctypes.c_int32),
                ("splits_contract", ctypes.c_int32), ("tile_contract_minus", ctypes.c_int32),
                ("splits_contract_minus", ctypes.c_int32), ("build_scratch_bytes", ctypes.c_uint64),
                ("max_step_pairs", ctypes.c_int64), ("flops_build", ctypes.c_double),
                ("flops_contract", ctypes.c_double)]


class ppl_iter_opts_t(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("start", ctypes.c_int32), ("tol", ctypes.c_double),
                ("switch_tol", ctypes.c_double), ("stagnation", ctypes.c_double),
                ("min_fp64_sweeps", ctypes.c_int32), ("fail_on_noconv", ctypes.c_int32),
                ("diverge_factor", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("diis", ctypes.c_int32), ("hhl", ctypes.c_int32), ("ring", ctypes.c_int32)]


class ppl_iter_report_t(ctypes.Structure):
    _fields_ = [("sweeps_lp", ctypes.c_int32), ("sweeps_fp64", ctypes.c_int32),
                ("status", ctypes.c_int32), ("restarted_mp2", ctypes.c_int32),
                ("residual", ctypes.c_double), ("energy", ctypes.c_double),
                ("energy_start", ctypes.c_double), ("first_residual", ctypes.c_double),
                ("diis_dropped", ctypes.c_int32)]


PPL_PROF_KINDS = 6
PROF_KINDS = ["build_gemm", "build_pack", "contract_plus", "contract_minus", "update", "other"]


class ppl_profile_t(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * PPL_PROF_KINDS), ("ms", ctypes.c_double * PPL_PROF_KINDS),
                ("flops", ctypes.c_double * PPL_PROF_KINDS)]


# name -> (restype, argtypes) of every symbol include/ppl.h declares
_P = ctypes.c_void_p
SIGNATURES = {
    "ppl_plan": (ctypes.c_int, [ctypes.POINTER(ppl_desc_t), ctypes.POINTER(_P)]),
    "ppl_plan_query": (ctypes.c_int, [_P, ctypes.POINTER(ppl_plan_info_t)]),
    "ppl_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "ppl_build_batch": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "ppl_contract": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double]),
    "ppl_contract_tau": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_double, ctypes.c_double]),
    "ppl_hhl": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_double, ctypes.c_double]),
    "ppl_ring_scratch_bytes": (ctypes.c_uint64, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "ppl_ring": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_double,
                                ctypes.c_double, _P, ctypes.c_uint64, _P]),
    "ppl_ring_static": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_double,
                                       ctypes.c_double, _P]),
    "ppl_iter_opts_default": (None, [ctypes.POINTER(ppl_iter_opts_t)]),
    "ppl_iterate": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(ppl_iter_opts_t),
                                   ctypes.POINTER(ppl_iter_report_t)]),
    "ppl_mp2": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "ppl_mlp_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P, ctypes.POINTER(_P)]),
    "ppl_mlp_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "ppl_mlp_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "ppl_mlp_param_count": (ctypes.c_int, [_P]),
    "ppl_mlp_init": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "ppl_mlp_set_params": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "ppl_mlp_get_params": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "ppl_mlp_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_float)]),
    "ppl_mlp_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_float)]),
    "ppl_mlp_sigma": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "ppl_mlp_samples": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_double, _P, ctypes.c_int64, _P, _P]),
    "ppl_mlp_guess": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_double, _P]),
    "ppl_mlp_destroy": (ctypes.c_int, [_P]),
    "ppl_batch_plan": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ppl_desc_t), ctypes.POINTER(_P)]),
    "ppl_batch_query": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32)]),
    "ppl_batch_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "ppl_batch_build": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "ppl_batch_autotune": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ppl_batch_contract": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "ppl_batch_graph_capture": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "ppl_batch_graph_capture_build": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                                     ctypes.POINTER(_P)]),
    "ppl_batch_graph_launch": (ctypes.c_int, [_P]),
    "ppl_batch_destroy": (ctypes.c_int, [_P]),
    "ppl_set_contract_config": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32]),
    "ppl_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "ppl_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "ppl_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(ppl_profile_t)]),
    "ppl_destroy": (ctypes.c_int, [_P]),
    "ppl_last_error": (ctypes.c_char_p, []),
    "ppl_tile_count": (ctypes.c_int, []),
    "ppl_tile_dims": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "ppl_version": (ctypes.c_char_p, []),
}

_lib = None


class PPLError(RuntimeError):
    def __init__(self, code, where, detail):
        self.code = code
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)} ({detail})")


def load(path: str = LIB_PATH):
    """Load libppl.so and declare its prototypes. Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libppl.so not found at {path}: build it with "
                           "`python -m paper_2603_20912_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, where):
    if rc != PPL_OK:
        raise PPLError(rc, where, load().ppl_last_error().decode())
    return rc


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


# ---------------------------------------------------------------- argument validation
# The C ABI receives bare device addresses and cannot see dtypes, shapes or devices: a
# wrong tensor would be read or written out of bounds on the GPU. Every wrapper below
# therefore checks each tensor against the layout include/ppl.h documents and raises
# ValueError before anything reaches libppl.
_DIMS = {}      # handle value -> {"o", "v", "naux"} (plans), list of shapes (batches), max_batch (MLPs)


def _layout(x, name, dtype, shape=None, optional=False):
    """Check dtype, shape and contiguity of tensor x (None only when optional)."""
    if x is None:
        if optional:
            return
        raise ValueError(f"{name}: a device tensor is required")
    if not isinstance(x, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(x).__name__}")
    if x.dtype != dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {x.dtype}")
    if shape is not None and tuple(x.shape) != tuple(int(d) for d in shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: must be C-contiguous")


def _ptrs(*specs):
    """Device addresses of the tensors of specs (x, name, dtype, shape, optional): the
    layouts of all of them are checked first, then that each lives on the GPU."""
    for sp in specs:
        _layout(*sp)
    out = []
    for x, name, *_ in specs:
        if x is None:
            out.append(None)
            continue
        if x.device.type != "cuda":
            raise ValueError(f"{name}: must live on the GPU (got device {x.device})")
        out.append(x.data_ptr())
    return out


def _dims(handle, what="plan"):
    key = getattr(handle, "value", handle)
    d = _DIMS.get(key)
    if d is None:
        raise ValueError(f"unknown or destroyed {what} handle")
    return d


def _L(x, d, name="L"):
    n = d["o"] + d["v"]
    return (x, name, torch.float64, (d["naux"], n, n), False)


def _amp(x, d, name, optional=False):
    return (x, name, torch.float64, (d["o"], d["o"], d["v"], d["v"]), optional)


def _eo(x, d):
    return (x, "e_occ", torch.float64, (d["o"],), False)


def _ev(x, d):
    return (x, "e_vir", torch.float64, (d["v"],), False)


def _workspace(ws, nbytes):
    if not isinstance(ws, torch.Tensor):
        raise ValueError("workspace: expected a torch.Tensor")
    if not ws.is_contiguous() or ws.device.type != "cuda":
        raise ValueError("workspace: must be a contiguous GPU tensor")
    have = ws.numel() * ws.element_size()
    n = have if nbytes is None else int(nbytes)
    if n > have:
        raise ValueError(f"workspace: {n} bytes requested from a {have}-byte tensor")
    return ws.data_ptr(), n


def _stream_handle(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- same names as the C ABI
PPL_PLAN_CONTRACT_ONLY = 1
PPL_PLAN_RING = 2


def ppl_plan(o, v, naux, prec="fp64", keep_fp64=False, hbm_budget=0, stream=None, tile_contract=-1,
             build_scratch=0, diis_max=0, flags=0, tune_cache=None):
    d = ppl_desc_t(o, v, naux, PREC[prec] if isinstance(prec, str) else int(prec), int(bool(keep_fp64)),
                   int(tile_contract), int(hbm_budget),
                   _stream_handle(stream) if stream is not False else None, int(build_scratch), int(diis_max),
                   int(flags), os.fsencode(tune_cache) if tune_cache else None)
    h = ctypes.c_void_p()
    _check(load().ppl_plan(ctypes.byref(d), ctypes.byref(h)), "ppl_plan")
    _DIMS[h.value] = {"o": int(o), "v": int(v), "naux": int(naux)}
    return h


def ppl_plan_query(plan) -> dict:
    info = ppl_plan_info_t()
    _check(load().ppl_plan_query(plan, ctypes.byref(info)), "ppl_plan_query")
    return {f: getattr(info, f) for f, _ in ppl_plan_info_t._fields_}


def ppl_bind_workspace(plan, ws, nbytes=None):
    ptr, n = _workspace(ws, nbytes)
    _check(load().ppl_bind_workspace(plan, ptr, n), "ppl_bind_workspace")


def ppl_build_batch(plan, L, batch=-1):
    (pL,) = _ptrs(_L(L, _dims(plan)))
    _check(load().ppl_build_batch(plan, pL, int(batch)), "ppl_build_batch")


def ppl_contract(plan, t2, R, alpha=1.0, beta=0.0):
    d = _dims(plan)
    pt, pr = _ptrs(_amp(t2, d, "t2"), _amp(R, d, "R"))
    _check(load().ppl_contract(plan, pt, pr, float(alpha), float(beta)), "ppl_contract")


def ppl_contract_tau(plan, t2, t1, R, alpha=1.0, beta=0.0):
    d = _dims(plan)
    pt, p1, pr = _ptrs(_amp(t2, d, "t2"), (t1, "t1", torch.float64, (d["o"], d["v"]), False), _amp(R, d, "R"))
    _check(load().ppl_contract_tau(plan, pt, p1, pr, float(alpha), float(beta)), "ppl_contract_tau")


def ppl_ring_scratch_bytes(o, v, naux):
    return int(load().ppl_ring_scratch_bytes(int(o), int(v), int(naux)))


def ppl_ring(o, v, naux, L, t2, R, scratch, alpha=1.0, beta=0.0, stream=None):
    d = {"o": int(o), "v": int(v), "naux": int(naux)}
    pL, pt, pr = _ptrs(_L(L, d), _amp(t2, d, "t2"), _amp(R, d, "R"))
    sp, sn = _workspace(scratch, None)
    _check(load().ppl_ring(d["o"], d["v"], d["naux"], pL, pt, pr, float(alpha), float(beta), sp, sn,
                           _stream_handle(stream)), "ppl_ring")


PPL_RING_STATIC_BYTES = 128 << 20


def ppl_ring_static(o, v, naux, L, t2, R, alpha=1.0, beta=0.0, stream=None):
    d = {"o": int(o), "v": int(v), "naux": int(naux)}
    pL, pt, pr = _ptrs(_L(L, d), _amp(t2, d, "t2"), _amp(R, d, "R"))
    _check(load().ppl_ring_static(d["o"], d["v"], d["naux"], pL, pt, pr, float(alpha), float(beta),
                                  _stream_handle(stream)), "ppl_ring_static")


def ppl_hhl(plan, L, t2, R, alpha=1.0, beta=0.0):
    d = _dims(plan)
    pL, pt, pr = _ptrs(_L(L, d), _amp(t2, d, "t2"), _amp(R, d, "R"))
    _check(load().ppl_hhl(plan, pL, pt, pr, float(alpha), float(beta)), "ppl_hhl")


def ppl_iter_opts_default() -> ppl_iter_opts_t:
    o = ppl_iter_opts_t()
    load().ppl_iter_opts_default(ctypes.byref(o))
    return o


def ppl_iterate(plan, L, e_occ, e_vir, t2, opts: ppl_iter_opts_t | None = None, raise_on_status=True):
    rep = ppl_iter_report_t()
    d = _dims(plan)
    pL, po, pv, pt = _ptrs(_L(L, d), _eo(e_occ, d), _ev(e_vir, d), _amp(t2, d, "t2"))
    rc = load().ppl_iterate(plan, pL, po, pv, pt,
                            ctypes.byref(opts) if opts is not None else None, ctypes.byref(rep))
    if raise_on_status:
        _check(rc, "ppl_iterate")
    out = {f: getattr(rep, f) for f, _ in ppl_iter_report_t._fields_}
    out["rc"] = rc
    return out


def ppl_set_contract_config(plan, tile_plus, splits_plus, tile_minus, splits_minus):
    _check(load().ppl_set_contract_config(plan, int(tile_plus), int(splits_plus), int(tile_minus),
                                          int(splits_minus)), "ppl_set_contract_config")


def ppl_autotune(plan, reps=3):
    best = (ctypes.c_double * 2)()
    _check(load().ppl_autotune(plan, int(reps), best), "ppl_autotune")
    return float(best[0]), float(best[1])


def ppl_profile_enable(plan, on=True):
    _check(load().ppl_profile_enable(plan, int(bool(on))), "ppl_profile_enable")


def ppl_profile_read(plan) -> dict:
    pr = ppl_profile_t()
    _check(load().ppl_profile_read(plan, ctypes.byref(pr)), "ppl_profile_read")
    return {k: {"launches": int(pr.launches[i]), "ms": float(pr.ms[i]), "flops": float(pr.flops[i])}
            for i, k in enumerate(PROF_KINDS)}


def ppl_mp2(plan, L, e_occ, e_vir, t2_out, want_energy=True):
    e = ctypes.c_double(0.0)
    d = _dims(plan)
    pL, po, pv, pt = _ptrs(_L(L, d), _eo(e_occ, d), _ev(e_vir, d), _amp(t2_out, d, "t2_out"))
    _check(load().ppl_mp2(plan, pL, po, pv, pt,
                          ctypes.byref(e) if want_energy else None), "ppl_mp2")
    return e.value if want_energy else None


def ppl_mlp_create(width=128, max_batch=65536, stream=None):
    h = ctypes.c_void_p()
    _check(load().ppl_mlp_create(int(width), int(max_batch), _stream_handle(stream), ctypes.byref(h)),
           "ppl_mlp_create")
    _DIMS[h.value] = {"max_batch": int(max_batch)}
    return h


def ppl_mlp_workspace_bytes(mlp) -> int:
    b = ctypes.c_uint64(0)
    _check(load().ppl_mlp_workspace_bytes(mlp, ctypes.byref(b)), "ppl_mlp_workspace_bytes")
    return int(b.value)


def ppl_mlp_bind_workspace(mlp, ws, nbytes=None):
    ptr, n = _workspace(ws, nbytes)
    _check(load().ppl_mlp_bind_workspace(mlp, ptr, n), "ppl_mlp_bind_workspace")


def ppl_mlp_param_count(mlp) -> int:
    return int(load().ppl_mlp_param_count(mlp))


def ppl_mlp_init(mlp, seed=0):
    _check(load().ppl_mlp_init(mlp, int(seed)), "ppl_mlp_init")


def ppl_mlp_set_params(mlp, params):
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(load().ppl_mlp_set_params(mlp, a.ctypes.data, a.size), "ppl_mlp_set_params")


def ppl_mlp_get_params(mlp):
    import numpy as np
    a = np.empty(ppl_mlp_param_count(mlp), dtype=np.float32)
    _check(load().ppl_mlp_get_params(mlp, a.ctypes.data, a.size), "ppl_mlp_get_params")
    return a


def _xy(X, Y, n):
    n = Y.numel() if (n is None and isinstance(Y, torch.Tensor)) else int(n if n is not None else -1)
    if n < 0:
        raise ValueError("Y: a device tensor is required")
    px, py = _ptrs((X, "X", torch.float32, (n, 4), False), (Y, "Y", torch.float32, (n,), False))
    return px, py, n


def ppl_mlp_grad(mlp, X, Y, n=None):
    import numpy as np
    px, py, n = _xy(X, Y, n)
    g = np.empty(ppl_mlp_param_count(mlp), dtype=np.float32)
    loss = ctypes.c_float(0.0)
    _check(load().ppl_mlp_grad(mlp, px, py, n, g.ctypes.data, ctypes.byref(loss)), "ppl_mlp_grad")
    return g, float(loss.value)


def ppl_mlp_train_step(mlp, X, Y, lr, n=None, want_loss=False):
    px, py, n = _xy(X, Y, n)
    loss = ctypes.c_float(0.0)
    _check(load().ppl_mlp_train_step(mlp, px, py, n, float(lr),
                                     ctypes.byref(loss) if want_loss else None), "ppl_mlp_train_step")
    return float(loss.value) if want_loss else None


def ppl_mlp_sigma(plan, t_mp2) -> float:
    s = ctypes.c_double(0.0)
    (pt,) = _ptrs(_amp(t_mp2, _dims(plan), "t_mp2"))
    _check(load().ppl_mlp_sigma(plan, pt, ctypes.byref(s)), "ppl_mlp_sigma")
    return float(s.value)


def ppl_mlp_samples(plan, t_mp2, t_star, e_occ, e_vir, sigma, idx, X, Y=None):
    d = _dims(plan)
    if not isinstance(idx, torch.Tensor):
        raise ValueError("idx: expected a torch.Tensor")
    n = idx.numel()
    if (t_star is None) != (Y is None):
        raise ValueError("t_star and Y are given together or not at all")
    p = _ptrs(_amp(t_mp2, d, "t_mp2"), _amp(t_star, d, "t_star", optional=True), _eo(e_occ, d), _ev(e_vir, d),
              (idx, "idx", torch.int64, (n,), False), (X, "X", torch.float32, (n, 4), False),
              (Y, "Y", torch.float32, (n,), True))
    _check(load().ppl_mlp_samples(plan, p[0], p[1], p[2], p[3], float(sigma), p[4], n, p[5], p[6]),
           "ppl_mlp_samples")


def ppl_mlp_guess(mlp, plan, t_mp2, e_occ, e_vir, sigma, t2_out):
    d = _dims(plan)
    pt, po, pv, pg = _ptrs(_amp(t_mp2, d, "t_mp2"), _eo(e_occ, d), _ev(e_vir, d), _amp(t2_out, d, "t2_out"))
    _check(load().ppl_mlp_guess(mlp, plan, pt, po, pv, float(sigma), pg), "ppl_mlp_guess")


def ppl_mlp_destroy(mlp):
    if mlp is not None:
        _DIMS.pop(getattr(mlp, "value", mlp), None)
        load().ppl_mlp_destroy(mlp)


def _ptr_array(ts, shapes, kind):
    """Host array of the device addresses of one tensor per instance, each checked against
    its instance's layout (kind "L": [naux][n][n]; "amp": [o][o][v][v])."""
    ts = list(ts)
    if len(ts) != len(shapes):
        raise ValueError(f"expected {len(shapes)} tensors (one per instance), got {len(ts)}")
    specs = []
    for i, (t, (o, v, naux)) in enumerate(zip(ts, shapes)):
        d = {"o": o, "v": v, "naux": naux}
        specs.append(_L(t, d, f"L[{i}]") if kind == "L" else _amp(t, d, f"{kind}[{i}]"))
    arr = (ctypes.c_void_p * len(ts))()
    for i, p in enumerate(_ptrs(*specs)):
        arr[i] = p
    return arr


def ppl_batch_plan(shapes, prec="fp64", stream=None):
    n = len(shapes)
    descs = (ppl_desc_t * n)()
    sh = _stream_handle(stream)
    for k, (o, v, naux) in enumerate(shapes):
        descs[k] = ppl_desc_t(o, v, naux, PREC[prec], 0, -1, 0, sh, 0)
    h = ctypes.c_void_p()
    _check(load().ppl_batch_plan(n, descs, ctypes.byref(h)), "ppl_batch_plan")
    _DIMS[h.value] = [(int(o), int(v), int(naux)) for (o, v, naux) in shapes]
    return h


def ppl_batch_query(batch):
    b = ctypes.c_uint64(0)
    n = ctypes.c_int32(0)
    _check(load().ppl_batch_query(batch, ctypes.byref(b), ctypes.byref(n)), "ppl_batch_query")
    return int(b.value), int(n.value)


def ppl_batch_bind_workspace(batch, ws, nbytes=None):
    ptr, n = _workspace(ws, nbytes)
    _check(load().ppl_batch_bind_workspace(batch, ptr, n), "ppl_batch_bind_workspace")


def ppl_batch_build(batch, Ls):
    _check(load().ppl_batch_build(batch, _ptr_array(Ls, _dims(batch, "batch"), "L")), "ppl_batch_build")


def ppl_batch_autotune(batch, reps=2):
    _check(load().ppl_batch_autotune(batch, int(reps)), "ppl_batch_autotune")


def ppl_batch_contract(batch, t2s, Rs):
    sh = _dims(batch, "batch")
    _check(load().ppl_batch_contract(batch, _ptr_array(t2s, sh, "t2"), _ptr_array(Rs, sh, "R")),
           "ppl_batch_contract")


def ppl_batch_graph_capture(batch, t2s, Rs):
    sh = _dims(batch, "batch")
    _check(load().ppl_batch_graph_capture(batch, _ptr_array(t2s, sh, "t2"), _ptr_array(Rs, sh, "R")),
           "ppl_batch_graph_capture")


def ppl_batch_graph_capture_build(batch, Ls, t2s, Rs):
    sh = _dims(batch, "batch")
    _check(load().ppl_batch_graph_capture_build(batch, _ptr_array(Ls, sh, "L"), _ptr_array(t2s, sh, "t2"),
                                                _ptr_array(Rs, sh, "R")), "ppl_batch_graph_capture_build")


def ppl_batch_graph_launch(batch):
    _check(load().ppl_batch_graph_launch(batch), "ppl_batch_graph_launch")


def ppl_batch_destroy(batch):
    if batch is not None:
        _DIMS.pop(getattr(batch, "value", batch), None)
        load().ppl_batch_destroy(batch)


def ppl_destroy(plan):
    if plan is not None:
        _DIMS.pop(getattr(plan, "value", plan), None)
        load().ppl_destroy(plan)


def ppl_last_error() -> str:
    return load().ppl_last_error().decode()


def ppl_tile_count() -> int:
    return load().ppl_tile_count()


def ppl_tile_dims(tile: int):
    """(bm, bn, threads) of contraction tile `tile`."""
    bm, bn, th = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().ppl_tile_dims(int(tile), ctypes.byref(bm), ctypes.byref(bn), ctypes.byref(th)), "ppl_tile_dims")
    return bm.value, bn.value, th.value


def ppl_version() -> str:
    return load().ppl_version().decode()
